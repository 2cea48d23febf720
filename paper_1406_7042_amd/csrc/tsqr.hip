// Tall-skinny FP64 kernels of the block orthogonalisation (real and complex):
//   gram    C (m x nb) = A^H B    over n >> m rows (split over row chunks,
//                                  register tiles, wave64 shuffle reductions)
//   update  X -= Q C               (every row of Q read once)
//   trsm    X = X R^-1              (R upper triangular nb x nb, per row)
// Block-to-work mapping of gram is XCD-aware: the 8 XCDs of the device take
// consecutive block ids round-robin, so the blocks that share a row chunk (and
// thus the rows of B) are given ids that land on the same XCD and its L2.
#include <vector>

#include "cplx.hpp"
#include "tsqr.hpp"

namespace yr {

namespace {
constexpr int kThreads = 256;
constexpr int kRowsPerThread = 32;
constexpr int kChunk = kThreads * kRowsPerThread;  // rows per block
constexpr int kXcd = 8;

template <typename S>
struct Ops;
template <>
struct Ops<double> {
  static __device__ double cmul(double a, double b) { return a * b; }  // conj(a) b
  static constexpr int W = 1;
  static __device__ void put(double* d, double v) { d[0] = v; }
  static __device__ double get(const double* d) { return d[0]; }
};
template <>
struct Ops<zd> {
  static __device__ zd cmul(zd a, zd b) { return conj(a) * b; }
  static constexpr int W = 2;
  static __device__ void put(double* d, zd v) {
    d[0] = v.re;
    d[1] = v.im;
  }
  static __device__ zd get(const double* d) { return zd(d[0], d[1]); }
};

__device__ inline double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
}  // namespace

// partial[chunk][tile][JT][NB] (doubles, x2 for complex)
template <typename S, int JT, int NB>
__global__ void __launch_bounds__(kThreads)
    k_gram_partial(const S* __restrict__ A, int64_t lda, int m, const S* __restrict__ B,
                   int64_t ldb, int nb, int64_t n, int ntiles, int nchunks,
                   double* __restrict__ partial) {
  constexpr int W = Ops<S>::W;
  __shared__ double lds[JT * NB * W * (kThreads / 64)];
  // XCD-aware decode of blockIdx.x -> (tile, chunk)
  const int b = blockIdx.x;
  const int xcd = b % kXcd, idx = b / kXcd;
  const int tile = idx % ntiles;
  const int chunk = (idx / ntiles) * kXcd + xcd;
  S acc[JT][NB];
#pragma unroll
  for (int t = 0; t < JT; ++t)
#pragma unroll
    for (int c = 0; c < NB; ++c) acc[t][c] = S(0);
  const int j0 = tile * JT;
  if (chunk < nchunks) {
    const int64_t r0 = (int64_t)chunk * kChunk;
    // columns past m (of A) or nb (of B) read the last valid column instead
    // of branching, so all loads of a row issue together; their sums land in
    // slots the reduction never stores
    const S* ac[JT];
    const S* bc[NB];
#pragma unroll
    for (int t = 0; t < JT; ++t) ac[t] = A + (int64_t)(j0 + t < m ? j0 + t : m - 1) * lda;
#pragma unroll
    for (int c = 0; c < NB; ++c) bc[c] = B + (int64_t)(c < nb ? c : nb - 1) * ldb;
    for (int rr = 0; rr < kRowsPerThread; ++rr) {
      const int64_t row = r0 + rr * kThreads + threadIdx.x;
      if (row >= n) break;
      S bv[NB], av[JT];
#pragma unroll
      for (int c = 0; c < NB; ++c) bv[c] = bc[c][row];
#pragma unroll
      for (int t = 0; t < JT; ++t) av[t] = ac[t][row];
#pragma unroll
      for (int t = 0; t < JT; ++t)
#pragma unroll
        for (int c = 0; c < NB; ++c) acc[t][c] = acc[t][c] + Ops<S>::cmul(av[t], bv[c]);
    }
  }
  // block reduction
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  constexpr int NV = JT * NB * W;
  double v[NV];
#pragma unroll
  for (int t = 0; t < JT; ++t)
#pragma unroll
    for (int c = 0; c < NB; ++c) Ops<S>::put(&v[(t * NB + c) * W], acc[t][c]);
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double s = wsum(v[q]);
    if (lane == 0) lds[q * (kThreads / 64) + wid] = s;
  }
  __syncthreads();
  if (chunk >= nchunks) return;
  double* out = partial + ((int64_t)chunk * ntiles + tile) * NV;
  for (int q = threadIdx.x; q < NV; q += blockDim.x) {
    double s = 0;
    for (int w = 0; w < kThreads / 64; ++w) s += lds[q * (kThreads / 64) + w];
    out[q] = s;
  }
}

// C[j + c*ldc] = sum over chunks: one block per tile; lane = value of the
// tile (JT NB W = 64 values, one coalesced 512-byte row of `partial` per
// chunk), waves over chunks, fixed summation order (deterministic)
template <typename S, int JT, int NB>
__global__ void __launch_bounds__(1024)
    k_gram_reduce(const double* __restrict__ partial, int ntiles, int nchunks, int m, int nb,
                  S* __restrict__ C, int ldc) {
  constexpr int W = Ops<S>::W;
  constexpr int NV = JT * NB * W;
  static_assert(NV == 64, "one wave per chunk row");
  __shared__ double lds[16][NV];
  const int tile = blockIdx.x;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  double acc = 0;
#pragma unroll 8
  for (int ch = wid; ch < nchunks; ch += nw)
    acc += partial[((int64_t)ch * ntiles + tile) * NV + lane];
  lds[wid][lane] = acc;
  __syncthreads();
  if (wid != 0) return;
  double sum = 0;
  for (int w = 0; w < nw; ++w) sum += lds[w][lane];
  const int tc = lane / W, part = lane % W;
  const int t = tc / NB, c = tc % NB;
  const int j = tile * JT + t;
  if (j < m && c < nb) reinterpret_cast<double*>(&C[j + (int64_t)c * ldc])[part] = sum;
}

// X[:, c] -= sum_j Q[:, j] C[j, c]   (C in LDS)
template <typename S, int NB>
__global__ void __launch_bounds__(kThreads)
    k_update(const S* __restrict__ Q, int64_t ldq, int m, const S* __restrict__ C, int ldc,
             S* __restrict__ X, int64_t ldx, int nb, int64_t n) {
  extern __shared__ unsigned char smem[];
  S* Cs = reinterpret_cast<S*>(smem);
  for (int g = threadIdx.x; g < m * NB; g += blockDim.x) {
    int j = g / NB, c = g % NB;
    Cs[g] = c < nb ? C[j + (int64_t)c * ldc] : S(0);
  }
  __syncthreads();
  for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < n;
       row += (int64_t)gridDim.x * blockDim.x) {
    S acc[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) acc[c] = S(0);
    for (int j = 0; j < m; ++j) {
      S qv = Q[(int64_t)j * ldq + row];
#pragma unroll
      for (int c = 0; c < NB; ++c) acc[c] = acc[c] + qv * Cs[j * NB + c];
    }
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < nb) X[c * ldx + row] = X[c * ldx + row] - acc[c];
  }
}

// X = X R^-1, R upper triangular nb x nb (column-major, ldr = nb), per row
template <typename S, int NB>
__global__ void __launch_bounds__(kThreads)
    k_trsm_right_upper(const S* __restrict__ R, S* __restrict__ X, int64_t ldx, int nb,
                       int64_t n) {
  __shared__ double Rs_raw[NB * NB * Ops<S>::W];
  S* Rs = reinterpret_cast<S*>(Rs_raw);
  for (int g = threadIdx.x; g < nb * nb; g += blockDim.x) Rs[g] = R[g];
  __syncthreads();
  for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < n;
       row += (int64_t)gridDim.x * blockDim.x) {
    S y[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      if (c < nb) {
        S v = X[c * ldx + row];
#pragma unroll
        for (int k = 0; k < NB; ++k)
          if (k < c) v = v - y[k] * Rs[k + c * nb];
        y[c] = cdiv_s(v, Rs[c + c * nb]);
      } else {
        y[c] = S(0);
      }
    }
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < nb) X[c * ldx + row] = y[c];
  }
}

// ---------------------------------------------------------------- host wrappers

namespace {
thread_local DevBuf g_partial;

unsigned rows_grid(int64_t n) {
  int64_t g = (n + kThreads - 1) / kThreads;
  return (unsigned)(g < 4096 ? (g < 1 ? 1 : g) : 4096);
}
}  // namespace

template <typename S, int JT, int NB>
static int gram_t(const S* A, int64_t lda, int m, const S* B, int64_t ldb, int nb, int64_t n,
                  S* C, int ldc, hipStream_t s) {
  constexpr int W = Ops<S>::W;
  const int ntiles = (m + JT - 1) / JT;
  int nchunks = (int)((n + kChunk - 1) / kChunk);
  const int nchunks_pad = (nchunks + kXcd - 1) / kXcd * kXcd;
  YR_CALL(g_partial.reserve((size_t)nchunks * ntiles * JT * NB * W * sizeof(double)));
  const unsigned grid = (unsigned)((int64_t)ntiles * nchunks_pad);
  k_gram_partial<S, JT, NB><<<grid, kThreads, 0, s>>>(A, lda, m, B, ldb, nb, n, ntiles, nchunks,
                                                     g_partial.as<double>());
  k_gram_reduce<S, JT, NB><<<ntiles, 1024, 0, s>>>(g_partial.as<double>(), ntiles, nchunks, m, nb,
                                                   C, ldc);
  YR_TRY_HIP(hipGetLastError());
  return YR_OK;
}

template <typename S>
int ts_gram(const S* A, int64_t lda, int m, const S* B, int64_t ldb, int nb, int64_t n, S* C,
            int ldc, hipStream_t s) {
  if (m == 0 || nb == 0) return YR_OK;
  // column blocks of B of at most 8 (real) / 4 (complex) columns per launch
  // pair, each launch reading A again; complex blocks wider than 4 columns
  // take 8 per launch against tiles of 4 columns of A (the same registers):
  // half the passes over A, B re-read from L2 twice as often
  constexpr bool CPLX = sizeof(S) == 16;
  if constexpr (CPLX) {
    if (nb > 4) {
      for (int c0 = 0; c0 < nb; c0 += 8) {
        int nbc = nb - c0 < 8 ? nb - c0 : 8;
        YR_CALL((gram_t<S, 4, 8>(A, lda, m, B + (int64_t)c0 * ldb, ldb, nbc, n,
                                 C + (int64_t)c0 * ldc, ldc, s)));
      }
      return YR_OK;
    }
  }
  constexpr int NB = CPLX ? 4 : 8;
  constexpr int JT = 8;
  for (int c0 = 0; c0 < nb; c0 += NB) {
    int nbc = nb - c0 < NB ? nb - c0 : NB;
    YR_CALL((gram_t<S, JT, NB>(A, lda, m, B + (int64_t)c0 * ldb, ldb, nbc, n,
                               C + (int64_t)c0 * ldc, ldc, s)));
  }
  return YR_OK;
}

template <typename S>
int ts_update(const S* Q, int64_t ldq, int m, const S* C, int ldc, S* X, int64_t ldx, int nb,
              int64_t n, hipStream_t s) {
  if (m == 0 || nb == 0) return YR_OK;
  // blocks of 9..16 columns in one launch (one pass over Q), narrower ones
  // in launches of 8
  if (nb > 8 && (size_t)m * 16 * sizeof(S) <= 64 * 1024) {
    k_update<S, 16><<<rows_grid(n), kThreads, (size_t)m * 16 * sizeof(S), s>>>(Q, ldq, m, C, ldc,
                                                                               X, ldx, nb, n);
    YR_TRY_HIP(hipGetLastError());
    return YR_OK;
  }
  constexpr int NB = 8;
  for (int c0 = 0; c0 < nb; c0 += NB) {
    int nbc = nb - c0 < NB ? nb - c0 : NB;
    size_t smem = (size_t)m * NB * sizeof(S);
    YR_REQUIRE(smem <= 64 * 1024, YR_EINVAL, "basis too wide for the update kernel");
    k_update<S, NB><<<rows_grid(n), kThreads, smem, s>>>(Q, ldq, m, C + (int64_t)c0 * ldc, ldc,
                                                         X + (int64_t)c0 * ldx, ldx, nbc, n);
  }
  YR_TRY_HIP(hipGetLastError());
  return YR_OK;
}

template <typename S>
int ts_trsm(const S* R, S* X, int64_t ldx, int nb, int64_t n, hipStream_t s) {
  if (nb == 0) return YR_OK;
  YR_REQUIRE(nb <= 32, YR_EINVAL, "block wider than 32 columns");
  if (nb <= 8)
    k_trsm_right_upper<S, 8><<<rows_grid(n), kThreads, 0, s>>>(R, X, ldx, nb, n);
  else if (nb <= 16)
    k_trsm_right_upper<S, 16><<<rows_grid(n), kThreads, 0, s>>>(R, X, ldx, nb, n);
  else
    k_trsm_right_upper<S, 32><<<rows_grid(n), kThreads, 0, s>>>(R, X, ldx, nb, n);
  YR_TRY_HIP(hipGetLastError());
  return YR_OK;
}

template int ts_gram<double>(const double*, int64_t, int, const double*, int64_t, int, int64_t,
                             double*, int, hipStream_t);
template int ts_gram<zd>(const zd*, int64_t, int, const zd*, int64_t, int, int64_t, zd*, int,
                         hipStream_t);
template int ts_update<double>(const double*, int64_t, int, const double*, int, double*, int64_t,
                               int, int64_t, hipStream_t);
template int ts_update<zd>(const zd*, int64_t, int, const zd*, int, zd*, int64_t, int, int64_t,
                           hipStream_t);
template int ts_trsm<double>(const double*, double*, int64_t, int, int64_t, hipStream_t);
template int ts_trsm<zd>(const zd*, zd*, int64_t, int, int64_t, hipStream_t);

}  // namespace yr
