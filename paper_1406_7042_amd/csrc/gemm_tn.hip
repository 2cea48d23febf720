// Tall-skinny FP64 products on the matrix cores (v_mfma_f64_16x16x4f64):
//   C (m x m)  = A^T diag(w) A   the Gram matrices of the orthogonalisation and
//                                the diagonal-material projections of eq.
//                                (R_and_Freduced) (V1^T De V1, V1^T Dse V1,
//                                V2^T Dm V2): tiles on and above the diagonal
//                                only, mirrored;
//   C (m x nc) = A^T diag(w) B   the projection V1^T (K V2) of the same
//                                equation: every tile;
//   X <- X U   (U upper triangular r x r)   the V R^-1 step of CholQR2, in
//                                place, row chunk by row chunk.
// A, B and X are column-major with n >> m rows, at most 256 columns.
//
// Gram and product: each workgroup (16 waves) streams its own band of rows
// through LDS in chunks of RB rows, RB = 32 for up to 256 columns and 64, 128,
// 256 for up to 128, 64, 32 (the next chunk is fetched into registers while
// the current one is multiplied; fewer columns, longer chunks, more bytes in
// flight; the two-operand product stages A and B in chunks of half as many
// rows, the registers holding half a chunk of each); each
// wave accumulates up to 6 output tiles of 16 x 16 in registers, one MFMA per
// tile and 4 rows.  MFMA operand layout (16x16x4, FP64): lane l supplies
// A_op[l % 16][l / 16] and B_op[l / 16][l % 16] and holds D[l / 16 + 4 r][l % 16],
// r = 0..3.  With A_op = (rows of A)^T and B_op = w (rows of B), D accumulates
// A^T diag(w) B.  The per-workgroup tiles are summed over workgroups in a
// fixed order (k_gram_reduce_mfma).
#include <algorithm>
#include <vector>

#include "gemm_tn.hpp"

namespace yr {

namespace {
typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kMaxCols = 256;          // m <= kMaxCols
constexpr int kRBMax = 256;            // rows per chunk at most
constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / 64;
constexpr int kTilesPerWave = 6;    // 16 waves x 6 tiles: a 256-column Gram in two launches
constexpr int kTilesPerLaunch = kWaves * kTilesPerWave;

constexpr int kBlocks = 256;           // one workgroup per compute unit (LDS)

constexpr int kPF = 8;  // prefetch slots per thread: RB * m <= kPF * kThreads for every class

// rows per chunk for m columns: the RB x (kPF * kThreads / RB) slots cover them
inline int gram_rb(int m) { return m <= 32 ? 256 : m <= 64 ? 128 : m <= 128 ? 64 : 32; }
// the two-operand product prefetches kPF / 2 slots of each operand: half the rows
inline int gemm_rb(int m) { return gram_rb(m) / 2; }

// output tile t -> (ti, tj) on or above the diagonal, row by row
__device__ inline void tile_of(int t, int TI, int& ti, int& tj) {
  ti = 0;
  while (t >= TI - ti) {
    t -= TI - ti;
    ++ti;
  }
  tj = ti + t;
}

// AB = false: B is A (Gram, tiles on and above the diagonal, t -> tile_of);
// AB = true: B has its own LDS tile, all TI x TJ tiles (t -> t / TJ, t % TJ)
template <int RB, bool AB>
__global__ void __launch_bounds__(kThreads)
    k_gram_mfma(const double* __restrict__ A, int64_t lda, int m, const double* __restrict__ B,
                int64_t ldb, int nc, const double* __restrict__ w, int64_t n,
                int64_t rows_per_block, int t0, int nt, double* __restrict__ partial) {
  static_assert(RB % 4 == 0 && RB <= kRBMax && kThreads % RB == 0, "chunk rows");
  // prefetch slots per thread and operand: the product holds two operands in
  // the registers the Gram gives one
  constexpr int PF = AB ? kPF / 2 : kPF;
  // LDS row stride: every slot column plus one.  The chunk is stored column
  // by column (consecutive lanes hold consecutive rows of one column): with an
  // odd stride those lanes write distinct banks, where a stride of 16 mod 32
  // doubles put all of them on one bank (50M x 200 Gram: 8.6 -> 6.2 ms).  The
  // MFMA reads take 16 consecutive doubles of a row per 16 lanes.  RB x ldA
  // is 64-72 KB (twice 32-40 KB with AB).
  constexpr int ldA = PF * kThreads / RB + 1;
  static_assert(RB * ldA >= kWaves * 256, "LDS tile");
  __shared__ double As[(AB ? 2 : 1) * RB * ldA];
  __shared__ double ws[kRBMax];
  double* Bs = AB ? As + RB * ldA : As;
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: tiles in SGPRs
  const int TI = (m + 15) / 16, TJ = (nc + 15) / 16;
  // zero the tiles once (the columns past the last slot are never written)
  for (int g = threadIdx.x; g < (AB ? 2 : 1) * RB * ldA; g += kThreads) As[g] = 0.0;
  // With fewer than half as many tiles as waves, nph waves share a tile and
  // take every nph-th group of 4 rows of each chunk (row phase ph); their
  // accumulators are summed at the end in phase order.
  constexpr int TPW = kTilesPerWave;
  const int nph = nt * 2 <= kWaves ? min(kWaves / nt, RB / 4) : 1;
  const int ph = wid / nt;          // row phase (nph > 1)
  const int wt = nph > 1 ? wid % nt : wid;
  int ti[TPW], tj[TPW];
  bool tv[TPW];
  v4d acc[TPW];
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    const int t = wt + kWaves * u;
    tv[u] = nph > 1 ? (u == 0 && ph < nph) : t < nt;
    ti[u] = tj[u] = 0;
    if (tv[u]) {
      if (AB) {
        ti[u] = (t0 + t) / TJ;
        tj[u] = (t0 + t) % TJ;
      } else {
        tile_of(t0 + t, TI, ti[u], tj[u]);
      }
    }
    acc[u] = v4d{0.0, 0.0, 0.0, 0.0};
  }
  const int k4_0 = nph > 1 ? 4 * ph : 0, k4_step = 4 * nph;
  const int64_t r0 = blockIdx.x * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < n ? r0 + rows_per_block : n;
  // register prefetch of one chunk: every slot loads (clamped row and column,
  // no branch), so the loads issue back to back; rows past the band and
  // columns past m are zeroed when stored to LDS.  The first RB threads load
  // the weights.
  double pa[PF], pb[AB ? PF : 1], pw = 1.0;
  auto fetch = [&](int64_t rc) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int g = threadIdx.x + u * kThreads;
      const int c = g / RB, r = g - c * RB;
      const int cc = c < m ? c : m - 1;
      const int64_t row = rc + r < r1 ? rc + r : r1 - 1;
      pa[u] = A[cc * lda + row];
      if (AB) pb[u] = B[(int64_t)(c < nc ? c : nc - 1) * ldb + row];
    }
    if (w && wid < (RB + 63) / 64) {
      const int r = threadIdx.x & (RB - 1);
      pw = w[rc + r < r1 ? rc + r : r1 - 1];
    }
  };
  if (r0 < r1) fetch(r0);
  __syncthreads();
  for (int64_t rc = r0; rc < r1; rc += RB) {
#pragma unroll
    for (int u = 0; u < PF; ++u) {  // c < PF * kThreads / RB = ldA - 1: inside the tile
      const int g = threadIdx.x + u * kThreads;
      const int c = g / RB, r = g - c * RB;
      As[r * ldA + c] = c < m && rc + r < r1 ? pa[u] : 0.0;
      if (AB) Bs[r * ldA + c] = c < nc && rc + r < r1 ? pb[u] : 0.0;
    }
    if (threadIdx.x < RB) ws[threadIdx.x] = rc + threadIdx.x < r1 ? pw : 0.0;
    __syncthreads();
    if (rc + RB < r1) fetch(rc + RB);  // in flight during the MFMAs
    for (int k4 = k4_0; k4 < RB; k4 += k4_step) {
      const int kr = k4 + (lane >> 4);
      const double wv = ws[kr];
      const double* arow = As + kr * ldA + (lane & 15);
      const double* brow = Bs + kr * ldA + (lane & 15);
#pragma unroll
      for (int u = 0; u < TPW; ++u) {
        if (tv[u]) {
          const double a = arow[ti[u] * 16];
          const double b = brow[tj[u] * 16] * wv;
          acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[u], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  if (nph > 1) {  // sum the row phases of each tile (As is free now), phase 0 stores
    if (tv[0] && ph > 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r)
        As[((ph - 1) * nt + wt) * 256 + ((lane >> 4) + 4 * r) * 16 + (lane & 15)] = acc[0][r];
    }
    __syncthreads();
    if (tv[0] && ph == 0) {
      for (int p = 1; p < nph; ++p)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc[0][r] += As[((p - 1) * nt + wt) * 256 + ((lane >> 4) + 4 * r) * 16 + (lane & 15)];
    }
  }
  // partial[block][tile][256]: lane l, r -> element (l / 16 + 4 r) * 16 + l % 16
#pragma unroll
  for (int u = 0; u < TPW; ++u) {
    const int t = wt + kWaves * u;
    if (!tv[u] || (nph > 1 && ph != 0)) continue;
    double* out = partial + ((int64_t)blockIdx.x * nt + t) * 256;
#pragma unroll
    for (int r = 0; r < 4; ++r) out[((lane >> 4) + 4 * r) * 16 + (lane & 15)] = acc[u][r];
  }
}

// C tile elements: sum over the workgroups in block order; a Gram (nc < 0)
// is mirrored, a two-operand product (nc columns) is not
__global__ void k_gram_reduce_mfma(const double* __restrict__ partial, int nblocks, int nt, int t0,
                                   int m, int nc, double* __restrict__ C, int ldc) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= (int64_t)nt * 256) return;
  const int t = (int)(g / 256), e = (int)(g - (int64_t)t * 256);
  int ti, tj;
  if (nc < 0) {
    tile_of(t0 + t, (m + 15) / 16, ti, tj);
  } else {
    ti = (t0 + t) / ((nc + 15) / 16);
    tj = (t0 + t) % ((nc + 15) / 16);
  }
  const int i = ti * 16 + e / 16, j = tj * 16 + e % 16;
  if (i >= m || j >= (nc < 0 ? m : nc)) return;
  double s = 0;
  for (int b = 0; b < nblocks; ++b) s += partial[((int64_t)b * nt + t) * 256 + e];
  C[i + (int64_t)j * ldc] = s;
  if (nc < 0 && i != j) C[j + (int64_t)i * ldc] = s;
}

// ---- X <- X U in place (U upper triangular, r x r)

constexpr int kTrThreads = 512;  // 8 waves, 2 per SIMD: 256 registers each
constexpr int kTrWaves = kTrThreads / 64;

// Each workgroup owns a band of rows and walks it in chunks of RB rows x CAP
// columns (CAP >= r): the chunk is staged in LDS (column-major), Y = X_chunk U
// is formed on the matrix cores and written over the chunk's rows, which no
// other chunk reads.  Wave -> output column tiles: the pair (p, TC-1-p), whose
// k-steps (4 per 16 columns up to the tile's last column) add up to 4 (TC + 1)
// at most, so the waves carry about equal MFMA counts; the CAP / 32 pairs
// share the 8 waves, each wave takes RTW of the chunk's row tiles.
// U enters as the A operand (U^T tile x X_chunk^T = Y^T tile): lane l
// supplies U[4 ks + l / 16][16 ct + l % 16], loaded once into registers for
// the whole launch (slot i < kA: k-step i of the first tile; slot KT-1-i,
// i < kB: k-step i of the second), so the only loads in flight during the
// MFMAs are the next chunk's; the wave holds Y[row0 + l % 16][16 ct + l / 16
// + 4 r], and each store instruction writes 16 consecutive rows of 4 columns.
template <int RB, int CAP>
__global__ void __launch_bounds__(kTrThreads)
    k_trmm_upper(double* __restrict__ X, int64_t ldx, int r, const double* __restrict__ U,
                 int64_t n, int64_t rows_per_block) {
  constexpr int RT = RB / 16;          // row tiles per chunk
  constexpr int NPM = CAP / 32;        // pairs at most
  constexpr int WPP = kTrWaves / NPM;  // waves per pair
  constexpr int RTW = RT / WPP;        // row tiles per wave
  constexpr int KT = CAP / 4 + 4;      // U operand slots of a pair: 4 (TC + 1), TC = CAP / 16
  constexpr int NPF = RB * CAP / kTrThreads;
  static_assert(kTrThreads % RB == 0 && WPP * NPM == kTrWaves && RTW * WPP == RT, "chunk shape");
  __shared__ double Xs[RB * CAP];  // Xs[c * RB + row]
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int TC = (r + 15) / 16, KR = (r + 3) / 4;
  const int npairs = (TC + 1) / 2;
  const int pr = wid % NPM, rt0 = (wid / NPM) * RTW;
  const bool active = pr < npairs;
  const int ctA = pr, ctB = TC - 1 - pr;
  const int kA = active ? min(4 * (ctA + 1), KR) : 0;
  const int kB = active && ctB > ctA ? min(4 * (ctB + 1), KR) : 0;
  double ub[KT];
#pragma unroll
  for (int i = 0; i < KT; ++i) {
    int kk = 0, cc = 0;
    bool ok = false;
    if (i < kA) {
      kk = 4 * i + (lane >> 4);
      cc = 16 * ctA + (lane & 15);
      ok = true;
    } else if (KT - 1 - i < kB) {
      kk = 4 * (KT - 1 - i) + (lane >> 4);
      cc = 16 * ctB + (lane & 15);
      ok = true;
    }
    ok = ok && kk <= cc && cc < r;  // the upper triangle only
    ub[i] = ok ? U[kk + (int64_t)cc * r] : 0.0;
  }
  const int64_t r0 = blockIdx.x * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < n ? r0 + rows_per_block : n;
  // slot u of this thread: row threadIdx.x % RB, column threadIdx.x / RB + u
  // kTrThreads / RB (clamped row and column: the loads never branch)
  const int prow = threadIdx.x % RB, pcol = threadIdx.x / RB;
  double pa[NPF];
  auto fetch = [&](int64_t rc) __attribute__((always_inline)) {
    const int64_t row = rc + prow < r1 ? rc + prow : r1 - 1;
#pragma unroll
    for (int u = 0; u < NPF; ++u) {
      const int c = pcol + u * (kTrThreads / RB);
      pa[u] = X[(int64_t)(c < r ? c : r - 1) * ldx + row];
    }
  };
  if (r0 < r1) fetch(r0);
  for (int64_t rc = r0; rc < r1; rc += RB) {
#pragma unroll
    for (int u = 0; u < NPF; ++u) {
      const int c = pcol + u * (kTrThreads / RB);
      Xs[c * RB + prow] = c < r && rc + prow < r1 ? pa[u] : 0.0;
    }
    __syncthreads();
    if (rc + RB < r1) fetch(rc + RB);  // in flight during the MFMAs
    v4d accA[RTW], accB[RTW];
#pragma unroll
    for (int i = 0; i < RTW; ++i) accA[i] = accB[i] = v4d{0.0, 0.0, 0.0, 0.0};
    // B_op[l / 16][l % 16] = X[row0 + l % 16][4 ks + l / 16]; 4 ks + 3 < CAP
    const double* xs = Xs + (lane >> 4) * RB + 16 * rt0 + (lane & 15);
#pragma unroll
    for (int ks = 0; ks < KT; ++ks) {
      if (ks < kA || ks < kB) {
#pragma unroll
        for (int i = 0; i < RTW; ++i) {
          const double xv = xs[4 * ks * RB + 16 * i];
          if (ks < kA) accA[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(ub[ks], xv, accA[i], 0, 0, 0);
          if (ks < kB)
            accB[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(ub[KT - 1 - ks], xv, accB[i], 0, 0, 0);
        }
      }
    }
    if (active) {
#pragma unroll
      for (int i = 0; i < RTW; ++i) {
        const int64_t row = rc + 16 * (rt0 + i) + (lane & 15);
        if (row >= r1) continue;
#pragma unroll
        for (int r4 = 0; r4 < 4; ++r4) {
          const int ca = 16 * ctA + (lane >> 4) + 4 * r4, cb = 16 * ctB + (lane >> 4) + 4 * r4;
          if (ca < r) X[ca * ldx + row] = accA[i][r4];
          if (kB > 0 && cb < r) X[cb * ldx + row] = accB[i][r4];
        }
      }
    }
    __syncthreads();  // the next chunk overwrites Xs
  }
}

// U = R^-1 for upper triangular R (r x r, column-major, ld r): block j (one
// wave) solves R u = e_j from the bottom row up, the partial sums split over
// the lanes and combined by shuffles
__global__ void __launch_bounds__(64)
    k_tri_inv_upper(const double* __restrict__ R, int r, double* __restrict__ U) {
  __shared__ double u[kMaxCols];
  const int lane = threadIdx.x, j = blockIdx.x;
  for (int m = lane; m < r; m += 64) u[m] = 0.0;
  __syncthreads();
  if (lane == 0) u[j] = 1.0 / R[j + (int64_t)j * r];
  __syncthreads();
  for (int i = j - 1; i >= 0; --i) {
    double acc = 0.0;
    for (int m = i + 1 + lane; m <= j; m += 64) acc += R[i + (int64_t)m * r] * u[m];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) u[i] = -acc / R[i + (int64_t)i * r];
    __syncthreads();
  }
  for (int m = lane; m < r; m += 64) U[m + (int64_t)j * r] = u[m];
}

// rows per chunk of the triangular product by column capacity (64, 128, 256)
constexpr int kTrRB64 = 64, kTrRB128 = 32, kTrRB256 = 16;
inline int trmm_rb(int r) { return r <= 64 ? kTrRB64 : r <= 128 ? kTrRB128 : kTrRB256; }

thread_local DevBuf g_tn_partial;

// rows per workgroup: the rows split evenly over kBlocks bands, a multiple of RB
int64_t band_rows(int64_t n, int RB) {
  int64_t rpb = (n + kBlocks - 1) / kBlocks;
  return (rpb + RB - 1) / RB * RB;
}
}  // namespace

// C = A^T diag(w) B; B null: the Gram of A (tiles on and above the diagonal)
static int tn_mfma(const double* A, int64_t lda, int m, const double* B, int64_t ldb, int nc,
                   const double* w, int64_t n, double* C, int ldc, hipStream_t s) {
  const bool ab = B != nullptr;
  YR_REQUIRE(m > 0 && m <= kMaxCols && (!ab || (nc > 0 && nc <= kMaxCols)), YR_EINVAL,
             "matrix-core product: 1..256 columns");
  YR_REQUIRE(n > 0, YR_EINVAL, "matrix-core product: no rows");
  const int TI = (m + 15) / 16, TJ = ab ? (nc + 15) / 16 : 0;
  const int ntiles = ab ? TI * TJ : TI * (TI + 1) / 2;
  const int RB = ab ? gemm_rb(std::max(m, nc)) : gram_rb(m);
  const int64_t rpb = band_rows(n, RB);
  const int nblocks = (int)((n + rpb - 1) / rpb);
  const int per_launch = kTilesPerLaunch;
  YR_CALL(g_tn_partial.reserve((size_t)nblocks * std::min(ntiles, per_launch) * 256 * 8));
  for (int t0 = 0; t0 < ntiles; t0 += per_launch) {
    const int nt = std::min(per_launch, ntiles - t0);
    if (ab) {
      auto* k = RB == 128 ? k_gram_mfma<128, true> : RB == 64 ? k_gram_mfma<64, true>
                : RB == 32 ? k_gram_mfma<32, true> : k_gram_mfma<16, true>;
      k<<<nblocks, kThreads, 0, s>>>(A, lda, m, B, ldb, nc, w, n, rpb, t0, nt,
                                     g_tn_partial.as<double>());
    } else {
      auto* k = RB == 256 ? k_gram_mfma<256, false> : RB == 128 ? k_gram_mfma<128, false>
                : RB == 64 ? k_gram_mfma<64, false> : k_gram_mfma<32, false>;
      k<<<nblocks, kThreads, 0, s>>>(A, lda, m, A, lda, m, w, n, rpb, t0, nt,
                                     g_tn_partial.as<double>());
    }
    const int64_t tot = (int64_t)nt * 256;
    k_gram_reduce_mfma<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(
        g_tn_partial.as<double>(), nblocks, nt, t0, m, ab ? nc : -1, C, ldc);
  }
  YR_TRY_HIP(hipGetLastError());
  return YR_OK;
}

int gram_mfma(const double* A, int64_t lda, int m, const double* w, int64_t n, double* C, int ldc,
              hipStream_t s) {
  return tn_mfma(A, lda, m, nullptr, 0, 0, w, n, C, ldc, s);
}

int gemm_tn_mfma(const double* A, int64_t lda, int m, const double* B, int64_t ldb, int nc,
                 const double* w, int64_t n, double* C, int ldc, hipStream_t s) {
  YR_REQUIRE(B, YR_EINVAL, "gemm_tn_mfma: null B");
  return tn_mfma(A, lda, m, B, ldb, nc, w, n, C, ldc, s);
}

int tri_inv_upper(const double* R, int r, double* U, hipStream_t s) {
  YR_REQUIRE(r > 0 && r <= kMaxCols, YR_EINVAL, "tri_inv_upper: 1..256 columns");
  k_tri_inv_upper<<<r, 64, 0, s>>>(R, r, U);
  YR_TRY_HIP(hipGetLastError());
  return YR_OK;
}

int trmm_upper_inplace(double* X, int64_t ldx, int r, const double* U, int64_t n, hipStream_t s) {
  YR_REQUIRE(r > 0 && r <= kMaxCols, YR_EINVAL, "trmm_upper_inplace: 1..256 columns");
  if (n == 0) return YR_OK;
  const int cap = r <= 64 ? 64 : r <= 128 ? 128 : 256;
  const int RB = trmm_rb(r);
  const int64_t rpb = band_rows(n, RB);
  const unsigned nblocks = (unsigned)((n + rpb - 1) / rpb);
  auto* k = cap == 64 ? k_trmm_upper<kTrRB64, 64> : cap == 128 ? k_trmm_upper<kTrRB128, 128>
                                                    : k_trmm_upper<kTrRB256, 256>;
  k<<<nblocks, kTrThreads, 0, s>>>(X, ldx, r, U, n, rpb);
  YR_TRY_HIP(hipGetLastError());
  return YR_OK;
}

}  // namespace yr
