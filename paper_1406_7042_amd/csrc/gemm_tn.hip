// C (m x m) = A^T diag(w) A for tall-skinny FP64 A (n x m), n >> m, m <= 256,
// on the FP64 matrix cores (v_mfma_f64_16x16x4f64): the Gram matrices of the
// orthogonalisation and the diagonal-material projections of eq.
// (R_and_Freduced) (V1^T De V1, V1^T Dse V1, V2^T Dm V2).  Only the output
// tiles on and above the diagonal are formed; the result is mirrored.
//
// Each workgroup (16 waves) streams its own band of rows through LDS in chunks
// of RB rows, RB = 32 for up to 256 columns and 64, 128, 256 for up to 128,
// 64, 32 (the next chunk is fetched into registers while the current one is
// multiplied; fewer columns, longer chunks, more bytes in flight); each wave
// accumulates up to 6 output tiles of 16 x 16 in registers, one MFMA per tile
// and 4 rows.  MFMA operand layout (16x16x4, FP64): lane l supplies
// A_op[l % 16][l / 16] and B_op[l / 16][l % 16] and holds D[l / 16 + 4 r][l % 16],
// r = 0..3.  With A_op = (rows of A)^T and
// B_op = w (rows of A), D accumulates A^T diag(w) A.  The per-workgroup tiles
// are summed over workgroups in a fixed order (k_gram_reduce_mfma).
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

// output tile t -> (ti, tj) on or above the diagonal, row by row
__device__ inline void tile_of(int t, int TI, int& ti, int& tj) {
  ti = 0;
  while (t >= TI - ti) {
    t -= TI - ti;
    ++ti;
  }
  tj = ti + t;
}

template <int RB>
__global__ void __launch_bounds__(kThreads)
    k_gram_mfma(const double* __restrict__ A, int64_t lda, int m, const double* __restrict__ w,
                int64_t n, int64_t rows_per_block, int t0, int nt, double* __restrict__ partial) {
  static_assert(RB % 4 == 0 && RB <= kRBMax && kThreads % RB == 0, "chunk rows");
  // LDS row stride: every slot column plus 16, an odd multiple of 16 (rows 32
  // banks apart); RB x ldA is 68-96 KB
  constexpr int ldA = kPF * kThreads / RB + 16;
  static_assert(ldA % 32 == 16 && RB * ldA >= kWaves * 256, "LDS tile");
  __shared__ double As[RB * ldA];
  __shared__ double ws[kRBMax];
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: tiles in SGPRs
  const int TI = (m + 15) / 16;
  // zero the tile once (the columns past the last slot are never written)
  for (int g = threadIdx.x; g < RB * ldA; g += kThreads) As[g] = 0.0;
  // With fewer than half as many tiles as waves, nph waves share a tile and
  // take every nph-th group of 4 rows of each chunk (row phase ph); their
  // accumulators are summed at the end in phase order.
  const int nph = nt * 2 <= kWaves ? min(kWaves / nt, RB / 4) : 1;
  const int ph = wid / nt;          // row phase (nph > 1)
  const int wt = nph > 1 ? wid % nt : wid;
  int ti[kTilesPerWave], tj[kTilesPerWave];
  bool tv[kTilesPerWave];
  v4d acc[kTilesPerWave];
#pragma unroll
  for (int u = 0; u < kTilesPerWave; ++u) {
    const int t = wt + kWaves * u;
    tv[u] = nph > 1 ? (u == 0 && ph < nph) : t < nt;
    ti[u] = tj[u] = 0;
    if (tv[u]) tile_of(t0 + t, TI, ti[u], tj[u]);
    acc[u] = v4d{0.0, 0.0, 0.0, 0.0};
  }
  const int k4_0 = nph > 1 ? 4 * ph : 0, k4_step = 4 * nph;
  const int64_t r0 = blockIdx.x * rows_per_block;
  const int64_t r1 = r0 + rows_per_block < n ? r0 + rows_per_block : n;
  // register prefetch of one chunk: every slot loads (clamped row and column,
  // no branch), so the loads issue back to back; rows past the band and
  // columns past m are zeroed when stored to LDS.  The first RB threads load
  // the weights.
  double pa[kPF], pw = 1.0;
  auto fetch = [&](int64_t rc) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < kPF; ++u) {
      const int g = threadIdx.x + u * kThreads;
      const int c = g / RB, r = g - c * RB;
      const int cc = c < m ? c : m - 1;
      const int64_t row = rc + r < r1 ? rc + r : r1 - 1;
      pa[u] = A[cc * lda + row];
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
    for (int u = 0; u < kPF; ++u) {  // c < kPF * kThreads / RB = ldA - 16: inside the tile
      const int g = threadIdx.x + u * kThreads;
      const int c = g / RB, r = g - c * RB;
      As[r * ldA + c] = c < m && rc + r < r1 ? pa[u] : 0.0;
    }
    if (threadIdx.x < RB) ws[threadIdx.x] = rc + threadIdx.x < r1 ? pw : 0.0;
    __syncthreads();
    if (rc + RB < r1) fetch(rc + RB);  // in flight during the MFMAs
#pragma unroll 2
    for (int k4 = k4_0; k4 < RB; k4 += k4_step) {
      const int kr = k4 + (lane >> 4);
      const double wv = ws[kr];
      const double* arow = As + kr * ldA + (lane & 15);
#pragma unroll
      for (int u = 0; u < kTilesPerWave; ++u) {
        if (tv[u]) {
          const double a = arow[ti[u] * 16];
          const double b = arow[tj[u] * 16] * wv;
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
  for (int u = 0; u < kTilesPerWave; ++u) {
    const int t = wt + kWaves * u;
    if (!tv[u] || (nph > 1 && ph != 0)) continue;
    double* out = partial + ((int64_t)blockIdx.x * nt + t) * 256;
#pragma unroll
    for (int r = 0; r < 4; ++r) out[((lane >> 4) + 4 * r) * 16 + (lane & 15)] = acc[u][r];
  }
}

// C tile elements: sum over the workgroups in block order, mirrored
__global__ void k_gram_reduce_mfma(const double* __restrict__ partial, int nblocks, int nt, int t0,
                                   int m, double* __restrict__ C, int ldc) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= (int64_t)nt * 256) return;
  const int t = (int)(g / 256), e = (int)(g - (int64_t)t * 256);
  int ti, tj;
  tile_of(t0 + t, (m + 15) / 16, ti, tj);
  const int i = ti * 16 + e / 16, j = tj * 16 + e % 16;
  if (i >= m || j >= m) return;
  double s = 0;
  for (int b = 0; b < nblocks; ++b) s += partial[((int64_t)b * nt + t) * 256 + e];
  C[i + (int64_t)j * ldc] = s;
  if (i != j) C[j + (int64_t)i * ldc] = s;
}

thread_local DevBuf g_tn_partial;
}  // namespace

int gram_mfma(const double* A, int64_t lda, int m, const double* w, int64_t n, double* C, int ldc,
              hipStream_t s) {
  YR_REQUIRE(m > 0 && m <= kMaxCols, YR_EINVAL, "gram_mfma: 1..256 columns");
  YR_REQUIRE(n > 0, YR_EINVAL, "gram_mfma: no rows");
  const int TI = (m + 15) / 16;
  const int ntiles = TI * (TI + 1) / 2;
  const int RB = gram_rb(m);
  int64_t rpb = (n + kBlocks - 1) / kBlocks;
  rpb = (rpb + RB - 1) / RB * RB;
  const int nblocks = (int)((n + rpb - 1) / rpb);
  YR_CALL(g_tn_partial.reserve((size_t)nblocks * std::min(ntiles, kTilesPerLaunch) * 256 * 8));
  for (int t0 = 0; t0 < ntiles; t0 += kTilesPerLaunch) {
    const int nt = std::min(kTilesPerLaunch, ntiles - t0);
    auto* k = RB == 256 ? k_gram_mfma<256> : RB == 128 ? k_gram_mfma<128>
              : RB == 64 ? k_gram_mfma<64> : k_gram_mfma<32>;
    k<<<nblocks, kThreads, 0, s>>>(A, lda, m, w, n, rpb, t0, nt, g_tn_partial.as<double>());
    const int64_t tot = (int64_t)nt * 256;
    k_gram_reduce_mfma<<<(unsigned)((tot + 255) / 256), 256, 0, s>>>(g_tn_partial.as<double>(),
                                                                     nblocks, nt, t0, m, C, ldc);
  }
  YR_TRY_HIP(hipGetLastError());
  return YR_OK;
}

}  // namespace yr
