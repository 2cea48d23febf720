// Stability enforcement above the CFL limit (Sec. III-A) and the reduced
// leapfrog (eq. (reducedMNAform), Sec. II-C last remark), batched over many
// reduced models (stage kernels and the stepping: one workgroup per model;
// Jacobi phases: several workgroups per model).
//
// rom_perturb works in FP64 on the device:
//   De~ = Le Le^T, Dm~ = Lm Lm^T (Cholesky),  A = Le^-1 K~ Lm^-T,
//   A = U S W^T (QR-preconditioned one-sided Jacobi),
//   s'_i = min(s_i, gamma 2/dt), A' = U S' W^T,  K~' = Le A' Lm^T.
// Any square root of De~, Dm~ gives the same K~' (the Cholesky factor and the
// symmetric root differ by an orthogonal factor that cancels).  The stepping
// form whitens the state, e' = Le^T e~, h' = Lm^T h~, and rotates it onto the
// eigenvectors of the whitened loss matrices Se = Le^-1 Dse~ Le^-T,
// Sm = Lm^-1 Dsm~ Lm^-T (Se = Qe diag(le) Qe^T), so that each step is
//   e <- ce*e - ge*(A'' h) + ge*(be u),  h <- cm*h + gm*(A''^T e) + gm*(bh u)
// with A'' = Qe^T A' Qm, ce = (1/dt - le/2)/(1/dt + le/2), ge = 1/(1/dt + le/2).
// With the values actually stored in the stepping precision, this is again a
// leapfrog of the form of eq. (MNAform) with diagonal De/dt = (1+ce)/(2ge) and
// losses (1-ce)/ge >= 0, so condition (Dstability2) reduces to
// sigma_max(M) < 2, M = diag(sqrt(2ge/(1+ce))) A'' diag(sqrt(2gm/(1+cm))),
// certified by an FP64 Cholesky factorisation of 4I - M^T M.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "rom.hpp"

namespace yr {

namespace {
constexpr int kPBlock = 1024;  // threads of the perturbation kernel
constexpr int kSBlock = 1024;  // threads of the stepping kernel
}  // namespace

// ---------------------------------------------------------------- WG dense FP64

__device__ inline void wg_copy(double* __restrict__ dst, const double* __restrict__ src,
                               int64_t n) {
  for (int64_t g = threadIdx.x; g < n; g += blockDim.x) dst[g] = src[g];
  __syncthreads();
}

__device__ inline void wg_identity(double* __restrict__ A, int n) {
  for (int64_t g = threadIdx.x; g < (int64_t)n * n; g += blockDim.x)
    A[g] = (g % n == g / n) ? 1.0 : 0.0;
  __syncthreads();
}

// in-place lower Cholesky of the n x n column-major A; returns false if not PD
__device__ bool wg_chol(double* __restrict__ A, int n, double* min_pivot) {
  __shared__ int fail;
  __shared__ double minp;
  if (threadIdx.x == 0) {
    fail = 0;
    minp = 1e300;
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      double d = A[j + (int64_t)j * n];
      if (!(d > 0)) fail = 1;
      else {
        minp = fmin(minp, d);
        A[j + (int64_t)j * n] = sqrt(d);
      }
    }
    __syncthreads();
    if (fail) break;
    const double piv = A[j + (int64_t)j * n];
    for (int i = j + 1 + threadIdx.x; i < n; i += blockDim.x) A[i + (int64_t)j * n] /= piv;
    __syncthreads();
    const int m = n - j - 1;
    for (int64_t idx = threadIdx.x; idx < (int64_t)m * m; idx += blockDim.x) {
      int c = j + 1 + (int)(idx / m);
      int r = j + 1 + (int)(idx % m);
      if (r >= c) A[r + (int64_t)c * n] -= A[r + (int64_t)j * n] * A[c + (int64_t)j * n];
    }
    __syncthreads();
  }
  bool ok = !fail;
  if (ok) {  // clear the strict upper triangle
    for (int64_t idx = threadIdx.x; idx < (int64_t)n * n; idx += blockDim.x) {
      int r = (int)(idx % n), c = (int)(idx / n);
      if (r < c) A[idx] = 0;
    }
  }
  if (min_pivot && threadIdx.x == 0) *min_pivot = minp;
  __syncthreads();
  return ok;
}

// Triangular solves in blocks of kTB rows (columns): a block is solved with
// one thread per right-hand side, then removed from the rest of X with every
// thread of the workgroup (a few barriers per block instead of one thread
// walking all n rows of its column).
constexpr int kTB = 16;

// X = L^-1 X   (L n x n lower, X n x m, ldx = n)
__device__ void wg_trsm_left_lower(const double* __restrict__ L, int n, double* __restrict__ X,
                                   int m) {
  for (int b = 0; b < n; b += kTB) {
    const int e = min(n, b + kTB);
    for (int c = threadIdx.x; c < m; c += blockDim.x) {
      double* x = X + (int64_t)c * n;
      for (int i = b; i < e; ++i) {
        double v = x[i];
        for (int k = b; k < i; ++k) v -= L[i + (int64_t)k * n] * x[k];
        x[i] = v / L[i + (int64_t)i * n];
      }
    }
    __syncthreads();
    const int rem = n - e;
    for (int64_t g = threadIdx.x; g < (int64_t)rem * m; g += blockDim.x) {
      const int r = e + (int)(g % rem), c = (int)(g / rem);
      double* x = X + (int64_t)c * n;
      double v = x[r];
      for (int k = b; k < e; ++k) v -= L[r + (int64_t)k * n] * x[k];
      x[r] = v;
    }
    __syncthreads();
  }
}

// X = X L^-T   (X m x n, ldx = m; L n x n lower): columns in blocks of kTB
__device__ void wg_trsm_right_lowerT(const double* __restrict__ L, int n, double* __restrict__ X,
                                     int m) {
  for (int b = 0; b < n; b += kTB) {
    const int e = min(n, b + kTB);
    for (int r = threadIdx.x; r < m; r += blockDim.x) {
      for (int j = b; j < e; ++j) {
        double v = X[r + (int64_t)j * m];
        for (int k = b; k < j; ++k) v -= X[r + (int64_t)k * m] * L[j + (int64_t)k * n];
        X[r + (int64_t)j * m] = v / L[j + (int64_t)j * n];
      }
    }
    __syncthreads();
    const int rem = n - e;
    for (int64_t g = threadIdx.x; g < (int64_t)rem * m; g += blockDim.x) {
      const int r = (int)(g % m), j = e + (int)(g / m);
      double v = X[r + (int64_t)j * m];
      for (int k = b; k < e; ++k) v -= X[r + (int64_t)k * m] * L[j + (int64_t)k * n];
      X[r + (int64_t)j * m] = v;
    }
    __syncthreads();
  }
}

// C (m x n) = op(A) op(B); A is (ta ? k x m : m x k), B is (tb ? n x k : k x n), col-major;
// C must not overlap A or B.  With 1024 threads: 64 x 64 output tiles, 2 x 2
// outputs per thread, operands staged through LDS 16 values of k at a time
// (each output still sums over k in order).
__device__ void wg_gemm(int m, int n, int k, const double* __restrict__ A, bool ta,
                        const double* __restrict__ B, bool tb, double* __restrict__ C) {
  constexpr int TM = 64, TN = 64, TK = 16;
  __shared__ double As[TK][TM + 1], Bs[TK][TN + 1];
  if (blockDim.x != 1024) {
    for (int64_t idx = threadIdx.x; idx < (int64_t)m * n; idx += blockDim.x) {
      int r = (int)(idx % m), c = (int)(idx / m);
      double v = 0;
      for (int q = 0; q < k; ++q) {
        double a = ta ? A[q + (int64_t)r * k] : A[r + (int64_t)q * m];
        double b = tb ? B[c + (int64_t)q * n] : B[q + (int64_t)c * k];
        v += a * b;
      }
      C[idx] = v;
    }
    __syncthreads();
    return;
  }
  const int tid = threadIdx.x;
  const int tr = (tid & 31) * 2, tc = (tid >> 5) * 2;
  // staging slots, arranged so that consecutive threads read consecutive addresses
  const int a_m = ta ? tid / TK : tid % TM, a_k = ta ? tid % TK : tid / TM;
  const int b_n = tb ? tid % TN : tid / TK, b_k = tb ? tid / TN : tid % TK;
  for (int m0 = 0; m0 < m; m0 += TM)
    for (int n0 = 0; n0 < n; n0 += TN) {
      double c00 = 0, c01 = 0, c10 = 0, c11 = 0;
      for (int k0 = 0; k0 < k; k0 += TK) {
        {
          const int r = m0 + a_m, q = k0 + a_k;
          double v = 0;
          if (r < m && q < k) v = ta ? A[q + (int64_t)r * k] : A[r + (int64_t)q * m];
          As[a_k][a_m] = v;
        }
        {
          const int c = n0 + b_n, q = k0 + b_k;
          double v = 0;
          if (c < n && q < k) v = tb ? B[c + (int64_t)q * n] : B[q + (int64_t)c * k];
          Bs[b_k][b_n] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; ++kk) {
          const double a0 = As[kk][tr], a1 = As[kk][tr + 1];
          const double b0 = Bs[kk][tc], b1 = Bs[kk][tc + 1];
          c00 += a0 * b0;
          c01 += a0 * b1;
          c10 += a1 * b0;
          c11 += a1 * b1;
        }
        __syncthreads();
      }
      const int r = m0 + tr, c = n0 + tc;
      if (r < m && c < n) C[r + (int64_t)c * m] = c00;
      if (r < m && c + 1 < n) C[r + (int64_t)(c + 1) * m] = c01;
      if (r + 1 < m && c < n) C[r + 1 + (int64_t)c * m] = c10;
      if (r + 1 < m && c + 1 < n) C[r + 1 + (int64_t)(c + 1) * m] = c11;
    }
  __syncthreads();
}

__device__ inline double wave_sum64(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One-sided Jacobi: rotates the columns of A (m x n) until they are mutually
// orthogonal, accumulating the rotations in V (n x n, initialised by caller).
// Round-robin tournament over column pairs, one wavefront per pair.  A round's
// cost is load latency (A and V live in L2), so a wave takes B of its pairs at
// once: the A and V columns of all B pairs are loaded together (R rows per
// lane, m, n <= 64 R; B R = 8 keeps 64 doubles in registers), their 3B dot
// products reduce side by side, and the rotated columns are stored.  Each
// rotation is decided from lane 0's sums, so every lane applies the same one.
constexpr int kJacRowsMax = 8;  // m, n <= 512
constexpr double kJacTol = 1e-14;  // rotate while |x_p^T x_q| > tol ||x_p|| ||x_q||
constexpr int kJacSweepsMax = 60;

__device__ inline void jac_pair(int rd, int pr, int np, int& p, int& q) {
  if (pr == 0) {
    p = np - 1;
    q = rd;
  } else {
    p = (rd + pr) % (np - 1);
    q = (rd - pr + np - 1) % (np - 1);
  }
}

template <int R, int B>
__device__ __noinline__ void wg_jacobi_r(double* __restrict__ A, int m, int n,
                                                           double* __restrict__ V, double tol,
                                                           int max_sweeps) {
  __shared__ int rotations;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int np = n + (n & 1);  // players (padded to even)
  const int npairs = np / 2;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (threadIdx.x == 0) rotations = 0;
    __syncthreads();
    for (int rd = 0; rd < np - 1; ++rd) {
      for (int base = wid; base < npairs; base += nw * B) {
        int p[B], q[B];
        bool ok[B];
        double x[B][R], y[B][R], u[B][R], w[B][R];
#pragma unroll
        for (int b = 0; b < B; ++b) {
          const int pr = base + b * nw;
          p[b] = q[b] = 0;
          if (pr < npairs) jac_pair(rd, pr, np, p[b], q[b]);
          ok[b] = pr < npairs && p[b] < n && q[b] < n;
          const double* a0 = A + (int64_t)p[b] * m;
          const double* a1 = A + (int64_t)q[b] * m;
          const double* v0 = V + (int64_t)p[b] * n;
          const double* v1 = V + (int64_t)q[b] * n;
#pragma unroll
          for (int t = 0; t < R; ++t) {
            const int i = lane + 64 * t;
            const bool im = ok[b] && i < m, in = ok[b] && i < n;
            x[b][t] = im ? a0[i] : 0.0;
            y[b][t] = im ? a1[i] : 0.0;
            u[b][t] = in ? v0[i] : 0.0;
            w[b][t] = in ? v1[i] : 0.0;
          }
        }
        double al[B], be[B], ga[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
          al[b] = be[b] = ga[b] = 0;
#pragma unroll
          for (int t = 0; t < R; ++t) {
            al[b] += x[b][t] * x[b][t];
            be[b] += y[b][t] * y[b][t];
            ga[b] += x[b][t] * y[b][t];
          }
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
          al[b] = __shfl(wave_sum64(al[b]), 0, 64);
          be[b] = __shfl(wave_sum64(be[b]), 0, 64);
          ga[b] = __shfl(wave_sum64(ga[b]), 0, 64);
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
          if (!ok[b] || ga[b] == 0 || fabs(ga[b]) <= tol * sqrt(al[b] * be[b])) continue;
          const double zeta = (be[b] - al[b]) / (2.0 * ga[b]);
          const double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double c = 1.0 / sqrt(1.0 + tt * tt), sn = c * tt;
          double* a0 = A + (int64_t)p[b] * m;
          double* a1 = A + (int64_t)q[b] * m;
          double* v0 = V + (int64_t)p[b] * n;
          double* v1 = V + (int64_t)q[b] * n;
#pragma unroll
          for (int t = 0; t < R; ++t) {
            const int i = lane + 64 * t;
            if (i < m) {
              a0[i] = c * x[b][t] - sn * y[b][t];
              a1[i] = sn * x[b][t] + c * y[b][t];
            }
            if (i < n) {
              v0[i] = c * u[b][t] - sn * w[b][t];
              v1[i] = sn * u[b][t] + c * w[b][t];
            }
          }
          if (lane == 0) atomicAdd(&rotations, 1);
        }
      }
      __syncthreads();
    }
    if (rotations == 0) break;
    __syncthreads();
  }
  __syncthreads();
}

// Long columns (R = 8): one pair at a time, A's columns first, then V's in
// the same registers.
template <int R>
__device__ __noinline__ void wg_jacobi_seq(double* __restrict__ A, int m, int n,
                                           double* __restrict__ V, double tol, int max_sweeps) {
  __shared__ int rotations;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int np = n + (n & 1);
  const int npairs = np / 2;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (threadIdx.x == 0) rotations = 0;
    __syncthreads();
    for (int rd = 0; rd < np - 1; ++rd) {
      for (int pr = wid; pr < npairs; pr += nw) {
        int p, q;
        jac_pair(rd, pr, np, p, q);
        if (p >= n || q >= n) continue;
        double* a0 = A + (int64_t)p * m;
        double* a1 = A + (int64_t)q * m;
        double x[R], y[R];
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const int i = lane + 64 * t;
          x[t] = i < m ? a0[i] : 0.0;
          y[t] = i < m ? a1[i] : 0.0;
        }
        double al = 0, be = 0, ga = 0;
#pragma unroll
        for (int t = 0; t < R; ++t) {
          al += x[t] * x[t];
          be += y[t] * y[t];
          ga += x[t] * y[t];
        }
        al = __shfl(wave_sum64(al), 0, 64);
        be = __shfl(wave_sum64(be), 0, 64);
        ga = __shfl(wave_sum64(ga), 0, 64);
        if (ga == 0 || fabs(ga) <= tol * sqrt(al * be)) continue;
        const double zeta = (be - al) / (2.0 * ga);
        const double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + tt * tt), sn = c * tt;
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const int i = lane + 64 * t;
          if (i < m) {
            a0[i] = c * x[t] - sn * y[t];
            a1[i] = sn * x[t] + c * y[t];
          }
        }
        double* v0 = V + (int64_t)p * n;
        double* v1 = V + (int64_t)q * n;
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const int i = lane + 64 * t;
          x[t] = i < n ? v0[i] : 0.0;
          y[t] = i < n ? v1[i] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const int i = lane + 64 * t;
          if (i < n) {
            v0[i] = c * x[t] - sn * y[t];
            v1[i] = sn * x[t] + c * y[t];
          }
        }
        if (lane == 0) atomicAdd(&rotations, 1);
      }
      __syncthreads();
    }
    if (rotations == 0) break;
    __syncthreads();
  }
  __syncthreads();
}

__device__ void wg_jacobi(double* __restrict__ A, int m, int n,
                                                         double* __restrict__ V, double tol,
                                                         int max_sweeps) {
  const int len = m > n ? m : n;
  if (len <= 64)
    wg_jacobi_r<1, 2>(A, m, n, V, tol, max_sweeps);
  else if (len <= 128)
    wg_jacobi_r<2, 1>(A, m, n, V, tol, max_sweeps);
  else if (len <= 256)
    wg_jacobi_r<4, 1>(A, m, n, V, tol, max_sweeps);
  else
    wg_jacobi_seq<kJacRowsMax>(A, m, n, V, tol, max_sweeps);
}

// Householder QR in place (m >= n): R in the upper triangle of A, reflector
// k's vector below the diagonal (its k-th entry is 1, not stored), tau[k];
// A = Q R with Q = H_0 H_1 ... H_{n-1}, H_k = I - tau_k v_k v_k^T.
// Wave 0 forms reflector k, then every wave updates its trailing columns.
__device__ void wg_qr(double* __restrict__ A, int m, int n, double* __restrict__ tau) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int k = 0; k < n; ++k) {
    double* a = A + (int64_t)k * m;
    if (wid == 0) {
      double ss = 0;
      for (int i = k + 1 + lane; i < m; i += 64) ss += a[i] * a[i];
      ss = __shfl(wave_sum64(ss), 0, 64);
      const double alpha = a[k];
      double tk = 0, scale = 0;
      if (ss > 0) {
        const double beta = alpha >= 0 ? -sqrt(alpha * alpha + ss) : sqrt(alpha * alpha + ss);
        tk = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
        for (int i = k + 1 + lane; i < m; i += 64) a[i] *= scale;
        if (lane == 0) a[k] = beta;
      }
      if (lane == 0) tau[k] = tk;
    }
    __syncthreads();
    const double tk = tau[k];
    if (tk != 0) {
      for (int j = k + 1 + wid; j < n; j += nw) {
        double* b = A + (int64_t)j * m;
        double d = 0;
        for (int i = k + 1 + lane; i < m; i += 64) d += a[i] * b[i];
        d = __shfl(wave_sum64(d), 0, 64) + b[k];
        const double f = tk * d;
        if (lane == 0) b[k] -= f;
        for (int i = k + 1 + lane; i < m; i += 64) b[i] -= f * a[i];
      }
    }
    __syncthreads();
  }
}

// B (m x nb) <- Q B with Q from wg_qr(A, m, n, tau).  Columns of B are
// independent: each wave keeps its columns in registers (R rows per lane)
// and applies H_{n-1} ... H_0 without barriers.
template <int R>
__device__ void wg_apply_q_r(const double* __restrict__ A, int m, int n,
                             const double* __restrict__ tau, double* __restrict__ B, int nb) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int j = wid; j < nb; j += nw) {
    double* b = B + (int64_t)j * m;
    double x[R];
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int i = lane + 64 * t;
      x[t] = i < m ? b[i] : 0.0;
    }
    for (int k = n - 1; k >= 0; --k) {
      const double tk = tau[k];
      if (tk == 0) continue;
      const double* v = A + (int64_t)k * m;
      double vr[R];
      double d = 0;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int i = lane + 64 * t;
        vr[t] = i > k && i < m ? v[i] : (i == k ? 1.0 : 0.0);
        d += vr[t] * x[t];
      }
      const double f = tk * __shfl(wave_sum64(d), 0, 64);
#pragma unroll
      for (int t = 0; t < R; ++t) x[t] -= f * vr[t];
    }
#pragma unroll
    for (int t = 0; t < R; ++t) {
      const int i = lane + 64 * t;
      if (i < m) b[i] = x[t];
    }
  }
  __syncthreads();
}

__device__ void wg_apply_q(const double* __restrict__ A, int m, int n,
                           const double* __restrict__ tau, double* __restrict__ B, int nb) {
  if (m <= 64)
    wg_apply_q_r<1>(A, m, n, tau, B, nb);
  else if (m <= 128)
    wg_apply_q_r<2>(A, m, n, tau, B, nb);
  else if (m <= 256)
    wg_apply_q_r<4>(A, m, n, tau, B, nb);
  else
    wg_apply_q_r<kJacRowsMax>(A, m, n, tau, B, nb);
}

// X (n x n) = R^T from the upper triangle of the QR factors in A (m x n)
__device__ void wg_rt(const double* __restrict__ A, int m, int n, double* __restrict__ X) {
  for (int64_t g = threadIdx.x; g < (int64_t)n * n; g += blockDim.x) {
    const int i = (int)(g % n), j = (int)(g / n);  // X[i][j] = R[j][i]
    X[g] = j <= i ? A[j + (int64_t)i * m] : 0.0;
  }
  __syncthreads();
}

// column norms of A (m x n) -> out[n]
__device__ void wg_colnorms(const double* __restrict__ A, int m, int n, double* __restrict__ out) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int c = wid; c < n; c += nw) {
    double s = 0;
    for (int i = lane; i < m; i += 64) s += A[i + (int64_t)c * m] * A[i + (int64_t)c * m];
    s = wave_sum64(s);
    if (lane == 0) out[c] = sqrt(s);
  }
  __syncthreads();
}

// X = L^-T X (L lower triangular n x n, X n x m), defined below
__device__ void wg_trsm_left_lowerT(const double* __restrict__ L, int n, double* __restrict__ X,
                                    int m);

// ---------------------------------------------------------------- perturbation kernel

struct PerturbDesc {
  int n1, n2, ns, np;
  int lossy_e, lossy_m;
  double dt, gamma;
  // inputs (device FP64, column-major)
  const double *De, *Dse, *Dm, *Dsm, *K, *B1, *B2, *L1, *L2;
  double* work;  // scratch
  // outputs (FP64)
  double* Kp;     // n1 x n2
  double* sigma;  // n2 (column norms after Jacobi; zero-padded)
  double* A2;     // n1 x n2  Qe^T A' Qm
  double* ce;     // n1
  double* ge;     // n1
  double* cm;     // n2
  double* gm;     // n2
  double* be;     // n1 x ns
  double* bh;     // n2 x ns
  double* oe;     // n1 x np
  double* oh;     // n2 x np
  double* Te;     // n1 x n1  Le^-T Qe (stepping -> reduced coordinates)
  double* Tm;     // n2 x n2  Lm^-T Qm
  int* status;    // 0 ok, 1 De not PD, 2 Dm not PD, 3 loss matrix not PSD
  int* nclamped;
};

__host__ __device__ inline size_t scratch_side(int n1, int n2, int ns, int np) {
  size_t a = (size_t)n1 > (size_t)n2 ? (size_t)n1 : (size_t)n2;
  size_t b = a;
  if ((size_t)ns > b) b = ns;
  if ((size_t)np > b) b = np;
  return a * b;
}

inline size_t perturb_work_doubles(int n1, int n2, int ns, int np) {
  size_t a = (size_t)n1 * n1, b = (size_t)n2 * n2, c = (size_t)n1 * n2;
  size_t mx = scratch_side(n1, n2, ns, np);
  return a + b + 2 * c + b + a + 2 * mx + 2 * ((size_t)n1 + n2) + 64;
}

// Work layout of one model (FP64 scratch), the same in every stage kernel
struct PerturbWork {
  double *Le, *Lm, *A, *V, *Qe, *T, *S1, *S2, *lam, *tau;
};

__host__ __device__ inline PerturbWork perturb_work(double* w, int n1, int n2, int ns, int np) {
  PerturbWork p;
  p.Le = w;
  w += (size_t)n1 * n1;
  p.Lm = w;
  w += (size_t)n2 * n2;
  p.A = w;
  w += (size_t)n1 * n2;
  p.V = w;
  w += (size_t)n2 * n2;
  p.Qe = w;
  w += (size_t)n1 * n1;
  p.T = w;
  w += (size_t)n1 * n2;
  const size_t mx = scratch_side(n1, n2, ns, np);
  p.S1 = w;
  w += mx;
  p.S2 = w;
  w += mx;
  p.lam = w;  // n1 + n2
  w += (size_t)n1 + n2;
  p.tau = w;  // max(n1, n2)
  return p;
}

// S (n x n) = L^-1 D L^-T, symmetrised (L lower triangular)
__device__ void wg_whiten(const double* __restrict__ L, const double* __restrict__ D, int n,
                          double* __restrict__ S) {
  wg_copy(S, D, (int64_t)n * n);
  wg_trsm_left_lower(L, n, S, n);
  wg_trsm_right_lowerT(L, n, S, n);
  for (int64_t g = threadIdx.x; g < (int64_t)n * n; g += blockDim.x) {
    const int r = (int)(g % n), c = (int)(g / n);
    if (r < c) {
      const double m = 0.5 * (S[g] + S[c + (int64_t)r * n]);
      S[g] = m;
      S[c + (int64_t)r * n] = m;
    }
  }
  __syncthreads();
}

// The clamp of Sec. III-A and the loss eigenvectors run in four stage kernels
// (one workgroup per model) around three one-sided Jacobi phases, each phase
// spread over many workgroups (k_bjac_round).  Both use the QR-preconditioned
// form: M = Q R, one-sided Jacobi on X = R^T accumulating W (R^T W = X with
// orthogonal columns), so M = (Q W) S (X S^-1)^T.  The clamped matrix is then
// M' = Q W diag(min(s, lim) / s) X^T (no division by small singular values),
// and for a symmetric positive semidefinite M the eigenvectors are Q W and the
// eigenvalues the column norms of X.  Jacobi on R^T converges in far fewer
// sweeps than on M when the singular values spread over decades.
//
// Stage 1: Cholesky factors, A = Le^-1 K Lm^-T, QR of A (of A^T when n1 < n2,
// whose clamp is the transpose of A's), X = R^T -> S1, W = I -> V.
__global__ void __launch_bounds__(kPBlock) k_perturb_s1(const PerturbDesc* __restrict__ descs) {
  const PerturbDesc d = descs[blockIdx.x];
  const int n1 = d.n1, n2 = d.n2, nsv = n1 < n2 ? n1 : n2;
  const PerturbWork w = perturb_work(d.work, n1, n2, d.ns, d.np);
  if (threadIdx.x == 0) {
    *d.status = 0;
    *d.nclamped = 0;
  }
  wg_copy(w.Le, d.De, (int64_t)n1 * n1);
  if (!wg_chol(w.Le, n1, nullptr)) {
    if (threadIdx.x == 0) *d.status = 1;
    return;
  }
  wg_copy(w.Lm, d.Dm, (int64_t)n2 * n2);
  if (!wg_chol(w.Lm, n2, nullptr)) {
    if (threadIdx.x == 0) *d.status = 2;
    return;
  }
  wg_copy(w.A, d.K, (int64_t)n1 * n2);
  wg_trsm_left_lower(w.Le, n1, w.A, n2);
  wg_trsm_right_lowerT(w.Lm, n2, w.A, n1);
  double* M = w.A;
  if (n1 < n2) {  // M = A^T (n2 x n1) in T
    for (int64_t g = threadIdx.x; g < (int64_t)n1 * n2; g += blockDim.x) {
      const int r = (int)(g % n1), c = (int)(g / n1);
      w.T[c + (int64_t)r * n2] = w.A[g];
    }
    __syncthreads();
    M = w.T;
  }
  const int mrow = n1 > n2 ? n1 : n2;
  wg_qr(M, mrow, nsv, w.tau);
  wg_rt(M, mrow, nsv, w.S1);
  wg_identity(w.V, nsv);
}

// Stage 2: singular values, clamped A' -> T, K~' = Le A' Lm^T; electric loss
// matrix Se = Le^-1 Dse Le^-T: QR, X -> S2, W = I -> Qe.
__global__ void __launch_bounds__(kPBlock) k_perturb_s2(const PerturbDesc* __restrict__ descs) {
  const PerturbDesc d = descs[blockIdx.x];
  if (*d.status != 0) return;
  const int n1 = d.n1, n2 = d.n2, nsv = n1 < n2 ? n1 : n2;
  const PerturbWork w = perturb_work(d.work, n1, n2, d.ns, d.np);
  const double lim = d.gamma * 2.0 / d.dt;
  const int mrow = n1 > n2 ? n1 : n2;
  wg_colnorms(w.S1, nsv, nsv, d.sigma);
  for (int i = nsv + threadIdx.x; i < n2; i += blockDim.x) d.sigma[i] = 0.0;
  for (int64_t g = threadIdx.x; g < (int64_t)nsv * nsv; g += blockDim.x) {
    const double sv = d.sigma[g / nsv];
    if (sv >= lim) w.V[g] *= lim / sv;
  }
  __syncthreads();
  wg_gemm(nsv, nsv, nsv, w.V, false, w.S1, true, w.S2);  // Z = W D X^T
  // Mc = Q [Z; 0]: into T (n1 >= n2) or into A, then transposed into T
  double* Mc = n1 >= n2 ? w.T : w.A;
  const double* Mq = n1 >= n2 ? w.A : w.T;
  for (int64_t g = threadIdx.x; g < (int64_t)mrow * nsv; g += blockDim.x) {
    const int r = (int)(g % mrow), c = (int)(g / mrow);
    Mc[g] = r < nsv ? w.S2[r + (int64_t)c * nsv] : 0.0;
  }
  __syncthreads();
  wg_apply_q(Mq, mrow, nsv, w.tau, Mc, nsv);
  if (n1 < n2) {
    for (int64_t g = threadIdx.x; g < (int64_t)n1 * n2; g += blockDim.x) {
      const int r = (int)(g % n1), c = (int)(g / n1);
      w.T[g] = w.A[c + (int64_t)r * n2];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int cnt = 0;
    for (int i = 0; i < nsv; ++i) cnt += d.sigma[i] >= lim;
    *d.nclamped = cnt;
  }
  wg_gemm(n1, n2, n1, w.Le, false, w.T, false, w.A);
  wg_gemm(n1, n2, n2, w.A, false, w.Lm, true, d.Kp);
  if (d.lossy_e) {
    wg_whiten(w.Le, d.Dse, n1, w.S1);
    wg_qr(w.S1, n1, n1, w.tau);
    wg_rt(w.S1, n1, n1, w.S2);
  }
  wg_identity(w.Qe, n1);
}

// Stage 3: electric eigenvalues and eigenvectors Qe = Q W; magnetic loss
// matrix Sm = Lm^-1 Dsm Lm^-T: QR, X -> S1, W = I -> V (Qm).
__global__ void __launch_bounds__(kPBlock) k_perturb_s3(const PerturbDesc* __restrict__ descs) {
  const PerturbDesc d = descs[blockIdx.x];
  if (*d.status != 0) return;
  const int n1 = d.n1, n2 = d.n2;
  const PerturbWork w = perturb_work(d.work, n1, n2, d.ns, d.np);
  if (d.lossy_e) {
    wg_colnorms(w.S2, n1, n1, w.lam);
    wg_apply_q(w.S1, n1, n1, w.tau, w.Qe, n1);
  } else {
    for (int i = threadIdx.x; i < n1; i += blockDim.x) w.lam[i] = 0;
  }
  if (d.lossy_m) {
    wg_whiten(w.Lm, d.Dsm, n2, w.S2);
    wg_qr(w.S2, n2, n2, w.tau);
    wg_rt(w.S2, n2, n2, w.S1);
  }
  wg_identity(w.V, n2);
}

// Stage 4: magnetic eigenvalues and Qm = Q W, then the stepping matrices.
__global__ void __launch_bounds__(kPBlock) k_perturb_s4(const PerturbDesc* __restrict__ descs) {
  const PerturbDesc d = descs[blockIdx.x];
  if (*d.status != 0) return;
  const int n1 = d.n1, n2 = d.n2;
  const PerturbWork w = perturb_work(d.work, n1, n2, d.ns, d.np);
  double* Qm = w.V;
  double* lam_m = w.lam + n1;
  if (d.lossy_m) {
    wg_colnorms(w.S1, n2, n2, lam_m);
    wg_apply_q(w.S2, n2, n2, w.tau, Qm, n2);
  } else {
    for (int i = threadIdx.x; i < n2; i += blockDim.x) lam_m[i] = 0;
    __syncthreads();
  }
  // A'' = Qe^T A' Qm   (A' is in T)
  wg_gemm(n1, n2, n1, w.Qe, true, w.T, false, w.A);
  wg_gemm(n1, n2, n2, w.A, false, Qm, false, d.A2);
  // sources and outputs: be = Qe^T Le^-1 B1, oe = Qe^T Le^-1 L1, ...
  if (d.ns) {
    wg_copy(w.S1, d.B1, (int64_t)n1 * d.ns);
    wg_trsm_left_lower(w.Le, n1, w.S1, d.ns);
    wg_gemm(n1, d.ns, n1, w.Qe, true, w.S1, false, d.be);
    wg_copy(w.S2, d.B2, (int64_t)n2 * d.ns);
    wg_trsm_left_lower(w.Lm, n2, w.S2, d.ns);
    wg_gemm(n2, d.ns, n2, Qm, true, w.S2, false, d.bh);
  }
  if (d.np) {
    wg_copy(w.S1, d.L1, (int64_t)n1 * d.np);
    wg_trsm_left_lower(w.Le, n1, w.S1, d.np);
    wg_gemm(n1, d.np, n1, w.Qe, true, w.S1, false, d.oe);
    wg_copy(w.S2, d.L2, (int64_t)n2 * d.np);
    wg_trsm_left_lower(w.Lm, n2, w.S2, d.np);
    wg_gemm(n2, d.np, n2, Qm, true, w.S2, false, d.oh);
  }
  // back-transforms of the stepping state: e~ = Le^-T Qe s_e, h~ = Lm^-T Qm s_h
  wg_copy(d.Te, w.Qe, (int64_t)n1 * n1);
  wg_trsm_left_lowerT(w.Le, n1, d.Te, n1);
  wg_copy(d.Tm, Qm, (int64_t)n2 * n2);
  wg_trsm_left_lowerT(w.Lm, n2, d.Tm, n2);
  // diagonal leapfrog coefficients in the whitened, rotated coordinates
  for (int i = threadIdx.x; i < n1 + n2; i += blockDim.x) {
    const double l = w.lam[i];
    const double p = 1.0 / d.dt + 0.5 * l, m = 1.0 / d.dt - 0.5 * l;
    if (i < n1) {
      d.ce[i] = m / p;
      d.ge[i] = 1.0 / p;
    } else {
      d.cm[i - n1] = m / p;
      d.gm[i - n1] = 1.0 / p;
    }
  }
}

// ---------------------------------------------------------------- block Jacobi

// One-sided Jacobi on X (n x n) accumulating W (n x n), over many workgroups:
// the columns form nblk blocks of bs (nblk even); a round-robin tournament
// over the blocks gives nblk - 1 rounds per sweep, and in a round each of the
// nblk / 2 workgroups of a matrix takes one block pair, holds its columns of X
// and W in LDS and rotates every column pair of the two blocks once (an inner
// round-robin sweep, one wavefront per pair).  The launch boundary between
// rounds is the only global barrier.  A sweep without a rotation above the
// tolerance ends that matrix's iteration.
struct JacDesc {
  double* X;
  double* W;
  int n, bs, nblk;
  int wg0;            // first workgroup of this matrix in a round's grid
  int* rot;           // rotations in the current sweep
  int* active;        // 1 until a sweep without rotations
  const int* status;  // the model's status (nonzero: nothing to do)
};

constexpr int kBjacLds = 4096;  // bs * n <= kBjacLds: a pair's X and W columns take 128 KB

template <int R>
__device__ void bjac_inner(double* __restrict__ Xs, double* __restrict__ Ws, int n, int nc,
                           double tol, int* cnt) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int np = nc + (nc & 1);
  for (int rd = 0; rd < np - 1; ++rd) {
    for (int pr = wid; pr < np / 2; pr += nw) {
      int p, q;
      jac_pair(rd, pr, np, p, q);
      if (p >= nc || q >= nc) continue;
      double* a0 = Xs + (int64_t)p * n;
      double* a1 = Xs + (int64_t)q * n;
      double x[R], y[R];
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int i = lane + 64 * t;
        x[t] = i < n ? a0[i] : 0.0;
        y[t] = i < n ? a1[i] : 0.0;
      }
      double al = 0, be = 0, ga = 0;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        al += x[t] * x[t];
        be += y[t] * y[t];
        ga += x[t] * y[t];
      }
      al = __shfl(wave_sum64(al), 0, 64);
      be = __shfl(wave_sum64(be), 0, 64);
      ga = __shfl(wave_sum64(ga), 0, 64);
      if (ga == 0 || fabs(ga) <= tol * sqrt(al * be)) continue;
      const double zeta = (be - al) / (2.0 * ga);
      const double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
      const double c = 1.0 / sqrt(1.0 + tt * tt), sn = c * tt;
      double* v0 = Ws + (int64_t)p * n;
      double* v1 = Ws + (int64_t)q * n;
#pragma unroll
      for (int t = 0; t < R; ++t) {
        const int i = lane + 64 * t;
        if (i < n) {
          a0[i] = c * x[t] - sn * y[t];
          a1[i] = sn * x[t] + c * y[t];
          const double u = v0[i], v = v1[i];
          v0[i] = c * u - sn * v;
          v1[i] = sn * u + c * v;
        }
      }
      if (lane == 0) atomicAdd(cnt, 1);
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(1024)
    k_bjac_round(const JacDesc* __restrict__ jd, const int* __restrict__ wg_desc, int round,
                 double tol) {
  __shared__ double lds[4 * kBjacLds];  // X then W, 2 bs columns of n each
  __shared__ int cnt;
  const JacDesc d = jd[wg_desc[blockIdx.x]];
  if (*d.status != 0 || *d.active == 0 || round >= d.nblk - 1) return;
  int I, J;
  jac_pair(round, (int)blockIdx.x - d.wg0, d.nblk, I, J);
  const int n = d.n, bs = d.bs;
  const int i0 = I * bs, j0 = J * bs;
  const int cI = max(0, min(bs, n - i0)), cJ = max(0, min(bs, n - j0));
  const int nc = cI + cJ;
  if (nc < 2) return;
  double* Xs = lds;
  double* Ws = lds + 2 * kBjacLds;
  for (int64_t g = threadIdx.x; g < (int64_t)nc * n; g += blockDim.x) {
    const int c = (int)(g / n), r = (int)(g % n);
    const int64_t col = c < cI ? i0 + c : j0 + (c - cI);
    Xs[g] = d.X[col * n + r];
    Ws[g] = d.W[col * n + r];
  }
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  if (n <= 64)
    bjac_inner<1>(Xs, Ws, n, nc, tol, &cnt);
  else if (n <= 128)
    bjac_inner<2>(Xs, Ws, n, nc, tol, &cnt);
  else if (n <= 256)
    bjac_inner<4>(Xs, Ws, n, nc, tol, &cnt);
  else
    bjac_inner<kJacRowsMax>(Xs, Ws, n, nc, tol, &cnt);
  for (int64_t g = threadIdx.x; g < (int64_t)nc * n; g += blockDim.x) {
    const int c = (int)(g / n), r = (int)(g % n);
    const int64_t col = c < cI ? i0 + c : j0 + (c - cI);
    d.X[col * n + r] = Xs[g];
    d.W[col * n + r] = Ws[g];
  }
  if (threadIdx.x == 0 && cnt > 0) atomicAdd(d.rot, cnt);
}

// end of a sweep: a matrix stays active while its sweep rotated something
__global__ void k_bjac_check(const JacDesc* __restrict__ jd, int nd) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nd; i += gridDim.x * blockDim.x) {
    const JacDesc d = jd[i];
    if (*d.active && *d.rot == 0) *d.active = 0;
    *d.rot = 0;
  }
}

// ---------------------------------------------------------------- rounding + guard

template <typename T>
__global__ void k_round(const double* __restrict__ src, T* __restrict__ dst, int64_t n,
                        int transpose_rows, int transpose_cols) {
  // transpose: src col-major (rows x cols) -> dst row-major
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= n) return;
  if (transpose_rows > 0) {
    int64_t r = g % transpose_rows, c = g / transpose_rows;
    dst[r * transpose_cols + c] = (T)src[g];
  } else {
    dst[g] = (T)src[g];
  }
}

// src col-major FP64 (rows x cols) -> dst row-major (rows x ld, zero padded),
// or its transpose (cols x ld) when `transpose` is set
template <typename T>
__global__ void k_round_rows(const double* __restrict__ src, int rows, int cols,
                             T* __restrict__ dst, int ld, int transpose) {
  const int orows = transpose ? cols : rows, ocols = transpose ? rows : cols;
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= (int64_t)orows * ld) return;
  const int r = (int)(g / ld), c = (int)(g % ld);
  T v = 0;
  if (c < ocols) v = (T)(transpose ? src[c + (int64_t)r * rows] : src[r + (int64_t)c * rows]);
  dst[g] = v;
}

struct GuardDesc {
  int n1, n2, lda;
  const void* A;    // stepping dtype, row-major n1 x n2
  const void* vec;  // stepping dtype: ce, ge, cm, gm
  double* work;     // n2*n2 + n1*n2
  double* out;      // [0] = certificate (min pivot of 4I - M^T M, <= 0 if it failed)
  int f64;
};

__global__ void __launch_bounds__(kPBlock) k_guard(const GuardDesc* __restrict__ descs) {
  const GuardDesc d = descs[blockIdx.x];
  const int n1 = d.n1, n2 = d.n2;
  double* M = d.work;               // n1 x n2 col-major
  double* G = d.work + (size_t)n1 * n2;  // n2 x n2
  auto ld = [&](const void* p, int64_t i) -> double {
    return d.f64 ? ((const double*)p)[i] : (double)((const float*)p)[i];
  };
  __shared__ int bad;
  if (threadIdx.x == 0) bad = 0;
  __syncthreads();
  for (int64_t g = threadIdx.x; g < (int64_t)n1 * n2; g += blockDim.x) {
    int r = (int)(g % n1), c = (int)(g / n1);
    double ce = ld(d.vec, r), ge = ld(d.vec, n1 + r);
    double cm = ld(d.vec, 2 * n1 + c), gm = ld(d.vec, 2 * n1 + n2 + c);
    if (!(ce <= 1.0 && ce > -1.0 && cm <= 1.0 && cm > -1.0 && ge > 0 && gm > 0)) bad = 1;
    double a = ld(d.A, (int64_t)r * d.lda + c);
    M[g] = sqrt(2.0 * ge / (1.0 + ce)) * a * sqrt(2.0 * gm / (1.0 + cm));
  }
  __syncthreads();
  wg_gemm(n2, n2, n1, M, true, M, false, G);
  for (int64_t g = threadIdx.x; g < (int64_t)n2 * n2; g += blockDim.x) {
    int r = (int)(g % n2), c = (int)(g / n2);
    G[g] = (r == c ? 4.0 : 0.0) - G[g];
  }
  __syncthreads();
  __shared__ double mp;
  bool ok = wg_chol(G, n2, &mp);
  if (threadIdx.x == 0) d.out[0] = (ok && !bad) ? mp : -1.0;
}

// ---------------------------------------------------------------- stepping kernel

struct StepDesc {
  int n1, n2, ns, np, lda, ldat;
  const void* A;    // row-major n1 x lda (dtype)
  const void* AT;   // row-major n2 x ldat, A transposed
  const void* vec;  // ce ge cm gm be bh oe oh (dtype)
  const void* u;    // [nsteps][ns]
  void* y;          // [nsteps][np]
  void* state;      // [n1 + n2] in/out, may be null
};

template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  using type = float4;
  static constexpr int W = 4;
  static __device__ void get(const type& v, float* o) {
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  }
};
template <>
struct Vec16<double> {
  using type = double2;
  static constexpr int W = 2;
  static __device__ void get(const type& v, double* o) {
    o[0] = v.x;
    o[1] = v.y;
  }
};

// Partial sums of out[c] = sum_r M[r ld + c] v[r] (c < nc, r < nr) into
// red[ty][c]: thread (tx, ty) owns the W columns W tx .. W tx + W-1 and the
// rows r = ty, ty + NY, ...; each row of M is read once, as 16-byte vectors
// coalesced across tx, four rows in flight per thread.  Products and sums are
// formed in FP64 whatever the storage type T of M and v.  Returns NY.
template <typename T>
__device__ inline int mv_partial(const T* __restrict__ M, int ld, int nr, int nc,
                                 const T* __restrict__ v, double* __restrict__ red) {
  using V = Vec16<T>;
  constexpr int W = V::W;
  const int nq = (nc + W - 1) / W;
  if (nq == 0) return 0;
  const int NY = blockDim.x / nq;
  const int tx = threadIdx.x % nq, ty = threadIdx.x / nq;
  if (ty < NY) {
    double acc[W];
#pragma unroll
    for (int k = 0; k < W; ++k) acc[k] = 0;
    const typename V::type* Mv = reinterpret_cast<const typename V::type*>(M) + tx;
    const int ldv = ld / W;
    int r = ty;
    for (; r + 3 * NY < nr; r += 4 * NY) {
      typename V::type a0 = Mv[(int64_t)r * ldv], a1 = Mv[(int64_t)(r + NY) * ldv],
                       a2 = Mv[(int64_t)(r + 2 * NY) * ldv], a3 = Mv[(int64_t)(r + 3 * NY) * ldv];
      T x[4][W];
      V::get(a0, x[0]);
      V::get(a1, x[1]);
      V::get(a2, x[2]);
      V::get(a3, x[3]);
      const double v0 = v[r], v1 = v[r + NY], v2 = v[r + 2 * NY], v3 = v[r + 3 * NY];
#pragma unroll
      for (int k = 0; k < W; ++k)
        acc[k] += (double)x[0][k] * v0 + (double)x[1][k] * v1 + (double)x[2][k] * v2 +
                  (double)x[3][k] * v3;
    }
    for (; r < nr; r += NY) {
      T x[W];
      V::get(Mv[(int64_t)r * ldv], x);
      const double vr = v[r];
#pragma unroll
      for (int k = 0; k < W; ++k) acc[k] += (double)x[k] * vr;
    }
#pragma unroll
    for (int k = 0; k < W; ++k) red[ty * nq * W + tx * W + k] = acc[k];
  }
  return NY;
}

// One workgroup per model.  Per step (lossy form, rotated coordinates):
//   e = ce e - ge (A h) + ge (be u);  h = cm h + gm (A^T e) + gm (bh u);
//   y = oe^T e + oh^T h.
// A h is formed from A^T's rows and A^T e from A's rows, so both products
// stream a row-major matrix with the same coalesced pattern.  Matrices and
// the state are stored in T; every product, sum and update is formed in FP64
// and rounded to T once (with FP32 storage the rounding of the stored values
// is then the only FP32 error: long FP32 sums of large terms that cancel to a
// small result lose several digits more).
template <typename T, int NT>
__global__ void __launch_bounds__(NT) k_rom_step(const StepDesc* __restrict__ descs,
                                                 int64_t nsteps, int qmax) {
  extern __shared__ unsigned char smem_raw[];
  double* red = reinterpret_cast<double*>(smem_raw);  // [NT * W]
  T* e = reinterpret_cast<T*>(smem_raw + (size_t)NT * Vec16<T>::W * sizeof(double));
  T* h = e + qmax;
  const StepDesc d = descs[blockIdx.x];
  const int n1 = d.n1, n2 = d.n2, ns = d.ns, np = d.np;
  const T* A = (const T*)d.A;
  const T* AT = (const T*)d.AT;
  const T* v = (const T*)d.vec;
  const T* ce = v;
  const T* ge = v + n1;
  const T* cm = v + 2 * n1;
  const T* gm = v + 2 * n1 + n2;
  const T* be = v + 2 * n1 + 2 * n2;
  const T* bh = be + (int64_t)n1 * ns;
  const T* oe = bh + (int64_t)n2 * ns;
  const T* oh = oe + (int64_t)n1 * np;
  const T* u = (const T*)d.u;
  T* y = (T*)d.y;
  T* st = (T*)d.state;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int i = threadIdx.x; i < n1 + n2; i += blockDim.x) {
    T val = st ? st[i] : (T)0;
    if (i < n1) e[i] = val;
    else h[i - n1] = val;
  }
  __syncthreads();
  for (int64_t n = 0; n < nsteps; ++n) {
    const T* un = u ? u + n * ns : nullptr;
    // electric half-step
    int NY = mv_partial<T>(AT, d.ldat, n2, n1, h, red);
    __syncthreads();
    {
      const int ld = ((n1 + Vec16<T>::W - 1) / Vec16<T>::W) * Vec16<T>::W;
      for (int i = threadIdx.x; i < n1; i += blockDim.x) {
        double acc = 0;
        for (int t = 0; t < NY; ++t) acc += red[t * ld + i];
        double src = 0;
        for (int p = 0; p < ns; ++p) src += (double)be[i + (int64_t)p * n1] * (double)un[p];
        const double g = ge[i];
        e[i] = (T)((double)ce[i] * (double)e[i] - g * acc + g * src);
      }
    }
    __syncthreads();
    // magnetic half-step
    NY = mv_partial<T>(A, d.lda, n1, n2, e, red);
    __syncthreads();
    {
      const int ld = ((n2 + Vec16<T>::W - 1) / Vec16<T>::W) * Vec16<T>::W;
      for (int j = threadIdx.x; j < n2; j += blockDim.x) {
        double acc = 0;
        for (int t = 0; t < NY; ++t) acc += red[t * ld + j];
        double src = 0;
        for (int p = 0; p < ns; ++p) src += (double)bh[j + (int64_t)p * n2] * (double)un[p];
        const double g = gm[j];
        h[j] = (T)((double)cm[j] * (double)h[j] + g * acc + g * src);
      }
    }
    __syncthreads();
    // outputs y = oe^T e + oh^T h (read only: the next step's first barrier
    // orders them before e changes)
    for (int p = wid; p < np; p += nw) {
      double acc = 0;
      for (int i = lane; i < n1; i += 64) acc += (double)oe[i + (int64_t)p * n1] * (double)e[i];
      for (int j = lane; j < n2; j += 64) acc += (double)oh[j + (int64_t)p * n2] * (double)h[j];
      for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
      if (lane == 0) y[n * np + p] = (T)acc;
    }
  }
  __syncthreads();
  if (st)
    for (int i = threadIdx.x; i < n1 + n2; i += blockDim.x) st[i] = i < n1 ? e[i] : h[i - n1];
}
// ---------------------------------------------------------------- reduced adjoint

// X = L^-T X   (L n x n lower, X n x m): back substitution in blocks of kTB
// rows from the bottom
__device__ void wg_trsm_left_lowerT(const double* __restrict__ L, int n, double* __restrict__ X,
                                    int m) {
  for (int e = n; e > 0; e -= kTB) {
    const int b = e - kTB > 0 ? e - kTB : 0;
    for (int c = threadIdx.x; c < m; c += blockDim.x) {
      double* x = X + (int64_t)c * n;
      for (int i = e - 1; i >= b; --i) {
        double v = x[i];
        for (int k = i + 1; k < e; ++k) v -= L[k + (int64_t)i * n] * x[k];
        x[i] = v / L[i + (int64_t)i * n];
      }
    }
    __syncthreads();
    for (int64_t g = threadIdx.x; g < (int64_t)b * m; g += blockDim.x) {
      const int r = (int)(g % b), c = (int)(g / b);
      double* x = X + (int64_t)c * n;
      double v = x[r];
      for (int k = b; k < e; ++k) v -= L[k + (int64_t)r * n] * x[k];
      x[r] = v;
    }
    __syncthreads();
  }
}

// X = P^-1 X with P = L L^T (Cholesky factor L)
__device__ inline void wg_chol_solve(const double* L, int n, double* X, int m) {
  wg_trsm_left_lower(L, n, X, m);
  wg_trsm_left_lowerT(L, n, X, m);
}

__device__ inline double wg_dot(const double* a, const double* b, int64_t n, double* red) {
  double s = 0;
  for (int64_t g = threadIdx.x; g < n; g += blockDim.x) s += a[g] * b[g];
  s = wave_sum64(s);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = s;
  __syncthreads();
  double t = 0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
  __syncthreads();
  return t;
}

struct AdjDesc {
  int n1, n2, ns, np;
  int64_t nsteps;
  double dt, gamma;
  int through_clamp;
  const double *De, *Dse, *Dm, *Dsm, *K, *B1, *B2, *L1, *L2;  // reduced matrices
  const double* u;     // [nsteps][ns]
  const double* dJdy;  // [nsteps][np]
  const double* dDe;   // n1 x n1 direction (may be null)
  double* work;
  double* gDe;  // n1 x n1
  double* gDse;
  double* gK;   // n1 x n2
  double* Kp;   // n1 x n2
  double* out;  // [0] J, [1] dJ (frozen clamp), [2] dJ (through the clamp), [3] status
};

inline size_t adj_work_doubles(int n1, int n2, int ns, int np, int64_t N) {
  size_t a = (size_t)n1 * n1, b = (size_t)n2 * n2, c = (size_t)n1 * n2;
  size_t side = scratch_side(n1, n2, ns, np);
  return 3 * a + 3 * b + 5 * c + (a > b ? a : b) + 4 * side + 2 * (size_t)(N + 1) * (n1 + n2) +
         4 * (n1 + n2) + 64;
}

__global__ void __launch_bounds__(kPBlock) k_rom_adjoint(const AdjDesc* __restrict__ descs) {
  const AdjDesc d = descs[blockIdx.x];
  const int n1 = d.n1, n2 = d.n2, ns = d.ns, np = d.np;
  const int64_t N = d.nsteps;
  const double dt = d.dt;
  __shared__ double red[kPBlock / 64];
  double* w = d.work;
  auto take = [&](size_t n) { double* p = w; w += n; return p; };
  double* Le = take((size_t)n1 * n1);
  double* Lp = take((size_t)n1 * n1);
  double* Ae = take((size_t)n1 * n1);
  double* Lm = take((size_t)n2 * n2);
  double* Lq = take((size_t)n2 * n2);
  double* Ah = take((size_t)n2 * n2);
  double* A0 = take((size_t)n1 * n2);
  double* A = take((size_t)n1 * n2);
  double* Ap = take((size_t)n1 * n2);
  double* Ke = take((size_t)n1 * n2);
  double* Kh = take((size_t)n1 * n2);  // n2 x n1
  double* V = take((size_t)n2 * n2 > (size_t)n1 * n1 ? (size_t)n2 * n2 : (size_t)n1 * n1);
  const size_t side = scratch_side(n1, n2, ns, np);
  double* be = take(side);
  double* bh = take(side);
  double* le = take(side);
  double* lh = take(side);
  double* X = take((size_t)(N + 1) * (n1 + n2));   // states x~^0..x~^N
  double* Lam = take((size_t)(N + 1) * (n1 + n2)); // adjoints, row n = lambda^n
  double* sig = take(n1 + n2);
  double* cur = take(2 * (n1 + n2));
  __syncthreads();
  // 1. clamp of Sec. III-A (Cholesky route), keeping U S, W and A0
  wg_copy(Le, d.De, (int64_t)n1 * n1);
  if (!wg_chol(Le, n1, nullptr)) {
    if (threadIdx.x == 0) d.out[3] = 1;
    return;
  }
  wg_copy(Lm, d.Dm, (int64_t)n2 * n2);
  if (!wg_chol(Lm, n2, nullptr)) {
    if (threadIdx.x == 0) d.out[3] = 2;
    return;
  }
  wg_copy(A0, d.K, (int64_t)n1 * n2);
  wg_trsm_left_lower(Le, n1, A0, n2);
  wg_trsm_right_lowerT(Lm, n2, A0, n1);
  wg_copy(A, A0, (int64_t)n1 * n2);
  wg_identity(V, n2);
  wg_jacobi(A, n1, n2, V, 1e-14, 60);
  wg_colnorms(A, n1, n2, sig);
  const double lim = d.gamma * 2.0 / dt;
  // Ap = (U min(S, lim)) W^T
  for (int64_t g = threadIdx.x; g < (int64_t)n1 * n2; g += blockDim.x) {
    int c = (int)(g / n1);
    double s = sig[c];
    Ke[g] = s >= lim ? A[g] * (lim / s) : A[g];  // Ke as scratch
  }
  __syncthreads();
  wg_gemm(n1, n2, n2, Ke, false, V, true, Ap);
  wg_gemm(n1, n2, n1, Le, false, Ap, false, Ke);
  wg_gemm(n1, n2, n2, Ke, false, Lm, true, d.Kp);
  // 2. leapfrog maps in the reduced coordinates: Pe = De/dt + Dse/2, Me = De/dt - Dse/2
  for (int64_t g = threadIdx.x; g < (int64_t)n1 * n1; g += blockDim.x) {
    Lp[g] = d.De[g] / dt + 0.5 * d.Dse[g];
    Ae[g] = d.De[g] / dt - 0.5 * d.Dse[g];
  }
  for (int64_t g = threadIdx.x; g < (int64_t)n2 * n2; g += blockDim.x) {
    Lq[g] = d.Dm[g] / dt + 0.5 * d.Dsm[g];
    Ah[g] = d.Dm[g] / dt - 0.5 * d.Dsm[g];
  }
  __syncthreads();
  if (!wg_chol(Lp, n1, nullptr) || !wg_chol(Lq, n2, nullptr)) {
    if (threadIdx.x == 0) d.out[3] = 3;
    return;
  }
  wg_chol_solve(Lp, n1, Ae, n1);                 // Ae = Pe^-1 Me
  wg_copy(Ke, d.Kp, (int64_t)n1 * n2);
  wg_chol_solve(Lp, n1, Ke, n2);                 // Ke = Pe^-1 K'
  wg_chol_solve(Lq, n2, Ah, n2);                 // Ah = Pm^-1 Mm
  for (int64_t g = threadIdx.x; g < (int64_t)n1 * n2; g += blockDim.x) {  // Kh = K'^T (n2 x n1)
    int r = (int)(g % n1), c = (int)(g / n1);
    Kh[c + (int64_t)r * n2] = d.Kp[g];
  }
  __syncthreads();
  wg_chol_solve(Lq, n2, Kh, n1);                 // Kh = Pm^-1 K'^T
  wg_copy(be, d.B1, (int64_t)n1 * ns);
  wg_chol_solve(Lp, n1, be, ns);
  wg_copy(bh, d.B2, (int64_t)n2 * ns);
  wg_chol_solve(Lq, n2, bh, ns);
  wg_copy(le, d.L1, (int64_t)n1 * np);
  wg_chol_solve(Lp, n1, le, np);
  wg_copy(lh, d.L2, (int64_t)n2 * np);
  wg_chol_solve(Lq, n2, lh, np);
  // 3. forward sweep of eq. (reducedMNAform), states stored
  const int q = n1 + n2;
  for (int g = threadIdx.x; g < q; g += blockDim.x) X[g] = 0;
  __syncthreads();
  double Jloc = 0;
  for (int64_t n = 0; n < N; ++n) {
    const double* xo = X + n * q;
    double* xn = X + (n + 1) * q;
    const double* un = d.u + n * ns;
    for (int i = threadIdx.x; i < n1; i += blockDim.x) {
      double v = 0;
      for (int j = 0; j < n1; ++j) v += Ae[i + (int64_t)j * n1] * xo[j];
      for (int j = 0; j < n2; ++j) v -= Ke[i + (int64_t)j * n1] * xo[n1 + j];
      for (int p = 0; p < ns; ++p) v += be[i + (int64_t)p * n1] * un[p];
      xn[i] = v;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n2; i += blockDim.x) {
      double v = 0;
      for (int j = 0; j < n2; ++j) v += Ah[i + (int64_t)j * n2] * xo[n1 + j];
      for (int j = 0; j < n1; ++j) v += Kh[i + (int64_t)j * n2] * xn[j];
      for (int p = 0; p < ns; ++p) v += bh[i + (int64_t)p * n2] * un[p];
      xn[n1 + i] = v;
    }
    __syncthreads();
    for (int p = 0; p < np; ++p) {
      double y = wg_dot(d.L1 + (int64_t)p * n1, xn, n1, red) + wg_dot(d.L2 + (int64_t)p * n2, xn + n1, n2, red);
      Jloc += dt * y * y;
    }
  }
  // 4. adjoint sweep: magnetic rows first, then electric rows
  for (int g = threadIdx.x; g < q; g += blockDim.x) Lam[N * q + g] = 0;  // scratch row
  for (int g = threadIdx.x; g < 2 * q; g += blockDim.x) cur[g] = 0;
  __syncthreads();
  double* la = cur;       // lambda^{n+1}
  double* lb = cur + q;   // lambda^n
  for (int64_t n = N; n >= 1; --n) {
    const double* gy = d.dJdy + (n - 1) * np;
    for (int i = threadIdx.x; i < n2; i += blockDim.x) {
      double v = 0;
      for (int j = 0; j < n2; ++j) v += Ah[i + (int64_t)j * n2] * la[n1 + j];
      for (int j = 0; j < n1; ++j) v -= Kh[i + (int64_t)j * n2] * la[j];
      for (int p = 0; p < np; ++p) v += lh[i + (int64_t)p * n2] * gy[p];
      lb[n1 + i] = v;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n1; i += blockDim.x) {
      double v = 0;
      for (int j = 0; j < n1; ++j) v += Ae[i + (int64_t)j * n1] * la[j];
      for (int j = 0; j < n2; ++j) v += Ke[i + (int64_t)j * n1] * lb[n1 + j];
      for (int p = 0; p < np; ++p) v += le[i + (int64_t)p * n1] * gy[p];
      lb[i] = v;
    }
    __syncthreads();
    for (int g = threadIdx.x; g < q; g += blockDim.x) {
      Lam[(n - 1) * q + g] = lb[g];  // row n-1 holds lambda^n
      la[g] = lb[g];
    }
    __syncthreads();
  }
  // 5. gradients: sums over n of outer products (lambda^n rows, state rows)
  for (int64_t g = threadIdx.x; g < (int64_t)n1 * n1; g += blockDim.x) {
    int a = (int)(g % n1), b = (int)(g / n1);
    double se = 0, ss = 0;
    for (int64_t n = 1; n <= N; ++n) {
      double l = Lam[(n - 1) * q + a];
      double en = X[n * q + b], ep = X[(n - 1) * q + b];
      se += l * (en - ep);
      ss += l * (en + ep);
    }
    d.gDe[g] = -se / dt;
    d.gDse[g] = -0.5 * ss;
  }
  for (int64_t g = threadIdx.x; g < (int64_t)n1 * n2; g += blockDim.x) {
    int a = (int)(g % n1), b = (int)(g / n1);
    double sk = 0;
    for (int64_t n = 1; n <= N; ++n)
      sk += -Lam[(n - 1) * q + a] * X[(n - 1) * q + n1 + b] + X[n * q + a] * Lam[(n - 1) * q + n1 + b];
    d.gK[g] = sk;
  }
  __syncthreads();
  double dJf = 0, dJc = 0;
  if (d.dDe) {
    dJf = wg_dot(d.gDe, d.dDe, (int64_t)n1 * n1, red);
    dJc = dJf;
    if (d.through_clamp && n1 == n2) {
      // dLe = Le Phi, Phi = lower(Le^-1 dDe Le^-T) with halved diagonal
      double* M = Lp;  // reuse (n1 x n1)
      wg_copy(M, d.dDe, (int64_t)n1 * n1);
      wg_trsm_left_lower(Le, n1, M, n1);
      wg_trsm_right_lowerT(Le, n1, M, n1);
      for (int64_t g = threadIdx.x; g < (int64_t)n1 * n1; g += blockDim.x) {
        int r = (int)(g % n1), c = (int)(g / n1);
        M[g] = r > c ? M[g] : (r == c ? 0.5 * M[g] : 0.0);
      }
      __syncthreads();
      // dA = -Phi A0 ; dX = U^T dA W with U = (A S^-1)
      double* dA = Ae;  // reuse (n1 x n1 >= n1 x n2 when square)
      wg_gemm(n1, n2, n1, M, false, A0, false, dA);
      double* T1 = Ah;  // n2 x n2
      wg_gemm(n1, n2, n2, dA, false, V, false, Kh);   // dA W  (n1 x n2) into Kh
      wg_gemm(n2, n2, n1, A, true, Kh, false, T1);    // (U S)^T dA W
      for (int64_t g = threadIdx.x; g < (int64_t)n2 * n2; g += blockDim.x) {
        int r = (int)(g % n2), c = (int)(g / n2);
        T1[g] = -T1[g] / (sig[r] > 0 ? sig[r] : 1.0);  // dX (with dA = -Phi A0)
      }
      __syncthreads();
      // G via divided differences of f(s) = min(s, lim); stored in Ke (n1 x n2 = n2 x n2)
      for (int64_t g = threadIdx.x; g < (int64_t)n2 * n2; g += blockDim.x) {
        int i = (int)(g % n2), j = (int)(g / n2);
        double si = sig[i], sj = sig[j];
        double fi = fmin(si, lim), fj = fmin(sj, lim);
        double dx = T1[g], dxt = T1[j + (int64_t)i * n2];
        double val;
        if (i == j) {
          val = (si < lim ? 1.0 : 0.0) * dx;
        } else {
          double ps = 0.5 * (dx + dxt), sk = 0.5 * (dx - dxt);
          double dd = si - sj;
          double q1 = fabs(dd) > 1e-14 * (si + sj) ? (fi - fj) / dd : (si < lim ? 1.0 : 0.0);
          double q2 = (si + sj) > 0 ? (fi + fj) / (si + sj) : 1.0;
          val = ps * q1 + sk * q2;
        }
        Ke[g] = val;
      }
      __syncthreads();
      // dA' = U G W^T ; U = A S^-1
      for (int64_t g = threadIdx.x; g < (int64_t)n1 * n2; g += blockDim.x) {
        int c = (int)(g / n1);
        Kh[g] = A[g] / (sig[c] > 0 ? sig[c] : 1.0);
      }
      __syncthreads();
      wg_gemm(n1, n2, n2, Kh, false, Ke, false, T1);   // U G (square)
      wg_gemm(n1, n2, n2, T1, false, V, true, Kh);     // dA'
      // dK' = dLe A' Lm^T + Le dA' Lm^T = Le (Phi A' + dA') Lm^T
      wg_gemm(n1, n2, n1, M, false, Ap, false, T1);
      for (int64_t g = threadIdx.x; g < (int64_t)n1 * n2; g += blockDim.x) T1[g] += Kh[g];
      __syncthreads();
      wg_gemm(n1, n2, n1, Le, false, T1, false, Kh);
      wg_gemm(n1, n2, n2, Kh, false, Lm, true, T1);    // dK'
      dJc = dJf + wg_dot(d.gK, T1, (int64_t)n1 * n2, red);
    }
  }
  if (threadIdx.x == 0) {
    d.out[0] = Jloc;
    d.out[1] = dJf;
    d.out[2] = dJc;
    d.out[3] = 0;
  }
}

// ---------------------------------------------------------------- host

static int upload(DevBuf& b, size_t off_doubles, const std::vector<double>& v) {
  if (v.empty()) return YR_OK;
  YR_TRY_HIP(hipMemcpy(b.as<double>() + off_doubles, v.data(), v.size() * 8, hipMemcpyHostToDevice));
  return YR_OK;
}

static bool any_nonzero(const std::vector<double>& v) {
  for (double x : v)
    if (x != 0) return true;
  return false;
}

// One block-Jacobi phase over the matrices `mats` (rounds launched back to
// back; the convergence flags are read once per sweep)
struct JacMat {
  double* X;
  double* W;
  int n;
  const int* status;
};

static int bjac_phase(const std::vector<JacMat>& mats) {
  const int nd = (int)mats.size();
  if (nd == 0) return YR_OK;
  std::vector<JacDesc> jd(nd);
  std::vector<int> wg_desc;
  DevBuf dflags, djd, dwg;
  YR_CALL(dflags.reserve((size_t)2 * nd * sizeof(int)));
  int* rot = dflags.as<int>();
  int* active = rot + nd;
  int rmax = 0;
  for (int i = 0; i < nd; ++i) {
    const int n = mats[i].n;
    const int bs = std::max(1, std::min({16, kBjacLds / std::max(n, 1), (n + 1) / 2}));
    int nblk = (n + bs - 1) / bs;
    nblk = std::max(2, nblk + (nblk & 1));
    jd[i] = JacDesc{mats[i].X, mats[i].W, n, bs, nblk, (int)wg_desc.size(), rot + i, active + i,
                    mats[i].status};
    for (int p = 0; p < nblk / 2; ++p) wg_desc.push_back(i);
    rmax = std::max(rmax, nblk - 1);
  }
  std::vector<int> flags((size_t)2 * nd, 0);
  for (int i = 0; i < nd; ++i) flags[(size_t)nd + i] = 1;
  YR_TRY_HIP(hipMemcpy(dflags.p, flags.data(), flags.size() * sizeof(int), hipMemcpyHostToDevice));
  YR_CALL(djd.reserve(jd.size() * sizeof(JacDesc)));
  YR_TRY_HIP(hipMemcpy(djd.p, jd.data(), jd.size() * sizeof(JacDesc), hipMemcpyHostToDevice));
  YR_CALL(dwg.reserve(wg_desc.size() * sizeof(int)));
  YR_TRY_HIP(hipMemcpy(dwg.p, wg_desc.data(), wg_desc.size() * sizeof(int), hipMemcpyHostToDevice));
  std::vector<int> act(nd);
  for (int sweep = 0; sweep < kJacSweepsMax; ++sweep) {
    for (int r = 0; r < rmax; ++r)
      k_bjac_round<<<(unsigned)wg_desc.size(), 1024>>>(djd.as<JacDesc>(), dwg.as<int>(), r, kJacTol);
    k_bjac_check<<<(nd + 255) / 256, 256>>>(djd.as<JacDesc>(), nd);
    YR_TRY_HIP(hipGetLastError());
    YR_TRY_HIP(hipMemcpy(act.data(), active, nd * sizeof(int), hipMemcpyDeviceToHost));
    bool any = false;
    for (int a : act) any = any || a != 0;
    if (!any) break;
  }
  return YR_OK;
}

static int perturb_batch(yr_rom* const* roms, int nm, double dt, double gamma, yr_dtype dtype,
                         int32_t* nclamped_out) {
  std::vector<PerturbDesc> descs(nm);
  std::vector<size_t> in_off(nm), out_off(nm), work_off(nm);
  size_t tot_in = 0, tot_out = 0, tot_work = 0;
  for (int m = 0; m < nm; ++m) {
    const yr_rom* r = roms[m];
    size_t n1 = r->q1, n2 = r->q2, ns = r->nsrc, np = r->nprb;
    in_off[m] = tot_in;
    tot_in += 2 * n1 * n1 + 2 * n2 * n2 + n1 * n2 + (n1 + n2) * (ns + np);
    out_off[m] = tot_out;
    tot_out += 2 * n1 * n2 + n2 + 2 * (n1 + n2) + (n1 + n2) * (ns + np) + 2;
    work_off[m] = tot_work;
    tot_work += perturb_work_doubles(r->q1, r->q2, r->nsrc, r->nprb);
  }
  DevBuf din, dout, dwork, ddesc;
  YR_CALL(din.reserve(tot_in * 8 + 8));
  YR_CALL(dout.reserve(tot_out * 8 + 8));
  YR_CALL(dwork.reserve(tot_work * 8 + 8));
  for (int m = 0; m < nm; ++m) {
    const yr_rom* r = roms[m];
    size_t n1 = r->q1, n2 = r->q2, ns = r->nsrc, np = r->nprb;
    double* ib = din.as<double>() + in_off[m];
    double* ob = dout.as<double>() + out_off[m];
    size_t o = 0;
    PerturbDesc& d = descs[m];
    d.n1 = (int)n1;
    d.n2 = (int)n2;
    d.ns = (int)ns;
    d.np = (int)np;
    d.dt = dt;
    d.gamma = gamma;
    d.lossy_e = any_nonzero(r->Dse);
    d.lossy_m = any_nonzero(r->Dsm);
    const std::vector<double>* src[9] = {&r->De, &r->Dse, &r->Dm, &r->Dsm, &r->K,
                                         &r->B1, &r->B2,  &r->L1, &r->L2};
    const double** dst[9] = {&d.De, &d.Dse, &d.Dm, &d.Dsm, &d.K, &d.B1, &d.B2, &d.L1, &d.L2};
    for (int a = 0; a < 9; ++a) {
      *dst[a] = ib + o;
      YR_CALL(upload(din, in_off[m] + o, *src[a]));
      o += src[a]->size();
    }
    size_t q = 0;
    d.Kp = ob + q;
    q += n1 * n2;
    d.A2 = ob + q;
    q += n1 * n2;
    d.sigma = ob + q;
    q += n2;
    d.ce = ob + q;
    q += n1;
    d.ge = ob + q;
    q += n1;
    d.cm = ob + q;
    q += n2;
    d.gm = ob + q;
    q += n2;
    d.be = ob + q;
    q += n1 * ns;
    d.bh = ob + q;
    q += n2 * ns;
    d.oe = ob + q;
    q += n1 * np;
    d.oh = ob + q;
    q += n2 * np;
    d.status = reinterpret_cast<int*>(ob + q);
    d.nclamped = reinterpret_cast<int*>(ob + q + 1);
    d.work = dwork.as<double>() + work_off[m];
    YR_CALL(roms[m]->lift.reserve((n1 * n1 + n2 * n2) * 8));
    d.Te = roms[m]->lift.as<double>();
    d.Tm = d.Te + n1 * n1;
  }
  YR_CALL(ddesc.reserve(descs.size() * sizeof(PerturbDesc)));
  YR_TRY_HIP(hipMemcpy(ddesc.p, descs.data(), descs.size() * sizeof(PerturbDesc), hipMemcpyHostToDevice));
  // stage kernels around the three Jacobi phases (singular values of the
  // whitened K~, eigen-decompositions of the whitened loss matrices)
  std::vector<JacMat> ph1, ph2, ph3;
  for (int m = 0; m < nm; ++m) {
    const PerturbDesc& d = descs[m];
    const PerturbWork w = perturb_work(d.work, d.n1, d.n2, d.ns, d.np);
    ph1.push_back(JacMat{w.S1, w.V, std::min(d.n1, d.n2), d.status});
    if (d.lossy_e) ph2.push_back(JacMat{w.S2, w.Qe, d.n1, d.status});
    if (d.lossy_m) ph3.push_back(JacMat{w.S1, w.V, d.n2, d.status});
  }
  const PerturbDesc* dd = ddesc.as<PerturbDesc>();
  k_perturb_s1<<<nm, kPBlock>>>(dd);
  YR_CALL(bjac_phase(ph1));
  k_perturb_s2<<<nm, kPBlock>>>(dd);
  YR_CALL(bjac_phase(ph2));
  k_perturb_s3<<<nm, kPBlock>>>(dd);
  YR_CALL(bjac_phase(ph3));
  k_perturb_s4<<<nm, kPBlock>>>(dd);
  YR_TRY_HIP(hipGetLastError());
  YR_TRY_HIP(hipDeviceSynchronize());
  std::vector<double> hout(tot_out);
  YR_TRY_HIP(hipMemcpy(hout.data(), dout.p, tot_out * 8, hipMemcpyDeviceToHost));
  // rounding to the stepping precision, stored per model
  const size_t es = dtype == YR_F64 ? 8 : 4;
  std::vector<GuardDesc> gd(nm);
  DevBuf gwork, gout;
  size_t gw_tot = 0;
  for (int m = 0; m < nm; ++m) gw_tot += (size_t)roms[m]->q2 * roms[m]->q2 + (size_t)roms[m]->q1 * roms[m]->q2;
  YR_CALL(gwork.reserve(gw_tot * 8 + 8));
  YR_CALL(gout.reserve(nm * 8 + 8));
  size_t gw = 0;
  for (int m = 0; m < nm; ++m) {
    yr_rom* r = roms[m];
    const PerturbDesc& d = descs[m];
    const double* ob = hout.data() + out_off[m];
    int status = reinterpret_cast<const int*>(ob + (d.oh - d.Kp) + (size_t)d.n2 * d.np)[0];
    int ncl = reinterpret_cast<const int*>(ob + (d.oh - d.Kp) + (size_t)d.n2 * d.np + 1)[0];
    YR_REQUIRE(status != 1, YR_EINVAL, "De~ is not positive definite");
    YR_REQUIRE(status != 2, YR_EINVAL, "Dm~ is not positive definite");
    size_t n1 = r->q1, n2 = r->q2, ns = r->nsrc, np = r->nprb;
    r->Kp.assign(ob, ob + n1 * n2);
    r->sigma.assign(ob + 2 * n1 * n2, ob + 2 * n1 * n2 + n2);
    std::sort(r->sigma.begin(), r->sigma.end(), [](double a, double b) { return a > b; });
    r->sigma.resize(std::min(n1, n2));
    r->n_clamped = ncl;
    if (nclamped_out) nclamped_out[m] = ncl;
    size_t nvec = 2 * n1 + 2 * n2 + (n1 + n2) * (ns + np);
    // A2 (col-major FP64) -> row-major stepping dtype, rows padded for 16-byte
    // vector loads, and its transpose; vectors are contiguous after sigma
    const int vw = (int)(16 / es);
    r->ld_a = (int)((n2 + vw - 1) / vw * vw);
    r->ld_at = (int)((n1 + vw - 1) / vw * vw);
    YR_CALL(r->A.reserve(std::max<size_t>(1, n1 * r->ld_a) * es));
    YR_CALL(r->AT.reserve(std::max<size_t>(1, n2 * r->ld_at) * es));
    YR_CALL(r->vec.reserve(nvec * es));
    const double* dA2 = d.A2;
    const double* dvec = d.ce;
    const int64_t na = (int64_t)n1 * r->ld_a, nat = (int64_t)n2 * r->ld_at;
    if (dtype == YR_F64) {
      if (na) k_round_rows<double><<<grid_for(na), kBlock>>>(dA2, (int)n1, (int)n2, r->A.as<double>(), r->ld_a, 0);
      if (nat) k_round_rows<double><<<grid_for(nat), kBlock>>>(dA2, (int)n1, (int)n2, r->AT.as<double>(), r->ld_at, 1);
      k_round<double><<<grid_for(nvec), kBlock>>>(dvec, r->vec.as<double>(), nvec, 0, 0);
    } else {
      if (na) k_round_rows<float><<<grid_for(na), kBlock>>>(dA2, (int)n1, (int)n2, r->A.as<float>(), r->ld_a, 0);
      if (nat) k_round_rows<float><<<grid_for(nat), kBlock>>>(dA2, (int)n1, (int)n2, r->AT.as<float>(), r->ld_at, 1);
      k_round<float><<<grid_for(nvec), kBlock>>>(dvec, r->vec.as<float>(), nvec, 0, 0);
    }
    YR_TRY_HIP(hipGetLastError());
    gd[m].n1 = (int)n1;
    gd[m].n2 = (int)n2;
    gd[m].lda = r->ld_a;
    gd[m].A = r->A.p;
    gd[m].vec = r->vec.p;
    gd[m].work = gwork.as<double>() + gw;
    gd[m].out = gout.as<double>() + m;
    gd[m].f64 = dtype == YR_F64;
    gw += n2 * n2 + n1 * n2;
  }
  DevBuf dgd;
  YR_CALL(dgd.reserve(gd.size() * sizeof(GuardDesc)));
  YR_TRY_HIP(hipMemcpy(dgd.p, gd.data(), gd.size() * sizeof(GuardDesc), hipMemcpyHostToDevice));
  k_guard<<<nm, kPBlock>>>(dgd.as<GuardDesc>());
  YR_TRY_HIP(hipGetLastError());
  std::vector<double> cert(nm);
  YR_TRY_HIP(hipMemcpy(cert.data(), gout.p, nm * 8, hipMemcpyDeviceToHost));
  for (int m = 0; m < nm; ++m) {
    roms[m]->guard_margin = cert[m];
    roms[m]->step_dt = cert[m] > 0 ? dt : -1;
    roms[m]->step_dtype = cert[m] > 0 ? (int)dtype : -1;
  }
  for (int m = 0; m < nm; ++m)
    YR_REQUIRE(cert[m] > 0, YR_EUNSTABLE,
               "stepping matrices fail the FP64 stability certificate sigma_max(M) < 2");
  return YR_OK;
}

// ---------------------------------------------------------------- stepping autotuner

template <typename T>
static void launch_step(int nt, int nmodels, const StepDesc* dd, int64_t nsteps, int qmax,
                        hipStream_t s) {
  const size_t es = sizeof(T);
  const size_t smem = (size_t)nt * (16 / es) * sizeof(double) + 2 * (size_t)qmax * es;
  if (nt == 256)
    k_rom_step<T, 256><<<nmodels, 256, smem, s>>>(dd, nsteps, qmax);
  else if (nt == 512)
    k_rom_step<T, 512><<<nmodels, 512, smem, s>>>(dd, nsteps, qmax);
  else
    k_rom_step<T, 1024><<<nmodels, 1024, smem, s>>>(dd, nsteps, qmax);
}

// Workgroup size per model (256, 512 or 1024 threads), picked by timing: the
// best one depends on the orders (rows per thread) and on how many models
// share the device.  Keyed by (dtype, largest order rounded up to 32, number
// of models rounded up to a power of two).  The trial launches step every
// model kTuneSteps times from a zero state into scratch outputs (the caller's
// inputs are only read) and are timed with HIP events on the stream.
constexpr int64_t kTuneMinSteps = 2048;  // shorter runs use kSBlock untuned
constexpr int kTuneSteps = 64;

static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int>, int> g_tune;

static int tuned_threads(const std::vector<StepDesc>& descs, yr_dtype dtype, int nmodels,
                         int qmax, hipStream_t s, int* nt_out) {
  int nm2 = 1;
  while (nm2 < nmodels) nm2 *= 2;
  const auto key = std::make_tuple((int)dtype, (qmax + 31) / 32, nm2);
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      *nt_out = it->second;
      return YR_OK;
    }
  }
  const size_t es = dtype == YR_F64 ? 8 : 4;
  std::vector<StepDesc> trial = descs;
  size_t ytot = 0;
  for (const auto& d : trial) ytot += (size_t)kTuneSteps * d.np;
  void* yscratch = nullptr;
  void* dd = nullptr;
  YR_TRY_HIP(hipMallocAsync(&yscratch, ytot * es + 16, s));
  size_t off = 0;
  for (auto& d : trial) {
    d.y = static_cast<char*>(yscratch) + off * es;
    d.state = nullptr;
    off += (size_t)kTuneSteps * d.np;
  }
  YR_TRY_HIP(hipMallocAsync(&dd, trial.size() * sizeof(StepDesc), s));
  YR_TRY_HIP(hipMemcpyAsync(dd, trial.data(), trial.size() * sizeof(StepDesc), hipMemcpyHostToDevice, s));
  YR_TRY_HIP(hipStreamSynchronize(s));
  hipEvent_t e0, e1;
  YR_TRY_HIP(hipEventCreate(&e0));
  YR_TRY_HIP(hipEventCreate(&e1));
  int best = kSBlock;
  float best_ms = 0;
  const int W = (int)(16 / es);
  for (int nt : {256, 512, 1024}) {
    if ((int64_t)nt * W < qmax) continue;  // every column needs a thread (mv_partial)
    for (int rep = 0; rep < 2; ++rep) {  // first launch warms caches and code
      (void)hipEventRecord(e0, s);
      if (dtype == YR_F64)
        launch_step<double>(nt, nmodels, (const StepDesc*)dd, kTuneSteps, qmax, s);
      else
        launch_step<float>(nt, nmodels, (const StepDesc*)dd, kTuneSteps, qmax, s);
      (void)hipEventRecord(e1, s);
    }
    YR_TRY_HIP(hipGetLastError());
    YR_TRY_HIP(hipEventSynchronize(e1));
    float ms = 0;
    YR_TRY_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (std::getenv("YR_VERBOSE"))
      fprintf(stderr, "[rom_step tune] models %d qmax %d threads %d: %.3f ms / %d steps\n",
              nmodels, qmax, nt, ms, kTuneSteps);
    if (best_ms == 0 || ms < best_ms) {
      best = nt;
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  YR_TRY_HIP(hipFreeAsync(dd, s));
  YR_TRY_HIP(hipFreeAsync(yscratch, s));
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = best;
  }
  *nt_out = best;
  return YR_OK;
}

// Stepping descriptors of nmodels prepared models (checks shared by rom_step
// and rom_step_noalloc).
static int fill_step_descs(yr_rom* const* roms, int nmodels, double dt, yr_dtype dtype,
                           const void* const* u, void* const* y, void* const* state,
                           StepDesc* descs, int* qmax_out) {
  int qmax = 0;
  for (int m = 0; m < nmodels; ++m) {
    const yr_rom* r = roms[m];
    YR_REQUIRE(r, YR_EINVAL, "null model");
    YR_REQUIRE(r->step_dt == dt && r->step_dtype == (int)dtype, YR_ESTATE,
               "model not prepared for this dt/dtype: call rom_perturb first");
    YR_REQUIRE(r->nsrc == 0 || (u && u[m]), YR_EINVAL, "missing input waveform");
    YR_REQUIRE(r->nprb == 0 || (y && y[m]), YR_EINVAL, "missing output buffer");
    qmax = std::max(qmax, std::max(r->q1, r->q2));
    descs[m].n1 = r->q1;
    descs[m].n2 = r->q2;
    descs[m].ns = r->nsrc;
    descs[m].np = r->nprb;
    descs[m].lda = r->ld_a;
    descs[m].ldat = r->ld_at;
    descs[m].A = r->A.p;
    descs[m].AT = r->AT.p;
    descs[m].vec = r->vec.p;
    descs[m].u = u ? u[m] : nullptr;
    descs[m].y = y ? y[m] : nullptr;
    descs[m].state = state ? state[m] : nullptr;
  }
  *qmax_out = qmax;
  return YR_OK;
}

// Workgroup size already picked by the autotuner for this shape, without
// running a trial (trials allocate their scratch outputs): kSBlock if none.
static int cached_threads(yr_dtype dtype, int nmodels, int qmax) {
  int nm2 = 1;
  while (nm2 < nmodels) nm2 *= 2;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(std::make_tuple((int)dtype, (qmax + 31) / 32, nm2));
  return it != g_tune.end() ? it->second : kSBlock;
}

// ------------------------------------------------ stepping without allocation
//
// rom_step_noalloc keeps its descriptor table in `scratch`, a fixed device
// array (each device holds its own copy for the life of the process), instead
// of stream-ordered allocations.  Host code must not take the array's name as
// a device address: the address of each device's copy comes from
// hipGetSymbolAddress, once per device, and only that address is used.
constexpr int kNoAllocModels = 4096;
static __device__ __align__(256) StepDesc scratch[kNoAllocModels];

constexpr int kMaxDevices = 64;
static std::mutex g_noalloc_mu;
static StepDesc* g_scratch_ptr[kMaxDevices];
static StepDesc g_noalloc_host[kNoAllocModels];

static int noalloc_scratch(StepDesc** out) {
  int dev = 0;
  YR_TRY_HIP(hipGetDevice(&dev));
  YR_REQUIRE(dev >= 0 && dev < kMaxDevices, YR_EDEVICE, "device index out of range");
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    YR_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    YR_REQUIRE(p, YR_EDEVICE, "no device address for the stepping scratch table");
    g_scratch_ptr[dev] = static_cast<StepDesc*>(p);
  }
  *out = g_scratch_ptr[dev];
  return YR_OK;
}

// ---------------------------------------------------------------- reconstruction

// xt[m][xoff + j] = sum_k Tr[j + k n] s[m][soff + k] in FP64 (Tr n x n, column-major)
template <typename T>
__global__ void k_lift_coeffs(const double* __restrict__ Tr, int n, const T* __restrict__ s,
                              int lds, int soff, int nstates, double* __restrict__ xt, int ldx,
                              int xoff) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= (int64_t)nstates * n) return;
  const int m = (int)(g / n), j = (int)(g % n);
  const T* sm = s + (int64_t)m * lds + soff;
  double acc = 0;
  for (int k = 0; k < n; ++k) acc += Tr[j + (int64_t)k * n] * (double)sm[k];
  xt[(int64_t)m * ldx + xoff + j] = acc;
}

constexpr int kLiftStates = 4;  // states per pass over the basis

// out[m][ooff + row] = sum_j V[j n + row] xt[m][xoff + j]: one block of the field
// buffer (E rows from V1 or H rows from V2); every basis row is read once per
// kLiftStates states, coalesced along the padded layout.
template <typename T>
__global__ void __launch_bounds__(256)
    k_lift_rows(const double* __restrict__ V, int64_t n, int q, const double* __restrict__ xt,
                int ldx, int xoff, int nstates, T* __restrict__ out, int64_t ldo, int64_t ooff) {
  extern __shared__ double xs[];  // [kLiftStates][q]
  for (int m0 = 0; m0 < nstates; m0 += kLiftStates) {
    const int nm = min(kLiftStates, nstates - m0);
    __syncthreads();
    for (int g = threadIdx.x; g < kLiftStates * q; g += blockDim.x) {
      const int t = g / q, j = g - t * q;
      xs[g] = t < nm ? xt[(int64_t)(m0 + t) * ldx + xoff + j] : 0.0;
    }
    __syncthreads();
    for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < n;
         row += (int64_t)gridDim.x * blockDim.x) {
      double acc[kLiftStates];
#pragma unroll
      for (int t = 0; t < kLiftStates; ++t) acc[t] = 0;
      for (int j = 0; j < q; ++j) {
        const double v = V[(int64_t)j * n + row];
#pragma unroll
        for (int t = 0; t < kLiftStates; ++t) acc[t] += v * xs[t * q + j];
      }
      for (int t = 0; t < nm; ++t) out[(int64_t)(m0 + t) * ldo + ooff + row] = (T)acc[t];
    }
  }
}

template <typename T>
static int lift_impl(const yr_operator* op, const yr_rom* r, int nstates, const void* states,
                     void* fields, hipStream_t s) {
  const int q1 = r->q1, q2 = r->q2, ld = q1 + q2;
  const int64_t flen = (int64_t)(op->ne_slots + op->nh_slots) * op->len;
  void* xt = nullptr;
  YR_TRY_HIP(hipMallocAsync(&xt, (size_t)nstates * ld * 8 + 8, s));
  const double* Te = r->lift.as<double>();
  const double* Tm = Te + (size_t)q1 * q1;
  const T* st = static_cast<const T*>(states);
  double* x = static_cast<double*>(xt);
  if (q1) k_lift_coeffs<T><<<grid_for((int64_t)nstates * q1), kBlock, 0, s>>>(Te, q1, st, ld, 0, nstates, x, ld, 0);
  if (q2) k_lift_coeffs<T><<<grid_for((int64_t)nstates * q2), kBlock, 0, s>>>(Tm, q2, st, ld, q1, nstates, x, ld, q1);
  auto rows_grid = [](int64_t n) { return (unsigned)std::min<int64_t>(std::max<int64_t>(1, (n + 255) / 256), 4096); };
  T* out = static_cast<T*>(fields);
  k_lift_rows<T><<<rows_grid(r->nE), 256, (size_t)kLiftStates * std::max(1, q1) * 8, s>>>(
      r->V1.as<double>(), r->nE, q1, x, ld, 0, nstates, out, flen, 0);
  k_lift_rows<T><<<rows_grid(r->nH), 256, (size_t)kLiftStates * std::max(1, q2) * 8, s>>>(
      r->V2.as<double>(), r->nH, q2, x, ld, q1, nstates, out, flen, r->nE);
  YR_TRY_HIP(hipGetLastError());
  YR_TRY_HIP(hipFreeAsync(xt, s));
  return YR_OK;
}

}  // namespace yr

using namespace yr;

extern "C" {

int rom_lift(const yr_operator* op, const yr_rom* rom, yr_dtype dtype, int32_t nstates,
             const void* states, void* fields, void* stream) {
  YR_REQUIRE(op && rom, YR_EINVAL, "null argument");
  YR_REQUIRE(nstates >= 0, YR_EINVAL, "nstates must be non-negative");
  YR_REQUIRE(dtype == YR_F32 || dtype == YR_F64, YR_EINVAL, "bad dtype");
  YR_REQUIRE(rom->nE > 0 && rom->nE == op->ne_slots * op->len && rom->nH == op->nh_slots * op->len,
             YR_ESTATE, "model was not reduced from this operator");
  YR_REQUIRE(rom->step_dt > 0 && rom->lift.p, YR_ESTATE, "model not prepared by rom_perturb");
  YR_REQUIRE(rom->q1 <= 1024 && rom->q2 <= 1024, YR_EINVAL, "reduced order above 1024");
  if (nstates == 0) return YR_OK;
  YR_REQUIRE(states && fields, YR_EINVAL, "null buffer");
  hipStream_t s = static_cast<hipStream_t>(stream);
  return dtype == YR_F64 ? lift_impl<double>(op, rom, nstates, states, fields, s)
                         : lift_impl<float>(op, rom, nstates, states, fields, s);
}

int rom_perturb_batch(yr_rom* const* roms, int32_t nmodels, double dt, double gamma,
                      yr_dtype step_dtype, int32_t* n_clamped) {
  YR_REQUIRE(roms && nmodels > 0, YR_EINVAL, "no models");
  YR_REQUIRE(dt > 0 && std::isfinite(dt), YR_EINVAL, "dt must be positive");
  YR_REQUIRE(gamma > 0 && gamma <= 4, YR_EINVAL, "gamma must lie in (0, 4]");
  YR_REQUIRE(step_dtype == YR_F32 || step_dtype == YR_F64, YR_EINVAL, "bad dtype");
  for (int m = 0; m < nmodels; ++m) {
    YR_REQUIRE(roms[m] && roms[m]->q1 > 0 && roms[m]->q2 > 0, YR_EINVAL, "empty reduced model");
    YR_REQUIRE(roms[m]->q1 <= 64 * kJacRowsMax && roms[m]->q2 <= 64 * kJacRowsMax, YR_EINVAL,
               "reduced order above 512");
  }
  return perturb_batch(roms, nmodels, dt, gamma, step_dtype, n_clamped);
}

int rom_perturb(yr_rom* rom, double dt, double gamma, yr_dtype step_dtype, int32_t* n_clamped) {
  return rom_perturb_batch(&rom, 1, dt, gamma, step_dtype, n_clamped);
}

int rom_adjoint(yr_rom* rom, double dt, double gamma, int64_t nsteps, const double* u,
                const double* dJdy, const double* dDe, int32_t through_clamp, double* gDe,
                double* gDse, double* gK, double* result) {
  YR_REQUIRE(rom && result && nsteps > 0 && dt > 0, YR_EINVAL, "bad arguments");
  YR_REQUIRE(gamma > 0 && gamma <= 4, YR_EINVAL, "gamma must lie in (0, 4]");
  YR_REQUIRE(rom->nsrc == 0 || u, YR_EINVAL, "missing input waveform");
  YR_REQUIRE(rom->nprb > 0 && dJdy, YR_EINVAL, "the objective needs probes and dJ/dy");
  YR_REQUIRE(!(dDe && through_clamp) || rom->q1 == rom->q2, YR_EINVAL,
             "the derivative through the clamp needs q1 == q2");
  const int n1 = rom->q1, n2 = rom->q2, ns = rom->nsrc, np = rom->nprb;
  const std::vector<double>* mats[9] = {&rom->De, &rom->Dse, &rom->Dm, &rom->Dsm, &rom->K,
                                        &rom->B1, &rom->B2,  &rom->L1, &rom->L2};
  size_t tin = 0;
  for (auto* m : mats) tin += m->size();
  tin += (size_t)n1 * n1;
  DevBuf din, dwork, dout, ddesc;
  const size_t tout = 2 * (size_t)n1 * n1 + 2 * (size_t)n1 * n2 + 8;
  YR_CALL(din.reserve(tin * 8 + 8));
  YR_CALL(dout.reserve(tout * 8));
  YR_CALL(dwork.reserve(adj_work_doubles(n1, n2, ns, np, nsteps) * 8));
  AdjDesc d{};
  d.n1 = n1;
  d.n2 = n2;
  d.ns = ns;
  d.np = np;
  d.nsteps = nsteps;
  d.dt = dt;
  d.gamma = gamma;
  d.through_clamp = through_clamp;
  size_t o = 0;
  const double** dst[9] = {&d.De, &d.Dse, &d.Dm, &d.Dsm, &d.K, &d.B1, &d.B2, &d.L1, &d.L2};
  for (int a = 0; a < 9; ++a) {
    *dst[a] = din.as<double>() + o;
    YR_CALL(upload(din, o, *mats[a]));
    o += mats[a]->size();
  }
  d.dDe = nullptr;
  if (dDe) {
    YR_TRY_HIP(hipMemcpy(din.as<double>() + o, dDe, (size_t)n1 * n1 * 8, hipMemcpyHostToDevice));
    d.dDe = din.as<double>() + o;
  }
  d.u = u;
  d.dJdy = dJdy;
  d.work = dwork.as<double>();
  double* ob = dout.as<double>();
  d.gDe = ob;
  d.gDse = ob + (size_t)n1 * n1;
  d.gK = ob + 2 * (size_t)n1 * n1;
  d.Kp = d.gK + (size_t)n1 * n2;
  d.out = d.Kp + (size_t)n1 * n2;
  YR_CALL(ddesc.reserve(sizeof(AdjDesc)));
  YR_TRY_HIP(hipMemcpy(ddesc.p, &d, sizeof(AdjDesc), hipMemcpyHostToDevice));
  YR_TRY_HIP(hipDeviceSynchronize());  // the caller's u / dJdy are complete
  k_rom_adjoint<<<1, kPBlock>>>(ddesc.as<AdjDesc>());
  YR_TRY_HIP(hipGetLastError());
  YR_TRY_HIP(hipDeviceSynchronize());
  std::vector<double> h(tout);
  YR_TRY_HIP(hipMemcpy(h.data(), ob, tout * 8, hipMemcpyDeviceToHost));
  const double* res = h.data() + 2 * (size_t)n1 * n1 + 2 * (size_t)n1 * n2;
  YR_REQUIRE(res[3] == 0, YR_EINVAL, "reduced matrices are not positive definite");
  if (gDe) std::memcpy(gDe, h.data(), (size_t)n1 * n1 * 8);
  if (gDse) std::memcpy(gDse, h.data() + (size_t)n1 * n1, (size_t)n1 * n1 * 8);
  if (gK) std::memcpy(gK, h.data() + 2 * (size_t)n1 * n1, (size_t)n1 * n2 * 8);
  result[0] = res[0];
  result[1] = res[1];
  result[2] = res[2];
  return YR_OK;
}

int rom_step(yr_rom* const* roms, int32_t nmodels, double dt, int64_t nsteps, yr_dtype dtype,
             const void* const* u, void* const* y, void* const* state, void* stream_) {
  YR_REQUIRE(roms && nmodels > 0 && nsteps >= 0, YR_EINVAL, "bad arguments");
  YR_REQUIRE(dtype == YR_F32 || dtype == YR_F64, YR_EINVAL, "bad dtype");
  int qmax = 0;
  std::vector<StepDesc> descs(nmodels);
  YR_CALL(fill_step_descs(roms, nmodels, dt, dtype, u, y, state, descs.data(), &qmax));
  YR_REQUIRE(qmax <= 2048, YR_EINVAL, "reduced order above 2048");
  if (nsteps == 0) return YR_OK;
  hipStream_t s = static_cast<hipStream_t>(stream_);
  int nt = kSBlock;
  if (nsteps >= kTuneMinSteps) {
    YR_CALL(tuned_threads(descs, dtype, nmodels, qmax, s, &nt));
  }
  // the descriptor table: every check that can fail is done before it is
  // allocated, so no error path leaves it behind
  void* dd = nullptr;
  YR_TRY_HIP(hipMallocAsync(&dd, descs.size() * sizeof(StepDesc), s));
  hipError_t ce = hipMemcpyAsync(dd, descs.data(), descs.size() * sizeof(StepDesc),
                                 hipMemcpyHostToDevice, s);
  if (ce == hipSuccess) ce = hipStreamSynchronize(s);  // the host table must outlive the copy
  if (ce != hipSuccess) {
    (void)hipFreeAsync(dd, s);
    YR_REQUIRE(false, YR_EDEVICE, std::string("descriptor table copy failed: ") + hipGetErrorString(ce));
  }
  if (dtype == YR_F64)
    launch_step<double>(nt, nmodels, (const StepDesc*)dd, nsteps, qmax, s);
  else
    launch_step<float>(nt, nmodels, (const StepDesc*)dd, nsteps, qmax, s);
  YR_TRY_HIP(hipGetLastError());
  YR_TRY_HIP(hipFreeAsync(dd, s));
  return YR_OK;
}

int rom_step_noalloc(yr_rom* const* roms, int32_t nmodels, double dt, int64_t nsteps,
                     yr_dtype dtype, const void* const* u, void* const* y, void* const* state,
                     void* stream_) {
  YR_REQUIRE(roms && nmodels > 0 && nsteps >= 0, YR_EINVAL, "bad arguments");
  YR_REQUIRE(nmodels <= kNoAllocModels, YR_EINVAL,
             "rom_step_noalloc takes at most 4096 models per call");
  YR_REQUIRE(dtype == YR_F32 || dtype == YR_F64, YR_EINVAL, "bad dtype");
  // one host table and one device table per process (calls on a device race)
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  int qmax = 0;
  YR_CALL(fill_step_descs(roms, nmodels, dt, dtype, u, y, state, g_noalloc_host, &qmax));
  YR_REQUIRE(qmax <= 2048, YR_EINVAL, "reduced order above 2048");
  if (nsteps == 0) return YR_OK;
  StepDesc* dd = nullptr;
  YR_CALL(noalloc_scratch(&dd));
  hipStream_t s = static_cast<hipStream_t>(stream_);
  YR_TRY_HIP(hipMemcpyAsync(dd, g_noalloc_host, (size_t)nmodels * sizeof(StepDesc),
                            hipMemcpyHostToDevice, s));
  // the host table is reused by the next call: the copy must have read it
  YR_TRY_HIP(hipStreamSynchronize(s));
  int nt = kSBlock;
  if (nsteps >= kTuneMinSteps) nt = cached_threads(dtype, nmodels, qmax);
  if (dtype == YR_F64)
    launch_step<double>(nt, nmodels, dd, nsteps, qmax, s);
  else
    launch_step<float>(nt, nmodels, dd, nsteps, qmax, s);
  YR_TRY_HIP(hipGetLastError());
  return YR_OK;
}

}  // extern "C"
