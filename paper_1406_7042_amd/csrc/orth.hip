// FP64 block Gram-Schmidt (CGS2) + CholQR2 with deflation (device-side
// factorisations); Gram-based CholQR2 of whole bases; weighted tall-skinny
// products for the projection of eq. (R_and_Freduced).
#include <rocblas/rocblas.h>

#include <cmath>
#include <complex>
#include <mutex>
#include <string>
#include <vector>

#include "gemm_tn.hpp"
#include "orth.hpp"
#include "tsqr.hpp"

namespace yr {

namespace {
std::mutex g_blas_mu;
rocblas_handle g_blas = nullptr;

int blas(rocblas_handle* h, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_blas_mu);
  if (!g_blas) {
    if (rocblas_create_handle(&g_blas) != rocblas_status_success) {
      set_error("rocblas_create_handle failed");
      return YR_EDEVICE;
    }
  }
  if (rocblas_set_stream(g_blas, s) != rocblas_status_success) {
    set_error("rocblas_set_stream failed");
    return YR_EDEVICE;
  }
  *h = g_blas;
  return YR_OK;
}

#define YR_TRY_BLAS(expr)                                                \
  do {                                                                   \
    rocblas_status b_ = (expr);                                          \
    if (b_ != rocblas_status_success) {                                  \
      set_error(std::string(#expr " failed: ") + rocblas_status_to_string(b_)); \
      return YR_EDEVICE;                                                 \
    }                                                                    \
  } while (0)

thread_local DevBuf g_tmp, g_tmp2, g_r, g_flags, g_vout;

// ---- type traits over double / complex<double>
template <typename S>
struct BT;

template <>
struct BT<double> {
  typedef double H;  // host type
  static rocblas_operation adj() { return rocblas_operation_transpose; }
  static rocblas_status gemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m,
                             int n, int k, double alpha, const double* A, int64_t lda,
                             const double* B, int64_t ldb, double beta, double* C, int64_t ldc) {
    return rocblas_dgemm(h, ta, tb, m, n, k, &alpha, A, (int)lda, B, (int)ldb, &beta, C, (int)ldc);
  }
  static rocblas_status trsm(rocblas_handle h, int m, int n, const double* R, int ldr, double* X,
                             int64_t ldx) {
    double one = 1.0;
    return rocblas_dtrsm(h, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none,
                         rocblas_diagonal_non_unit, m, n, &one, R, ldr, X, (int)ldx);
  }
  static double absq(H v) { return v * v; }
  static H cj(H v) { return v; }
  static double re(H v) { return v; }
};

template <>
struct BT<zd> {
  typedef std::complex<double> H;
  static rocblas_operation adj() { return rocblas_operation_conjugate_transpose; }
  static rocblas_status gemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m,
                             int n, int k, double alpha, const zd* A, int64_t lda, const zd* B,
                             int64_t ldb, double beta, zd* C, int64_t ldc) {
    rocblas_double_complex a = {alpha, 0.0}, b = {beta, 0.0};
    return rocblas_zgemm(h, ta, tb, m, n, k, &a, (const rocblas_double_complex*)A, (int)lda,
                         (const rocblas_double_complex*)B, (int)ldb, &b,
                         (rocblas_double_complex*)C, (int)ldc);
  }
  static rocblas_status trsm(rocblas_handle h, int m, int n, const zd* R, int ldr, zd* X,
                             int64_t ldx) {
    rocblas_double_complex one = {1.0, 0.0};
    return rocblas_ztrsm(h, rocblas_side_right, rocblas_fill_upper, rocblas_operation_none,
                         rocblas_diagonal_non_unit, m, n, &one, (const rocblas_double_complex*)R,
                         ldr, (rocblas_double_complex*)X, (int)ldx);
  }
  static double absq(H v) { return std::norm(v); }
  static H cj(H v) { return std::conj(v); }
  static double re(H v) { return v.real(); }
};

// ---- small factorisations on the device (one workgroup)

inline double abs2(double v) { return v * v; }
inline double abs2(const zd& v) { return v.re * v.re + v.im * v.im; }
inline double re_part(double v) { return v; }
inline double re_part(const zd& v) { return v.re; }
__device__ inline double re_of(double v) { return v; }
__device__ inline double re_of(zd v) { return v.re; }
__device__ inline double cj_of(double v) { return v; }
__device__ inline zd cj_of(zd v) { return conj(v); }
__device__ inline double scale_by(double v, double s) { return v * s; }
__device__ inline zd scale_by(zd v, double s) { return zd(v.re * s, v.im * s); }

// Right-looking Cholesky G = R^H R of a c x c Hermitian Gram matrix (device,
// column-major, overwritten) in column order with deflation: column k is
// dropped when its Schur-complement diagonal (its squared norm after
// projection on the kept earlier columns) is not above (defl n0_k)^2, with
// n0_k = sqrt(G0[k + k ld0]) its norm before any orthogonalisation (G0 null:
// no deflation; a non-positive pivot is then a failure).  A dropped column
// contributes no update, which is the same as removing it from the set.
// Outputs: keep[k] (1 kept), st[0] = kept count r, st[1] = 1 on failure, and
// R (r x r, column-major, upper) over the kept columns in order.
template <typename S>
__global__ void __launch_bounds__(1024)
    k_chol_deflate(S* __restrict__ G, int c, const S* __restrict__ G0, int ld0, double defl,
                   S* __restrict__ R, int* __restrict__ keep, int* __restrict__ st) {
  __shared__ int ok;
  __shared__ int kept_idx[1024];
  __shared__ int nkept;
  const int tid = threadIdx.x, bs = blockDim.x;
  if (tid == 0) st[1] = 0;
  for (int k = 0; k < c; ++k) {
    if (tid == 0) {
      const double d = re_of(G[k + (int64_t)k * c]);
      int good = d > 0;
      if (G0) {
        const double n0 = sqrt(fmax(0.0, re_of(G0[k + (int64_t)k * ld0])));
        good = good && n0 > 0 && sqrt(d) > defl * n0;
      } else if (!good) {
        st[1] = 1;
      }
      keep[k] = good;
      if (good) G[k + (int64_t)k * c] = S(sqrt(d));
      ok = good;
    }
    __syncthreads();
    if (!ok) continue;
    const double inv = 1.0 / re_of(G[k + (int64_t)k * c]);
    for (int j = k + 1 + tid; j < c; j += bs) G[k + (int64_t)j * c] = scale_by(G[k + (int64_t)j * c], inv);
    __syncthreads();
    const int m = c - k - 1;
    for (int t = tid; t < m * m; t += bs) {
      const int i = k + 1 + t % m, j = k + 1 + t / m;
      if (i <= j) G[i + (int64_t)j * c] = G[i + (int64_t)j * c] - cj_of(G[k + (int64_t)i * c]) * G[k + (int64_t)j * c];
    }
    __syncthreads();
  }
  if (tid == 0) {
    int r = 0;
    for (int k = 0; k < c; ++k)
      if (keep[k]) kept_idx[r++] = k;
    nkept = r;
    st[0] = r;
  }
  __syncthreads();
  const int r = nkept;
  for (int t = tid; t < r * r; t += bs) {
    const int a = t % r, b = t / r;
    R[t] = a <= b ? G[kept_idx[a] + (int64_t)kept_idx[b] * c] : S(0);
  }
}

// deflating Cholesky of the device Gram G (c x c) -> compact R on the device;
// returns the kept count and the kept flags (host)
template <typename S>
static int chol_device(S* G, int c, const S* G0, int ld0, double defl, S* R,
                       std::vector<int>& keep, int* kept, hipStream_t s) {
  YR_REQUIRE(c <= 1024, YR_EINVAL, "more than 1024 columns in one factorisation");
  YR_CALL(g_flags.reserve(((size_t)c + 2) * sizeof(int)));
  int* dkeep = g_flags.as<int>();
  k_chol_deflate<S><<<1, 1024, 0, s>>>(G, c, G0, ld0, defl, R, dkeep + 2, dkeep);
  YR_TRY_HIP(hipGetLastError());
  std::vector<int> h((size_t)c + 2);
  YR_TRY_HIP(hipMemcpyAsync(h.data(), dkeep, ((size_t)c + 2) * sizeof(int), hipMemcpyDeviceToHost, s));
  YR_TRY_HIP(hipStreamSynchronize(s));
  YR_REQUIRE(h[1] == 0, YR_EINVAL, "CholQR: Gram matrix lost positive definiteness");
  keep.assign(h.begin() + 2, h.end());
  *kept = h[0];
  return YR_OK;
}

// move the kept columns of X (n rows, ld) to the front, in order
template <typename S>
static int compact_columns(S* X, int64_t ld, int64_t n, const std::vector<int>& keep,
                           hipStream_t s) {
  int a = 0;
  for (int c = 0; c < (int)keep.size(); ++c) {
    if (!keep[c]) continue;
    if (c != a)
      YR_TRY_HIP(hipMemcpyAsync(X + (int64_t)a * ld, X + (int64_t)c * ld, n * sizeof(S),
                                hipMemcpyDeviceToDevice, s));
    ++a;
  }
  return YR_OK;
}

}  // namespace

template <typename S>
int orth_block(S* Q, int64_t ld, int64_t n, int k, int nb, double defl, int* kept,
               std::vector<int>* keep_idx, int max_passes, hipStream_t s) {
  S* X = Q + (int64_t)k * ld;
  // the Gram of the block before orthogonalisation (reference norms for
  // deflation) comes with the first projection: [Q X]^H X, one pass over X
  YR_CALL(g_tmp2.reserve((size_t)(k + nb) * nb * sizeof(S)));
  S* C = g_tmp2.as<S>();  // (k + nb) x nb: Q^H X, then X^H X in rows k..k+nb-1
  const int ldc = k + nb;
  const S* G0 = C + k;
  YR_CALL(ts_gram<S>(Q, ld, k + nb, X, ld, nb, n, C, ldc, s));
  if (k > 0) {
    // classical Gram-Schmidt; a second pass (DGKS criterion) only when the
    // first removed more than half of some column's squared norm: with Q
    // orthonormal, ||x - Q c||^2 = ||x||^2 - ||c||^2 (c = Q^H x), so the test
    // needs the coefficients and the Gram diagonal only
    YR_CALL(ts_update<S>(Q, ld, k, C, ldc, X, ld, nb, n, s));
    bool again = false;
    if (max_passes > 1) {
      std::vector<S> hc((size_t)ldc * nb);
      YR_TRY_HIP(hipMemcpyAsync(hc.data(), C, hc.size() * sizeof(S), hipMemcpyDeviceToHost, s));
      YR_TRY_HIP(hipStreamSynchronize(s));
      for (int j = 0; j < nb && !again; ++j) {
        double cc = 0;
        for (int i = 0; i < k; ++i) cc += abs2(hc[i + (size_t)j * ldc]);
        again = cc > 0.5 * re_part(hc[k + j + (size_t)j * ldc]);
      }
    }
    if (again) {  // C's rows 0..k-1 are overwritten, G0 (rows k..) is kept
      YR_CALL(ts_gram<S>(Q, ld, k, X, ld, nb, n, C, ldc, s));
      YR_CALL(ts_update<S>(Q, ld, k, C, ldc, X, ld, nb, n, s));
    }
  }
  // CholQR with deflation (device factorisation)
  YR_CALL(g_tmp.reserve((size_t)nb * nb * sizeof(S)));
  YR_CALL(g_r.reserve((size_t)nb * nb * sizeof(S)));
  YR_CALL(ts_gram<S>(X, ld, nb, X, ld, nb, n, g_tmp.as<S>(), nb, s));
  std::vector<int> keep;
  int nk = 0;
  YR_CALL(chol_device<S>(g_tmp.as<S>(), nb, G0, ldc, defl, g_r.as<S>(), keep, &nk, s));
  *kept = nk;
  if (keep_idx) {
    keep_idx->clear();
    for (int c = 0; c < nb; ++c)
      if (keep[c]) keep_idx->push_back(c);
  }
  if (nk == 0) return YR_OK;
  YR_CALL(compact_columns<S>(X, ld, n, keep, s));
  YR_CALL(ts_trsm<S>(g_r.as<S>(), X, ld, nk, n, s));
  // second CholQR pass (no deflation)
  YR_CALL(ts_gram<S>(X, ld, nk, X, ld, nk, n, g_tmp.as<S>(), nk, s));
  std::vector<int> keep2;
  int nk2 = 0;
  YR_CALL(chol_device<S>(g_tmp.as<S>(), nk, (const S*)nullptr, 0, 0.0, g_r.as<S>(), keep2, &nk2, s));
  YR_CALL(ts_trsm<S>(g_r.as<S>(), X, ld, nk, n, s));
  YR_TRY_HIP(hipStreamSynchronize(s));
  return YR_OK;
}

int cholqr2_columns(DevBuf& Vb, int64_t n, int c, double defl, int* kept, hipStream_t s) {
  *kept = 0;
  if (c == 0) return YR_OK;
  DevBuf G, G0, R, Ri;
  YR_CALL(G.reserve((size_t)c * c * 8));
  YR_CALL(G0.reserve((size_t)c * c * 8));
  YR_CALL(R.reserve((size_t)c * c * 8));
  YR_CALL(Ri.reserve((size_t)c * c * 8));
  // up to 256 columns: V R^-1 in place on the matrix cores; wider bases go
  // out of place through rocBLAS (TRTRI + DGEMM into a second buffer)
  const bool native = c <= 256;
  rocblas_handle h = nullptr;
  if (!native) {
    YR_REQUIRE(n < (int64_t)1 << 31, YR_EINVAL, "vector length exceeds the 32-bit BLAS interface");
    YR_CALL(blas(&h, s));
    YR_CALL(g_vout.reserve((size_t)n * c * 8));
  }
  const double one = 1.0, zero = 0.0;
  int r = c;
  for (int pass = 0; pass < 2; ++pass) {
    double* V = Vb.as<double>();
    YR_CALL(gemm_tn_weighted(V, n, r, V, n, r, nullptr, n, G.as<double>(), r, s));
    std::vector<int> keep;
    int nk = 0;
    if (pass == 0) {
      YR_TRY_HIP(hipMemcpyAsync(G0.p, G.p, (size_t)r * r * 8, hipMemcpyDeviceToDevice, s));
      YR_CALL(chol_device<double>(G.as<double>(), r, G0.as<double>(), r, defl, R.as<double>(), keep, &nk, s));
      if (nk == 0) return YR_OK;
      YR_CALL(compact_columns<double>(V, n, n, keep, s));
    } else {
      YR_CALL(chol_device<double>(G.as<double>(), r, (const double*)nullptr, 0, 0.0, R.as<double>(), keep, &nk, s));
    }
    r = nk;
    if (native) {
      // V R^-1 = V (R^-1): the explicit inverse of the r x r factor, then the
      // triangular product over the rows in place
      YR_CALL(tri_inv_upper(R.as<double>(), r, Ri.as<double>(), s));
      YR_CALL(trmm_upper_inplace(V, n, r, Ri.as<double>(), n, s));
    } else {
      YR_TRY_HIP(hipMemsetAsync(Ri.p, 0, (size_t)r * r * 8, s));  // strict lower part stays zero
      YR_TRY_BLAS(rocblas_dtrtri(h, rocblas_fill_upper, rocblas_diagonal_non_unit, r,
                                 R.as<double>(), r, Ri.as<double>(), r));
      YR_TRY_BLAS(rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, (int)n, r, r,
                                &one, V, (int)n, Ri.as<double>(), r, &zero,
                                g_vout.as<double>(), (int)n));
      Vb.swap(g_vout);
    }
  }
  YR_TRY_HIP(hipStreamSynchronize(s));
  *kept = r;
  return YR_OK;
}

__global__ void k_row_scale(double* __restrict__ out, const double* __restrict__ B, int64_t ldb,
                            const double* __restrict__ w, int64_t n, int nc) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= n) return;
  double wv = w[g];
  for (int c = 0; c < nc; ++c) out[c * n + g] = wv * B[c * ldb + g];
}

int gemm_tn_weighted(const double* A, int64_t lda, int m, const double* B, int64_t ldb, int nc,
                     const double* w, int64_t n, double* C, int ldc, hipStream_t s) {
  // Gram matrices A^T diag(w) A of up to 256 columns: the matrix-core kernel
  // (weights fused, upper tiles only)
  if (A == B && lda == ldb && m == nc && m > 0 && m <= 256 && n > 0)
    return gram_mfma(A, lda, m, w, n, C, ldc, s);
  // products of up to 256 x 256 columns: the same kernel with two operands
  if (m > 0 && m <= 256 && nc > 0 && nc <= 256 && n > 0)
    return gemm_tn_mfma(A, lda, m, B, ldb, nc, w, n, C, ldc, s);
  YR_REQUIRE(n < (int64_t)1 << 31 && lda < (int64_t)1 << 31, YR_EINVAL,
             "vector length exceeds the 32-bit BLAS interface");
  rocblas_handle h;
  YR_CALL(blas(&h, s));
  const double* Bp = B;
  int64_t ldbp = ldb;
  if (w) {
    YR_CALL(g_tmp2.reserve((size_t)n * nc * sizeof(double)));
    k_row_scale<<<grid_for(n), kBlock, 0, s>>>(g_tmp2.as<double>(), B, ldb, w, n, nc);
    YR_TRY_HIP(hipGetLastError());
    Bp = g_tmp2.as<double>();
    ldbp = n;
  }
  YR_TRY_BLAS(BT<double>::gemm(h, rocblas_operation_transpose, rocblas_operation_none, m, nc,
                               (int)n, 1.0, A, lda, Bp, ldbp, 0.0, C, ldc));
  return YR_OK;
}

template int orth_block<double>(double*, int64_t, int64_t, int, int, double, int*,
                                std::vector<int>*, int, hipStream_t);
template int orth_block<zd>(zd*, int64_t, int64_t, int, int, double, int*, std::vector<int>*,
                            int, hipStream_t);
}  // namespace yr
