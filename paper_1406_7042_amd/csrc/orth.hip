// FP64 block Gram-Schmidt (CGS2) + CholQR2 with deflation; weighted
// tall-skinny products for the projection of eq. (R_and_Freduced).
#include <rocblas/rocblas.h>

#include <cmath>
#include <complex>
#include <mutex>
#include <string>
#include <vector>

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

thread_local DevBuf g_tmp, g_tmp2;

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

template <typename S>
int gram_host(const S* X, int64_t ld, int64_t n, int nb, std::vector<typename BT<S>::H>& G,
              hipStream_t s) {
  YR_CALL(g_tmp.reserve((size_t)nb * nb * sizeof(S)));
  YR_CALL(ts_gram<S>(X, ld, nb, X, ld, nb, n, g_tmp.as<S>(), nb, s));
  G.resize((size_t)nb * nb);
  YR_TRY_HIP(hipMemcpyAsync(G.data(), g_tmp.p, (size_t)nb * nb * sizeof(S), hipMemcpyDeviceToHost, s));
  YR_TRY_HIP(hipStreamSynchronize(s));
  return YR_OK;
}

}  // namespace

template <typename S>
int orth_block(S* Q, int64_t ld, int64_t n, int k, int nb, double defl, int* kept,
               std::vector<int>* keep_idx, hipStream_t s) {
  typedef typename BT<S>::H H;
  S* X = Q + (int64_t)k * ld;
  std::vector<H> G;
  YR_CALL(gram_host<S>(X, ld, n, nb, G, s));
  std::vector<double> n0(nb);
  for (int c = 0; c < nb; ++c) n0[c] = std::sqrt(std::max(0.0, BT<S>::re(G[c * nb + c])));
  if (k > 0) {
    YR_CALL(g_tmp2.reserve((size_t)k * nb * sizeof(S)));
    for (int pass = 0; pass < 2; ++pass) {  // classical Gram-Schmidt, twice
      YR_CALL(ts_gram<S>(Q, ld, k, X, ld, nb, n, g_tmp2.as<S>(), k, s));
      YR_CALL(ts_update<S>(Q, ld, k, g_tmp2.as<S>(), k, X, ld, nb, n, s));
    }
  }
  YR_CALL(gram_host<S>(X, ld, n, nb, G, s));
  // greedy Cholesky with deflation (column order), G column-major
  std::vector<int> K;
  std::vector<H> R((size_t)nb * nb, H(0));  // R[j + c*nb] for kept j (in kept order)
  for (int c = 0; c < nb; ++c) {
    std::vector<H> col(K.size());
    double d = BT<S>::re(G[c + c * nb]);
    for (size_t a = 0; a < K.size(); ++a) {
      H v = G[K[a] + c * nb];
      for (size_t b = 0; b < a; ++b) v -= BT<S>::cj(R[b + K[a] * nb]) * col[b];
      v /= R[a + K[a] * nb];
      col[a] = v;
      d -= BT<S>::absq(v);
    }
    if (!(d > 0) || std::sqrt(d) <= defl * n0[c] || n0[c] == 0) continue;  // deflate
    for (size_t a = 0; a < K.size(); ++a) R[a + c * nb] = col[a];
    R[K.size() + c * nb] = H(std::sqrt(d));
    K.push_back(c);
  }
  const int nk = (int)K.size();
  *kept = nk;
  if (keep_idx) *keep_idx = K;
  if (nk == 0) return YR_OK;
  // compact kept columns to the front of the block; R in kept order
  std::vector<H> Rk((size_t)nk * nk, H(0));
  for (int a = 0; a < nk; ++a) {
    if (K[a] != a)
      YR_TRY_HIP(hipMemcpyAsync(X + (int64_t)a * ld, X + (int64_t)K[a] * ld, n * sizeof(S),
                                hipMemcpyDeviceToDevice, s));
    for (int b = 0; b <= a; ++b) Rk[b + a * nk] = R[b + K[a] * nb];
  }
  YR_CALL(g_tmp.reserve((size_t)nk * nk * sizeof(S)));
  YR_TRY_HIP(hipMemcpyAsync(g_tmp.p, Rk.data(), (size_t)nk * nk * sizeof(S), hipMemcpyHostToDevice, s));
  YR_CALL(ts_trsm<S>(g_tmp.as<S>(), X, ld, nk, n, s));
  // second CholQR pass (no deflation)
  YR_CALL(gram_host<S>(X, ld, n, nk, G, s));
  std::vector<H> R2((size_t)nk * nk, H(0));
  for (int c = 0; c < nk; ++c) {
    for (int a = 0; a <= c; ++a) {
      H v = G[a + c * nk];
      for (int b = 0; b < a; ++b) v -= BT<S>::cj(R2[b + a * nk]) * R2[b + c * nk];
      if (a < c) {
        R2[a + c * nk] = v / R2[a + a * nk];
      } else {
        double d = BT<S>::re(v);
        YR_REQUIRE(d > 0, YR_EINVAL, "CholQR2: second pass lost positive definiteness");
        R2[c + c * nk] = H(std::sqrt(d));
      }
    }
  }
  YR_CALL(g_tmp.reserve((size_t)nk * nk * sizeof(S)));
  YR_TRY_HIP(hipMemcpyAsync(g_tmp.p, R2.data(), (size_t)nk * nk * sizeof(S), hipMemcpyHostToDevice, s));
  YR_CALL(ts_trsm<S>(g_tmp.as<S>(), X, ld, nk, n, s));
  YR_TRY_HIP(hipStreamSynchronize(s));
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
                                std::vector<int>*, hipStream_t);
template int orth_block<zd>(zd*, int64_t, int64_t, int, int, double, int*, std::vector<int>*,
                            hipStream_t);
}  // namespace yr
