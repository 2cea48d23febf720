// Tall-skinny FP64 kernels (Gram, update, triangular solve) for block
// Gram-Schmidt; S = double or cplx<double>.
#pragma once

#include "common.hpp"
#include "cplx.hpp"

namespace yr {

__host__ __device__ inline double cdiv_s(double a, double b) { return a / b; }
__host__ __device__ inline zd cdiv_s(zd a, zd b) { return cdiv(a, b); }

// C (m x nb, column-major, ldc, device) = A^H B over n rows.
template <typename S>
int ts_gram(const S* A, int64_t lda, int m, const S* B, int64_t ldb, int nb, int64_t n, S* C,
            int ldc, hipStream_t s);

// X (n x nb) -= Q (n x m) C (m x nb, device).
template <typename S>
int ts_update(const S* Q, int64_t ldq, int m, const S* C, int ldc, S* X, int64_t ldx, int nb,
              int64_t n, hipStream_t s);

// X (n x nb) = X R^-1, R upper triangular nb x nb (device, column-major).
template <typename S>
int ts_trsm(const S* R, S* X, int64_t ldx, int nb, int64_t n, hipStream_t s);

}  // namespace yr
