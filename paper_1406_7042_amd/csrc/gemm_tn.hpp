// Tall-skinny FP64 products on the matrix cores (gemm_tn.hip).
#pragma once

#include "common.hpp"

namespace yr {

// C (m x m, column-major, ldc) = A^T diag(w) A over n rows; A: n x m (lda),
// w: n weights or null (identity); all on the device; 1 <= m <= 256.  Only
// the tiles on and above the diagonal are computed, then mirrored.
// Asynchronous on stream s.
int gram_mfma(const double* A, int64_t lda, int m, const double* w, int64_t n, double* C, int ldc,
              hipStream_t s);

// C (m x nc, column-major, ldc) = A^T diag(w) B over n rows; A: n x m (lda),
// B: n x nc (ldb); 1 <= m, nc <= 256.  Asynchronous on stream s.
int gemm_tn_mfma(const double* A, int64_t lda, int m, const double* B, int64_t ldb, int nc,
                 const double* w, int64_t n, double* C, int ldc, hipStream_t s);

// U = R^-1 for upper triangular R (r x r, column-major, ld r, device); U is
// written whole (zeros below the diagonal); 1 <= r <= 256.  Asynchronous.
int tri_inv_upper(const double* R, int r, double* U, hipStream_t s);

// X <- X U in place for X: n x r (column-major, ldx) and upper triangular U
// (r x r, ld r; only its upper triangle is read); 1 <= r <= 256.  Asynchronous.
int trmm_upper_inplace(double* X, int64_t ldx, int r, const double* U, int64_t n, hipStream_t s);

}  // namespace yr
