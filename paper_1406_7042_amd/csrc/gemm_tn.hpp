// Tall-skinny FP64 Gram C = A^T diag(w) A on the matrix cores (gemm_tn.hip).
#pragma once

#include "common.hpp"

namespace yr {

// C (m x m, column-major, ldc) = A^T diag(w) A over n rows; A: n x m (lda),
// w: n weights or null (identity); all on the device; 1 <= m <= 256.  Only
// the tiles on and above the diagonal are computed, then mirrored.
// Asynchronous on stream s.
int gram_mfma(const double* A, int64_t lda, int m, const double* w, int64_t n, double* C, int ldc,
              hipStream_t s);

}  // namespace yr
