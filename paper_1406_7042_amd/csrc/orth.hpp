// Block orthogonalisation in FP64 (Sec. II-C, "robust Arnoldi"): classical
// Gram-Schmidt twice against an existing basis, then CholQR2 of the new block
// with rank deflation.  Tall-skinny products run in the kernels of tsqr.hip;
// the small Cholesky factorisations run in one workgroup on the device.
#pragma once

#include <vector>

#include "common.hpp"
#include "cplx.hpp"

namespace yr {

// Orthonormalise the nb columns at Q + k*ld against columns [0, k) of Q
// (orthonormal already), in place; deflated columns are dropped and the kept
// ones compacted.  A column is deflated when its norm after projection is
// below defl * (its norm before).  Returns the number of kept columns in *kept
// and their original indices in keep_idx.  max_passes: 1 = one classical
// Gram-Schmidt pass, 2 = a second one when the first removed more than half
// of a column's squared norm (DGKS).  S = double or zd.
template <typename S>
int orth_block(S* Q, int64_t ld, int64_t n, int k, int nb, double defl, int* kept,
               std::vector<int>* keep_idx, int max_passes, hipStream_t s);

// Orthonormalise the c columns of V (n rows, ld = n) by a deflating CholQR2
// on their FP64 Gram matrix: column k is dropped when its norm after
// projection on the kept earlier columns is not above defl times its own
// norm (resolvable for defl >~ 1e-7 in FP64), the kept ones are compacted to
// the front and orthonormalised (two passes).  *kept = their number.  Each
// pass forms V R^-1 with R^-1 explicit: in place on the matrix cores for up
// to 256 columns; for more, out of place (one DGEMM) into a second buffer of
// the same size, swapped with V (V's allocation changes).
int cholqr2_columns(DevBuf& V, int64_t n, int c, double defl, int* kept, hipStream_t s);

// C (m x nc, column-major, ldc) = A^T diag(w) B  over n rows (A: n x m, lda;
// B: n x nc, ldb); w may be null (identity).  FP64, C on the device.
int gemm_tn_weighted(const double* A, int64_t lda, int m, const double* B, int64_t ldb, int nc,
                     const double* w, int64_t n, double* C, int ldc, hipStream_t s);

}  // namespace yr
