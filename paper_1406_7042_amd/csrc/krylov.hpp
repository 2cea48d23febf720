// Shifted solves of the reduction (Sec. IV-B) on the device.
#pragma once

#include "common.hpp"
#include "cplx.hpp"
#include "stencil.hpp"

namespace yr {

// Per-column scalars of the batched COCG iteration.
struct ColState {
  double rho_re, rho_im;    // r^T r (bilinear)
  double alpha_re, alpha_im;
  double beta_re, beta_im;
  double rr;                // ||r||^2
  double bb;                // ||b||^2
  int status;               // 0 active, 1 converged, 2 breakdown
  int iters;
  double alpha1_re, alpha1_im;  // alpha used by the column's latest pass (delayed x update)
};

// Workspace of one expansion point: the Schur operator
//   S = A11 - A12 A22^{-1} A21 = W_e [a11 - z curl_d(a22^{-1} cp(.))]
// with a11 = (z-1) eps/dt + (z+1) sigma_e/2, a22 = (z-1) mu/dt + (z+1) sigma_m/2
// (field form of eqs. (reduced_linear_system_solution1/2)).
template <typename T>
struct SchurOp {
  const yr_operator* op;
  double dt;
  zd z;
  DevBuf a11;       // cplx<T>[nE]
  DevBuf a11r;      // T[nE], real part of a11 (real shifts only)
  DevBuf a22inv;    // cplx<T>[nH] (non-uniform magnetic materials only)
  cplx<T> a22inv_s; // uniform case
  int prepare(const yr_operator* o, double dt_, zd z_, hipStream_t s);
};

struct SolveOpts {
  double tol = 1e-4;   // normalized residual ||b - S x|| / ||b|| (Sec. IV-B)
  int max_iter = 5000;
  int check_every = 8;
  int matvec = 0;  // 0: automatic, 1: two sweeps, 2: one pass where it exists
};

struct SolveStats {
  int iters = 0;          // iterations of the batch
  int col_iters_max = 0;
  double relres_max = 0;  // ||r|| / ||b|| over the columns at exit
  int64_t matvecs = 0;    // column matvecs (one per column per iteration)
};

// Solve S X1 = Bhat for nb columns (E-vectors, ld = nE), X1 overwritten.
template <typename T>
int cocg_solve(const SchurOp<T>& S, const cplx<T>* bhat, cplx<T>* x1, int nb,
               const SolveOpts& o, SolveStats& st, hipStream_t s);

// g = (pm * v2 * hscale - cp(v1)) * a22^{-1}, pm = mu/dt + sigma_m/2 (H-vectors).
// v: FP64 complex full vectors (E rows then H rows, ld = nE + nH).
template <typename T>
int rhs_magnetic(const SchurOp<T>& S, const zd* v, int64_t ldv, double hscale, int nb,
                 cplx<T>* g, hipStream_t s);

// bhat = W_e (pe * v1 + curl_d(g)), pe = eps/dt + sigma_e/2.
template <typename T>
int rhs_electric(const SchurOp<T>& S, const zd* v, int64_t ldv, const cplx<T>* g, int nb,
                 cplx<T>* bhat, hipStream_t s);

// x2 = g + z a22^{-1} cp(x1)  (g may be null), then pack [x1; hscale_inv * x2]
// into FP64 complex full vectors out (ld = nE + nH).
template <typename T>
int recover_pack(const SchurOp<T>& S, const cplx<T>* x1, const cplx<T>* g, int nb,
                 double hs_out, zd* out, int64_t ldo, hipStream_t s);

// Frees the solver's cached vector workspace (it grows to the largest batch
// solved on this thread and is kept between calls otherwise).
void cocg_release_workspace();

// Apply S to nb columns (testing hook).
template <typename T>
int schur_apply(const SchurOp<T>& S, const cplx<T>* x, cplx<T>* y, int nb, hipStream_t s);

}  // namespace yr
