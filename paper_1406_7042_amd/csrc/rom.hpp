// Reduced model object shared by mor_reduce, rom_perturb and rom_step.
#pragma once

#include <vector>

#include "common.hpp"

struct yr_rom {
  int q1 = 0, q2 = 0;  // columns of V1, V2 (reduced orders of the two blocks)
  int nsrc = 0, nprb = 0;
  // projection basis (device FP64, padded layout); empty for models given as matrices
  yr::DevBuf V1, V2;
  int64_t nE = 0, nH = 0;
  // reduced matrices of eq. (R_and_Freduced), host FP64, column-major
  std::vector<double> De, Dse, Dm, Dsm, K, Kp, B1, B2, L1, L2;
  std::vector<double> sigma;  // singular values of De^-1/2 K Dm^-1/2 (after rom_perturb)
  // reduction statistics
  int deflated = 0;
  int64_t solve_iters = 0, matvecs = 0;
  double relres_max = 0;
  double seconds_solve = 0, seconds_orth = 0, seconds_project = 0;
  // stepping data, prepared by rom_perturb for one dt / dtype
  double step_dt = -1;
  int step_dtype = -1;
  int n_clamped = 0;
  double guard_margin = 0;  // smallest eigenvalue of 4I - M^T M (the stability certificate)
  yr::DevBuf A;             // q1 x q2, row-major with rows padded to ld_a (dtype)
  yr::DevBuf AT;            // q2 x q1 (A transposed), row-major with rows padded to ld_at
  int ld_a = 0, ld_at = 0;  // multiples of 16 bytes / element size (vector loads)
  yr::DevBuf vec;           // ce[q1] ge[q1] cm[q2] gm[q2] be[q1*nsrc] bh[q2*nsrc] oe[q1*nprb] oh[q2*nprb]
  yr::DevBuf scratch;       // FP64 workspace of rom_perturb
  yr::DevBuf lift;          // FP64 Te (q1 x q1) then Tm (q2 x q2), column-major:
                            // x~_e = Te s_e, x~_h = Tm s_h for stepping state s
};
