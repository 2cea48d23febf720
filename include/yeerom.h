/*
 * yeerom — structure-preserving reduction of Yee FDTD equations on AMD
 * Instinct MI355X (gfx950).  C ABI of libyeerom.so.
 *
 * Li, Sarris, Triverio, "Structure-Preserving Reduction of Finite-Difference
 * Time-Domain Equations with Controllable Stability Beyond the CFL Limit"
 * (arXiv 1406.7042).
 *
 * General rules
 *  - Every call returns a yr_status; 0 is success, negative is an error and
 *    yr_last_error() (thread-local) holds a message.  No C++ exception ever
 *    crosses this interface.
 *  - "host" pointers are ordinary CPU memory, "device" pointers are HIP
 *    device memory of the current device (for example torch tensor storage).
 *    The caller owns every buffer it passes in; the library never frees them.
 *    Objects created by the library (yr_operator, yr_rom) are freed by their
 *    *_destroy call.
 *  - Calls that take a `stream` (a hipStream_t, NULL = the null stream)
 *    are asynchronous with respect to the host; all others are synchronous.
 *  - Calls on the same yr_operator or yr_rom must not overlap.
 *
 * Field layout on the device
 *  A grid of nx x ny x nz cells (dim 2: Ez-polarisation, nz = 1) is a PEC
 *  box.  Every field component lives in a padded array of
 *      len = (nx+1) * (ny+1) * (nz+1)      (dim 2: (nx+1) * (ny+1))
 *  entries, index ((k*(ny+1) + j)*(nx+1) + i).  Sample (i,j,k) of each
 *  component sits at the Yee position
 *      Ex (i+1/2, j, k)   Ey (i, j+1/2, k)   Ez (i, j, k+1/2)
 *      Hx (i, j+1/2, k+1/2)  Hy (i+1/2, j, k+1/2)  Hz (i+1/2, j+1/2, k)
 *  (dim 2: Ez at node (i,j), Hx at (i, j+1/2), Hy at (i+1/2, j)).
 *  A field buffer holds the components one after the other:
 *      dim 3: Ex, Ey, Ez, Hx, Hy, Hz   (6 * len values)
 *      dim 2: Ez, Hx, Hy               (3 * len values)
 *  Entries that are not unknowns of eq. (matrix) (tangential E and normal H
 *  on the walls, E on PEC objects, the unused padding) are zero and stay
 *  zero.  Electric vectors of the reduction use the electric half only
 *  (3*len or len values), magnetic vectors the magnetic half.
 *
 * Matrix form.  eq. (matrix) of the paper holds on these samples with
 *  D_eps = eps_e W_e, D_sigma_e = sigma_e W_e, D_mu = mu_f W_f,
 *  D_sigma_m = sigma_m W_f and -K H = W_e (curl H), K^T E = -W_f (curl E),
 *  where eps_e, sigma_e (mu_f, sigma_m) are per-cell values averaged onto
 *  each electric (magnetic) sample with dual-area (dual-length) weights,
 *  and W_e = dual area x primal length / V0, W_f = primal area x dual
 *  length / V0 with V0 the volume of cell (0,0,0).  On a uniform grid all
 *  weights are 1: D_eps holds eps per sample and K holds +-1/Delta exactly
 *  as in Sec. II-A.  The source matrix B has entry weight*W_e at each port
 *  sample, the probe matrix L the plain weight.
 */
#ifndef YEEROM_H
#define YEEROM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  YR_OK = 0,
  YR_EINVAL = -1,     /* bad argument (sizes, pointers, ports off the grid) */
  YR_ENOMEM = -2,     /* device allocation failed */
  YR_EUNSTABLE = -3,  /* time step violates a stability condition */
  YR_ENOCONV = -4,    /* iterative solver missed its tolerance */
  YR_EDEVICE = -5,    /* HIP runtime error */
  YR_ESTATE = -6      /* object not prepared for this call (see rom_step) */
} yr_status;

typedef enum { YR_F32 = 0, YR_F64 = 1 } yr_dtype;

/* PEC box of nx*ny*nz cells.  dx, dy, dz: host arrays of the nx, ny, nz cell
 * spacings in metres (dim 2: dz may be NULL, nz must be 1). */
typedef struct {
  int32_t dim;
  int32_t nx, ny, nz;
  const double* dx;
  const double* dy;
  const double* dz;
} yr_grid;

/* Per-cell materials, host FP64 arrays of nx*ny*nz values, index
 * (k*ny + j)*nx + i.  NULL means eps_r = 1, sigma_e = 0, mu_r = 1,
 * sigma_m = 0.  pec: n_pec quadruples (c, i, j, k) of electric samples
 * (c = 0,1,2 for Ex,Ey,Ez) that lie on perfectly conducting objects; they are
 * removed from the unknowns (held at zero). */
typedef struct {
  const double* eps_r;
  const double* sigma_e;
  const double* mu_r;
  const double* sigma_m;
  int64_t n_pec;
  const int32_t* pec;
} yr_materials;

/* n ports, each a list of electric samples: entries offset[p] .. offset[p+1]-1
 * of sample (4 int32 per entry: c, i, j, k) and weight.  Host memory. */
typedef struct {
  int32_t n;
  const int32_t* offset;
  const int32_t* sample;
  const double* weight;
} yr_ports;

/* ---------------------------------------------------------------- operator */

typedef struct yr_operator yr_operator;

/* Discretise one structure (Sec. II-A, eq. (matrix)): averages the per-cell
 * materials onto the Yee samples and keeps D_eps, D_sigma_e, D_mu,
 * D_sigma_m and the grid spacings resident on the current device.  The grid
 * and materials are copied; the caller may free them afterwards.
 * Errors: YR_EINVAL for a malformed grid or PEC list, YR_ENOMEM. */
int yr_operator_create(const yr_grid* grid, const yr_materials* mat, yr_operator** out);
void yr_operator_destroy(yr_operator* op);

/* len: entries per component array; n_e, n_h: unknown counts N_e, N_h of
 * eq. (x); dt_max: the CFL limit eq. (CFL) with the vacuum speed of light and
 * the smallest spacings. */
int yr_operator_info(const yr_operator* op, int64_t* len, int64_t* n_e, int64_t* n_h,
                     double* dt_max);

/* --------------------------------------------------------- full-order FDTD */

/* fdtd_step — nsteps of the Yee leapfrog, eq. (MNAform) (eqs. (FDTD1/2) in
 * 3-D): per step
 *   (De/dt + Dse/2) E^{n+1} = (De/dt - Dse/2) E^n - K H^{n+1/2} + B u^{n+1}
 *   (Dm/dt + Dsm/2) H^{n+3/2} = (Dm/dt - Dsm/2) H^{n+1/2} + K^T E^{n+1}
 * fields: device, dtype, the field buffer (layout above), updated in place.
 * src:    host port list (may be NULL), u: device, dtype, [nsteps][src->n];
 *         u[n][p] drives the update that produces E^{n+1}.
 * probes: host port list (may be NULL), y: device, dtype, [nsteps][probes->n];
 *         y[n][p] = sum over entries of weight * E^{n+1}.
 * Errors: YR_EUNSTABLE if dt > dt_max (1 + 1e-12) (condition (Dstability2)
 * fails beyond eq. (CFL)); YR_EINVAL for bad ports or sizes. */
int fdtd_step(yr_operator* op, yr_dtype dtype, double dt, int64_t nsteps, void* fields,
              const yr_ports* src, const void* u, const yr_ports* probes, void* y,
              void* stream);

#ifdef __cplusplus
}
#endif

#endif /* YEEROM_H */
