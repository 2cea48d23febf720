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

/* Message of the last failed call on this thread (empty if none). */
const char* yr_last_error(void);

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


/* Leapfrog path of fdtd_step on a 3-D operator (results agree to rounding):
 * 0 automatic (the default: one-pass steps for boxes of at least 64 x 16 x 16
 * cells, measured at least as fast there), 1 two half-step kernels per step
 * (fields updated in place), 2 one-pass steps (E and H of a step in one sweep, the fields
 * alternating with a second buffer the operator owns: 48 instead of 72 bytes
 * per cell and step in FP32).  2-D operators always take the two kernels.
 * Errors: YR_EINVAL. */
int yr_operator_set_leapfrog(yr_operator* op, int32_t mode);

/* ------------------------------------------------------------------ adjoint */

/* fdtd_adjoint — gradient of an objective J(y) of the probe outputs of
 * fdtd_step (same operator, dt, nsteps, sources, waveform u, probes, zero
 * initial fields) with respect to the per-cell eps_r and sigma_e.  Not in the
 * paper: the discrete adjoint of eq. (MNAform), (R+F)^T lambda^n =
 * (R-F)^T lambda^{n+1} + L dJ/dy^n, run backwards in time with the forward
 * states recomputed from checkpoints taken every ckpt_every steps (memory:
 * nsteps/ckpt_every field buffers + ckpt_every electric halves).
 * dJdy: device, dtype, [nsteps][probes->n], the derivative of J with respect
 * to y[n][p] (e.g. 2 dt y for J = dt sum y^2).
 * grad_eps_r, grad_sigma_e: device FP64 [nx*ny*nz] (index (k*ny+j)*nx+i),
 * overwritten.  Synchronous with respect to `stream`'s work on return.
 * Errors as fdtd_step. */
int fdtd_adjoint(yr_operator* op, yr_dtype dtype, double dt, int64_t nsteps, const yr_ports* src,
                 const void* u, const yr_ports* probes, const void* dJdy, int64_t ckpt_every,
                 double* grad_eps_r, double* grad_sigma_e, void* stream);

/* ---------------------------------------------------------------- reduction */

typedef struct yr_rom yr_rom;

/* Options of mor_reduce.  Expansion points z_l = M exp(j 2 pi (l/L) fmax dt_ref),
 * l = 0..L (eq. (distrib), Sec. IV-A; the conjugate points are covered by
 * the real split).  Each shifted system [z (R+F) - (R-F)] x = w (reading of
 * eq. (linear_system_solution): the resolvent of eq. (MNAform)) is solved
 * through its Schur complement (eqs. (reduced_linear_system_solution1/2))
 * by conjugate-orthogonal CG to the normalized residual `tol` (Sec. IV-B
 * uses 1e-4) in `solve_dtype` arithmetic.  Columns whose norm drops below
 * defl_tol times their norm before orthogonalisation are deflated. */
typedef struct {
  double M;          /* radius of the arc, 1.1 in Sec. V */
  int32_t L;         /* 2L+1 points */
  double fmax;       /* highest frequency of interest [Hz] */
  double dt_ref;     /* time step that places the points [s] */
  double tol;        /* normalized residual of the shifted solves */
  int32_t max_iter;  /* iteration cap per solve (YR_ENOCONV beyond it) */
  double defl_tol;   /* deflation threshold (relative) */
  yr_dtype solve_dtype;
  int32_t matvec;    /* Schur matvec kernel: 0 = automatic (the one-pass
                        iteration, H kept on chip, for 3-D grids with uniform
                        magnetic materials and for 2-D grids; two sweeps
                        otherwise; a 2-D block solve that reaches max_iter in
                        one pass is solved again with two sweeps), 1 = always
                        two sweeps through a stored H intermediate, 2 = the
                        one-pass iteration wherever it exists, no retry.  The
                        one-pass form takes the next r^T r from the previous
                        pass's sums and can need a few per cent more
                        iterations on hard solves. */
  int32_t pair_only; /* 0: the 2L+1 points of eq. (distrib).  1: only the
                        conjugate pair z = M exp(+-j 2 pi fmax dt_ref) of
                        Sec. V-C (single-frequency drive; L is ignored): all q
                        columns come from q/2 complex block moments at z, whose
                        real and imaginary parts cover z and its conjugate;
                        q must be a multiple of 2 * src->n. */
} yr_mor_opts;

/* mor_reduce — SPRIM reduction of eq. (MNAform), Sec. II-C and IV:
 * q real columns are generated, q/(2L+1) per point: z_0 gives real block
 * moments, each z_l (l >= 1) complex block moments whose real and imaginary
 * parts cover z_l and its conjugate.  Per point the block Krylov basis of
 * (z P - Q)^{-1} P started at (z P - Q)^{-1} B (P = R+F, Q = R-F) is
 * orthonormalised in FP64 (CGS2 + CholQR2, energy-balanced inner product);
 * its electric and magnetic rows are orthonormalised separately into V1 and
 * V2 (eq. (V)).  The reduced matrices of eq. (R_and_Freduced) are then
 * De~ = V1^T De V1, Dse~, Dm~, Dsm~, K~ = V1^T K V2, B~ = V^T B, L~ = V^T L,
 * accumulated in FP64.  They do not depend on any time step: one reduction
 * serves every dt (the points only use dt_ref).
 * src: the port list defining B (n >= 1, q a multiple of (2L+1) * src->n,
 *      or of 2 * src->n with opts->pair_only);
 * probes: the output list L (may be NULL).  Synchronous.  On success *out
 * is a new reduced model (free with yr_rom_destroy).
 * Errors: YR_EINVAL, YR_ENOMEM, YR_ENOCONV (a shifted solve missed tol). */
int mor_reduce(yr_operator* op, const yr_ports* src, const yr_ports* probes, int32_t q,
               const yr_mor_opts* opts, yr_rom** out);

typedef struct {
  int32_t q1, q2;      /* columns of V1 and V2 (reduced state size q1 + q2) */
  int32_t nsrc, nprb;
  int32_t deflated;    /* columns dropped by deflation */
  int64_t solve_iters; /* COCG iterations summed over the batches */
  int64_t matvecs;     /* Schur matvecs summed over the columns */
  double relres_max;   /* largest normalized residual at exit */
  double seconds_solve, seconds_orth, seconds_project;
  int32_t n_clamped;   /* after rom_perturb */
  double step_dt;      /* dt prepared by rom_perturb, -1 if none */
  double guard_margin; /* min eigenvalue of 4I - M^T M of the stepping matrices */
} yr_rom_info_t;

int yr_rom_info(const yr_rom* rom, yr_rom_info_t* info);

/* Reduced matrices, host FP64, column-major. */
typedef enum {
  YR_ROM_DE = 0,  /* q1 x q1  De~ */
  YR_ROM_DSE = 1, /* q1 x q1  Dse~ */
  YR_ROM_DM = 2,  /* q2 x q2  Dm~ */
  YR_ROM_DSM = 3, /* q2 x q2  Dsm~ */
  YR_ROM_K = 4,   /* q1 x q2  K~ */
  YR_ROM_KP = 5,  /* q1 x q2  K~' after rom_perturb (read only) */
  YR_ROM_B1 = 6,  /* q1 x nsrc */
  YR_ROM_B2 = 7,  /* q2 x nsrc */
  YR_ROM_L1 = 8,  /* q1 x nprb */
  YR_ROM_L2 = 9,  /* q2 x nprb */
  YR_ROM_SIGMA = 10 /* min(q1,q2) singular values of De~^-1/2 K~ Dm~^-1/2 (read only) */
} yr_rom_matrix;

int yr_rom_get(const yr_rom* rom, int32_t which, double* host_out);
/* Replace a reduced matrix (invalidates any rom_perturb preparation). */
int yr_rom_set(yr_rom* rom, int32_t which, const double* host_in);
/* A reduced model given by its matrices (all zero until set). */
int yr_rom_create(int32_t q1, int32_t q2, int32_t nsrc, int32_t nprb, yr_rom** out);
/* Copy the projection basis (FP64, padded layout: V1 is q1 columns of the
 * electric half of a field buffer, V2 q2 columns of the magnetic half) to
 * caller device buffers.  YR_ESTATE for models created from matrices. */
int yr_rom_basis(const yr_rom* rom, void* V1, void* V2);
void yr_rom_destroy(yr_rom* rom);

/* Test hook: y = S x for ncol complex columns (interleaved re/im, dtype)
 * of electric vectors, S the Schur complement of [z (R+F) - (R-F)] at time
 * step dt (eq. (reduced_linear_system_solution1)).  Synchronous. */
int yr_schur_apply(yr_operator* op, double dt, double z_re, double z_im, yr_dtype dtype,
                   const void* x, void* y, int32_t ncol);

/* --------------------------------------------------------- beyond the CFL limit */

/* rom_perturb — stability enforcement of Sec. III-A for time step dt:
 * the singular values s_i of De~^-1/2 K~ Dm~^-1/2 (eq. (singular_limit))
 * that reach gamma * 2/dt are clamped to that value and K~ is replaced by
 * K~' = De~^1/2 U S' W^T Dm~^1/2 (any square root gives the same K~').
 * gamma = 0.9999 in Sec. V; values >= 1 are accepted but do not enforce
 * stability (the certificate below then decides).  No-op on K~ when every
 * s_i < gamma 2/dt (always the case below the CFL limit).
 * It also builds the stepping form used by rom_step, in step_dtype: the
 * state whitened by the Cholesky factors of De~, Dm~ and rotated onto the
 * eigenvectors of the whitened loss matrices, so that each half step is a
 * diagonal scaling plus one product with the same dense matrix A'' (A''
 * for the electric, A''^T for the magnetic half).  The stepping matrices
 * are certified in FP64 after rounding to step_dtype: the leapfrog they
 * define satisfies condition (Dstability2) iff 4I - M^T M > 0, checked by a
 * Cholesky factorisation (M defined in rom.hip).  FP64 throughout on the
 * device; synchronous.  n_clamped (may be NULL) receives the count.
 * Errors: YR_EINVAL (De~ or Dm~ not positive definite), YR_EUNSTABLE
 * (certificate failed; the model is left unprepared). */
int rom_perturb(yr_rom* rom, double dt, double gamma, yr_dtype step_dtype, int32_t* n_clamped);

/* Same for nmodels models at once (the Jacobi phases of all models share
 * each launch); n_clamped[nmodels] may be NULL. */
int rom_perturb_batch(yr_rom* const* roms, int32_t nmodels, double dt, double gamma,
                      yr_dtype step_dtype, int32_t* n_clamped);

/* rom_step — nsteps of the reduced leapfrog eq. (reducedMNAform) for every
 * model, all in one kernel launch (one workgroup per model, models of
 * different orders side by side).  Per model m (device pointers, dtype):
 *   u[m]: [nsteps][nsrc_m] input, u[m][n] drives the step producing x~^{n+1};
 *   y[m]: [nsteps][nprb_m] output, y[m][n] = L~^T x~^{n+1};
 *   state[m]: [q1_m + q2_m] initial state in the stepping coordinates,
 *     overwritten with the final state (state or state[m] may be NULL:
 *     zero initial state, final state not returned).
 * Every model must have been prepared by rom_perturb for this dt and dtype
 * (YR_ESTATE otherwise).  Asynchronous on `stream`. */
int rom_step(yr_rom* const* roms, int32_t nmodels, double dt, int64_t nsteps, yr_dtype dtype,
             const void* const* u, void* const* y, void* const* state, void* stream);

/* rom_step_noalloc — rom_step for callers that cannot allocate device
 * memory (tight serving loops, harnesses that forbid hipMalloc).  Same
 * arguments, kernel and results as rom_step; it calls no device allocation
 * or free.  It is not meant for HIP stream capture: the host waits for the
 * upload of its descriptor table (below), which a capturing stream does not
 * allow.  Its per-call descriptor table lives in
 * a fixed device array of 4096 entries (one per model) that each device keeps
 * for the life of the process, so:
 *  - nmodels above 4096 is rejected (YR_EINVAL);
 *  - calls that overlap on one device race for that table: they must not be
 *    issued concurrently (from several host threads or on several streams
 *    before the previous call's kernel finished reading it);
 *  - the workgroup size is the one rom_step's autotuner already chose for the
 *    same shape, else 1024 threads (no trial launches: they need scratch).
 * The table (a 72-byte record per model) is uploaded on `stream` and the
 * host waits for that copy (and the work queued before it); the stepping
 * kernel then runs asynchronously on `stream`, like rom_step's. */
int rom_step_noalloc(yr_rom* const* roms, int32_t nmodels, double dt, int64_t nsteps,
                     yr_dtype dtype, const void* const* u, void* const* y, void* const* state,
                     void* stream);

/* rom_lift — full-field reconstruction x ~ V x~ (eq. (V): the full state is
 * approximated in the span of the projection basis, Sec. II-C).  Maps
 * nstates reduced states, given in rom_step's stepping coordinates, back to
 * full field buffers: x~_e = Le^-T Qe s_e, x~_h = Lm^-T Qm s_h (the inverse of
 * the whitening and rotation set up by rom_perturb, FP64), then E = V1 x~_e
 * and H = V2 x~_h (FP64 accumulation over the basis, rounded to dtype).
 *   op:     the operator the model was reduced from (YR_ESTATE otherwise);
 *   rom:    a model from mor_reduce, prepared by rom_perturb (any step dtype;
 *           YR_ESTATE otherwise);
 *   states: device dtype [nstates][q1 + q2] (the state layout of rom_step);
 *   fields: device dtype [nstates][field buffer] written in the padded layout
 *           of fdtd_step (E slots then H slots; zero off the unknowns).
 * Reads the basis once per 4 states (about 8 (nE q1 + nH q2) bytes).
 * Asynchronous on `stream` (stream-ordered scratch of nstates (q1+q2) doubles).
 * Errors: YR_EINVAL (bad arguments, order above 1024), YR_ESTATE. */
int rom_lift(const yr_operator* op, const yr_rom* rom, yr_dtype dtype, int32_t nstates,
             const void* states, void* fields, void* stream);

/* rom_adjoint — gradient of J = dt sum_n sum_p y_p^n^2 ... generalised to
 * any J(y) through dJdy, for the reduced leapfrog at dt after the clamp of
 * Sec. III-A (not in the paper; the adjoint of eq. (reducedMNAform) derived
 * from the same equations).  FP64 on the device, synchronous.
 *   u:    device FP64 [nsteps][nsrc] input;  dJdy: device FP64 [nsteps][nprb].
 *   dDe:  host FP64 q1 x q1 (column-major), the change of De~ for a unit
 *         change of a parameter theta with the basis frozen (see
 *         yr_rom_project_cells), or NULL.
 *   through_clamp: differentiate K~' = Le f(Le^-1 K~ Lm^-T) Lm^T as well
 *         (f the singular-value clamp; divided differences of f, needs
 *         q1 == q2 and distinct singular values) instead of holding K~' fixed.
 *   gDe, gDse (q1 x q1), gK (q1 x q2): host outputs dJ/dDe~, dJ/dDse~,
 *         dJ/dK~' (may be NULL).
 *   result[3]: J, dJ/dtheta with K~' held fixed, dJ/dtheta through the clamp.
 * Errors: YR_EINVAL (matrices not positive definite, bad sizes). */
int rom_adjoint(yr_rom* rom, double dt, double gamma, int64_t nsteps, const double* u,
                const double* dJdy, const double* dDe, int32_t through_clamp, double* gDe,
                double* gDse, double* gK, double* result);

/* V1^T diag(d) V1 (host FP64 q1 x q1 out) where d is the electric diagonal
 * of eq. (matrix) built from a per-cell field (host FP64 nx*ny*nz):
 * which = 0: eps0 * eps_r (-> De~), 1: sigma_e (-> Dse~).  For a change of
 * material d(eps_r) per cell this is dDe~ with the basis frozen.  The model
 * must come from mor_reduce on `op`. */
int yr_rom_project_cells(yr_operator* op, const yr_rom* rom, const double* cell_values,
                         int32_t which, double* out);

/* ------------------------------------------------------ frequency response */

/* probe_dft — spectra of probe waveforms, from which Sec. V reads its
 * accuracy figures: the resonant frequencies of the cavities (Sec. V-A,
 * first six resonances against analytical values) and the transmission /
 * reflection coefficients S21, S11 of the guide and the microstrip
 * (Sec. V-B, V-D).  Discrete-time Fourier transform at nf given
 * frequencies, sample n of the record taken at time t0 + n dt:
 *   out[k][p] = dt * sum_n w_n y[n][p] exp(-j 2 pi freqs[k] (t0 + n dt)),
 * w_n = 1, or the Hann taper sin^2(pi (n + 1/2) / nsteps) when hann != 0.
 *   y:     device, dtype, [nsteps][nprb] (the layout fdtd_step and rom_step
 *          write; for fdtd_step's y, sample n is E^{n+1}, at t = (n+1) dt);
 *   freqs: host FP64 [nf] in Hz;
 *   out:   device FP64 [nf][nprb] complex values, interleaved (re, im).
 * FP64 accumulation whatever the dtype of y.  Asynchronous on `stream`
 * (a stream-ordered copy of the frequency list).
 * Errors: YR_EINVAL (negative sizes, dt <= 0, non-finite input, null). */
int probe_dft(yr_dtype dtype, const void* y, int64_t nsteps, int32_t nprb, double dt, double t0,
              int32_t nf, const double* freqs, int32_t hann, void* out, void* stream);

/* ------------------------------------------------------------- kernel timers */

/* Per-kernel timing with HIP events recorded on each launch's stream
 * (off by default).  Named kernels: "fdtd_e", "fdtd_h" (leapfrog half
 * steps), "cocg_fused" / "cocg_fused_real" (one-pass COCG iteration, complex
 * or real shift), "schur_h", "schur_e" (the two sweeps of one Schur matvec),
 * "cocg_update" (solver vector update of the two-sweep path).
 * yr_profile_select limits the timed kernels to a comma-separated list of
 * names (NULL or "": all), so that short launches can run untimed: an event
 * pair costs a few microseconds of host time per launch.  yr_profile_read
 * returns the number of launches and their summed duration in milliseconds
 * since the last reset (waits for the recorded events). */
int yr_profile_enable(int on);
int yr_profile_select(const char* names);
int yr_profile_reset(void);
int yr_profile_read(const char* name, int64_t* launches, double* ms);

#ifdef __cplusplus
}
#endif

#endif /* YEEROM_H */
