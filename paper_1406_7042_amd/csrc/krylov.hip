// Shifted linear solves of the reduction, Sec. IV-B.  The system
// [z (R+F) - (R-F)] x = w is reduced to its Schur complement on the electric
// unknowns (eqs. (reduced_linear_system_solution1/2)); A11 and A22 are
// diagonal, so S = A11 - A12 A22^{-1} A21 is applied as two stencil sweeps.
// S is complex symmetric (not Hermitian), so the iterative solver is the
// conjugate-orthogonal CG (bilinear form x^T y) run to the normalized residual
// the paper uses, on a batch of right-hand sides at once.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <type_traits>
#include <vector>

#include "krylov.hpp"
#include "profile.hpp"

namespace yr {

namespace {
constexpr int kRedBlocksMax = 1024;
constexpr int kMaxVals = 48;  // 3 * 16 partial values per block

unsigned red_grid(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  return (unsigned)(g < kRedBlocksMax ? (g < 1 ? 1 : g) : kRedBlocksMax);
}
}  // namespace

// ---------------------------------------------------------------- coefficients

template <typename T>
__global__ void k_real_part(const cplx<T>* __restrict__ src, T* __restrict__ dst, int64_t n) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g < n) dst[g] = src[g].re;
}

template <typename T>
__global__ void k_to_complex(const T* __restrict__ src, cplx<T>* __restrict__ dst, int64_t n) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g < n) dst[g] = cplx<T>(src[g], (T)0);
}

template <typename T>
__global__ void k_zero_real(T* __restrict__ dst, int64_t n) {
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g < n) dst[g] = (T)0;
}

template <typename T>
__global__ void k_prepare_diag(cplx<T>* __restrict__ out, const double* __restrict__ d,
                               const double* __restrict__ s, const uint8_t* __restrict__ mask,
                               int64_t n, double dt, double zr, double zi, int invert) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= n) return;
  if (mask[g] != 1) {
    out[g] = cplx<T>(0, 0);
    return;
  }
  // (z-1) d/dt + (z+1) s/2
  zd v((zr - 1.0) * d[g] / dt + (zr + 1.0) * s[g] * 0.5, zi * d[g] / dt + zi * s[g] * 0.5);
  if (invert) v = cdiv(zd(1.0, 0.0), v);
  out[g] = cplx<T>((T)v.re, (T)v.im);
}

template <typename T>
int SchurOp<T>::prepare(const yr_operator* o, double dt_, zd z_, hipStream_t s) {
  op = o;
  dt = dt_;
  z = z_;
  int64_t nE = o->ne_slots * o->len, nH = o->nh_slots * o->len;
  YR_CALL(a11.reserve(nE * sizeof(cplx<T>)));
  k_prepare_diag<T><<<grid_for(nE), kBlock, 0, s>>>(a11.as<cplx<T>>(), o->eps_e.as<double>(),
                                                   o->sig_e.as<double>(), o->emask.as<uint8_t>(),
                                                   nE, dt, z.re, z.im, 0);
  YR_TRY_HIP(hipGetLastError());
  if (z.im == 0) {  // real shift: a real copy for the real-arithmetic solver
    YR_CALL(a11r.reserve(nE * sizeof(T)));
    k_real_part<T><<<grid_for(nE), kBlock, 0, s>>>(a11.as<cplx<T>>(), a11r.as<T>(), nE);
    YR_TRY_HIP(hipGetLastError());
  }
  // uniform magnetic materials: a22 = (z-1) mu0/dt
  const double mu0 = 1.25663706212e-6;
  zd a22((z.re - 1.0) * mu0 / dt, z.im * mu0 / dt);
  zd inv = cdiv(zd(1.0, 0.0), a22);
  a22inv_s = cplx<T>((T)inv.re, (T)inv.im);
  if (!o->uniform_h) {
    YR_CALL(a22inv.reserve(nH * sizeof(cplx<T>)));
    k_prepare_diag<T><<<grid_for(nH), kBlock, 0, s>>>(
        a22inv.as<cplx<T>>(), o->mu_h.as<double>(), o->sigm_h.as<double>(),
        o->hmask.as<uint8_t>(), nH, dt, z.re, z.im, 1);
    YR_TRY_HIP(hipGetLastError());
  }
  return YR_OK;
}

// ---------------------------------------------------------------- Schur matvec

// h = a22^{-1} cp(r + beta p)   (H-vectors)
template <typename T, int NB, bool UNI>
__global__ void __launch_bounds__(kBlock)
    k_schur_h(const cplx<T>* __restrict__ r, const cplx<T>* __restrict__ p,
              const ColState* __restrict__ st, cplx<T>* __restrict__ h,
              const cplx<T>* __restrict__ a22inv, cplx<T> a22s, const uint8_t* __restrict__ hmask,
              Axes<T> ax, Geo g, int64_t ldE, int64_t ldH, int use_beta) {
  cplx<T> beta[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c)
    beta[c] = use_beta ? cplx<T>((T)st[c].beta_re, (T)st[c].beta_im) : cplx<T>(0, 0);
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < g.len;
       t += (int64_t)gridDim.x * blockDim.x) {
    int i, j, k;
    decode(t, g, i, j, k);
    for (int s = 0; s < g.nh_slots; ++s) {
      int64_t gi = s * g.len + t;
      if (hmask[gi] != 1) {
#pragma unroll
        for (int c = 0; c < NB; ++c) h[c * ldH + gi] = cplx<T>(0, 0);
        continue;
      }
      cplx<T> a = UNI ? a22s : a22inv[gi];
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const cplx<T>* rc = r + c * ldE;
        const cplx<T>* pc = p + c * ldE;
        const cplx<T> b = beta[c];
        auto ev = [&](int sl, int64_t idx) {
          int64_t q = sl * g.len + idx;
          return rc[q] + b * pc[q];
        };
        h[c * ldH + gi] = a * curl_p<cplx<T>>(g, ax, s, t, i, j, k, ev);
      }
    }
  }
}

// p = r + beta p ; q = W_e (a11 p - z curl_d(h)) ; partial sums of p^T q
template <typename T, int NB>
__global__ void __launch_bounds__(kBlock)
    k_schur_e(const cplx<T>* __restrict__ r, cplx<T>* __restrict__ p,
              const ColState* __restrict__ st, const cplx<T>* __restrict__ h,
              cplx<T>* __restrict__ q, const cplx<T>* __restrict__ a11,
              const uint8_t* __restrict__ emask, Axes<T> ax, Geo g, int64_t ldE, int64_t ldH,
              double zr, double zi, int use_beta, double* __restrict__ partial) {
  __shared__ double lds[kMaxVals * (kBlock / 64)];
  cplx<T> beta[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c)
    beta[c] = use_beta ? cplx<T>((T)st[c].beta_re, (T)st[c].beta_im) : cplx<T>(0, 0);
  const cplx<T> z((T)zr, (T)zi);
  double acc[2 * NB];
#pragma unroll
  for (int c = 0; c < 2 * NB; ++c) acc[c] = 0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < g.len;
       t += (int64_t)gridDim.x * blockDim.x) {
    int i, j, k;
    decode(t, g, i, j, k);
    for (int s = 0; s < g.ne_slots; ++s) {
      int64_t gi = s * g.len + t;
      if (emask[gi] != 1) {
#pragma unroll
        for (int c = 0; c < NB; ++c) q[c * ldE + gi] = cplx<T>(0, 0);
        continue;
      }
      const T we = w_e<T>(g, ax, s, i, j, k);
      const cplx<T> a = a11[gi];
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const cplx<T>* hc = h + c * ldH;
        auto hv = [&](int sl, int64_t idx) { return hc[sl * g.len + idx]; };
        cplx<T> pn = r[c * ldE + gi] + beta[c] * p[c * ldE + gi];
        cplx<T> cd = curl_d<cplx<T>>(g, ax, s, t, i, j, k, hv);
        cplx<T> qv = (a * pn - z * cd) * we;
        p[c * ldE + gi] = pn;
        q[c * ldE + gi] = qv;
        acc[2 * c] += (double)pn.re * qv.re - (double)pn.im * qv.im;
        acc[2 * c + 1] += (double)pn.re * qv.im + (double)pn.im * qv.re;
      }
    }
  }
  block_sum<2 * NB>(acc, lds, partial + (int64_t)blockIdx.x * 2 * NB);
}

// x += alpha p ; r -= alpha q ; partial sums of r^T r and ||r||^2
template <typename T, int NB>
__global__ void __launch_bounds__(kBlock)
    k_cocg_update(cplx<T>* __restrict__ x, cplx<T>* __restrict__ r,
                  const cplx<T>* __restrict__ p, const cplx<T>* __restrict__ q,
                  const ColState* __restrict__ st, int64_t n, int64_t ldE, int do_update,
                  double* __restrict__ partial) {
  __shared__ double lds[kMaxVals * (kBlock / 64)];
  cplx<T> alpha[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) alpha[c] = cplx<T>((T)st[c].alpha_re, (T)st[c].alpha_im);
  double acc[3 * NB];
#pragma unroll
  for (int c = 0; c < 3 * NB; ++c) acc[c] = 0;
  for (int64_t gi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; gi < n;
       gi += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      cplx<T> rv = r[c * ldE + gi];
      if (do_update) {
        x[c * ldE + gi] = x[c * ldE + gi] + alpha[c] * p[c * ldE + gi];
        rv = rv - alpha[c] * q[c * ldE + gi];
        r[c * ldE + gi] = rv;
      }
      acc[3 * c] += (double)rv.re * rv.re - (double)rv.im * rv.im;
      acc[3 * c + 1] += 2.0 * (double)rv.re * rv.im;
      acc[3 * c + 2] += (double)rv.re * rv.re + (double)rv.im * rv.im;
    }
  }
  block_sum<3 * NB>(acc, lds, partial + (int64_t)blockIdx.x * 3 * NB);
}

// One COCG iteration in one pass (3-D, uniform magnetic materials).
// With alpha = alpha_{i-1} and beta = beta_i of the column:
//   r_i = r_{i-1} - alpha q_{i-1}     p_i = r_i + beta p_{i-1}
//   q_i = S p_i   (H kept on chip)
// and the bilinear sums rho_i = r_i^T r_i, ||r_i||^2, pi_i = q_{i-1}^T p_i,
// sigma_i = p_i^T q_i, omega_i = q_i^T q_i that fix alpha_i and beta_{i+1}
// (k_cocg_scalar_fused).  x is needed only at the end: the variant with XU
// set (odd passes) forms x_i = x_{i-2} + alpha_{i-2} p_{i-2} + alpha_{i-1}
// p_{i-1}, the other one leaves x alone (k_x_fixup completes a column whose
// last pass was even).  r and q are double buffered, p rotates over three
// buffers (neighbouring tiles read the previous iterate in their halo, the
// x update reads p_{i-2}).
// Work decomposition: an xy tile of TX x TY electric positions and a chunk of
// KZ z-planes per block, one RHS column per block, marching up in z.  Only the
// columns still iterating get blocks: the column map lists them, and the host
// re-plans the grid (more z chunks for fewer columns) whenever it reads the
// convergence flags.  LDS holds p_i on planes k and k+1 over the tile plus a
// one-cell halo and h on planes k-1 (Hx, Hy) and k; plane k+2 is fetched into
// registers while plane k is computed, so the load latency hides behind the
// two stencils.
// Electric unknowns never lie at i = nx, j = ny or k = nz, so the positions a
// block owns are its tile's cells of planes [k0, k1).
// Block order is XCD-aware: consecutive block ids go round-robin over the 8
// XCDs, so block b works on tile-chunk xcd*per_xcd + (b/8)/n of mapped column
// (b/8)%n: each XCD owns a contiguous run of tiles (halo re-reads hit its own
// L2) and the n columns of a tile run side by side there (a11 and the mask
// are read once).
struct FusedTiling {
  int KZ, ntx, nty, nkz, ntiles, per_xcd;
};

constexpr int kMaxCols = 16;  // right-hand sides per solver chunk
struct ColMap {
  int n;              // columns in this pass
  int c[kMaxCols];    // their indices
};

template <typename T>
struct FusedCfg;
template <>
struct FusedCfg<float> {  // 128-wide rows: fewer partial cache lines per tile row
  static constexpr int TX = 128, TY = 8, NT = 1024;
};
template <>
struct FusedCfg<double> {
  static constexpr int TX = 32, TY = 8, NT = 256;
};

constexpr int kFusedVals = 9;  // rho (2), ||r||^2, pi (2), sigma (2), omega (2)

// Value-type helpers: V = cplx<T> for a complex shift, V = T at a real one
// (the real expansion point: real system, real right-hand sides).
template <typename V>
struct FV;
template <typename T>
struct FV<cplx<T>> {
  static constexpr int CW = 2;
  // an unconditional use of a loaded value (the wave waits for the load)
  static __device__ void use(cplx<T> x) {
    FV<T>::use(x.re);
    FV<T>::use(x.im);
  }
  static __device__ cplx<T> mk(double re, double im) { return cplx<T>((T)re, (T)im); }
  // a += x^T y (bilinear, complex: two doubles)
  static __device__ void bil(double* a, cplx<T> x, cplx<T> y) {
    a[0] += (double)x.re * y.re - (double)x.im * y.im;
    a[1] += (double)x.re * y.im + (double)x.im * y.re;
  }
  static __device__ double nrm(cplx<T> x) { return (double)x.re * x.re + (double)x.im * x.im; }
};
template <>
struct FV<float> {
  static constexpr int CW = 1;
  static __device__ void use(float x) { asm volatile("" ::"v"(x)); }
  static __device__ float mk(double re, double) { return (float)re; }
  static __device__ void bil(double* a, float x, float y) { a[0] += (double)x * y; }
  static __device__ double nrm(float x) { return (double)x * x; }
};
template <>
struct FV<double> {
  static constexpr int CW = 1;
  static __device__ void use(double x) { asm volatile("" ::"v"(x)); }
  static __device__ double mk(double re, double) { return re; }
  static __device__ void bil(double* a, double x, double y) { a[0] += x * y; }
  static __device__ double nrm(double x) { return x * x; }
};

template <typename T, typename V, int TX, int TY, int NT, bool XU>
__global__ void __launch_bounds__(NT)
    k_cocg_fused3(const V* __restrict__ rin, const V* __restrict__ qin, const V* __restrict__ pin,
                  const V* __restrict__ p2in,
                  V* __restrict__ rout, V* __restrict__ qout, V* __restrict__ pout,
                  V* __restrict__ x, const ColState* __restrict__ st, const V* __restrict__ a11,
                  V a22s,
                  const uint8_t* __restrict__ emask, Axes<T> ax, Geo g, int64_t ldE, int nx,
                  int ny, int nz, FusedTiling ft, ColMap cm, double zr, double zi,
                  double* __restrict__ partial) {
  constexpr int PW = TX + 2, PH = TY + 2, PT = PW * PH;  // p tile with halo
  constexpr int HW = TX + 1, HH = TY + 1, HT = HW * HH;  // h tile, low-side halo
  constexpr int NL = (3 * PT + NT - 1) / NT;             // plane loads per thread
  constexpr int NE = (TX * TY + NT - 1) / NT;            // outputs per thread
  constexpr int CW = FV<V>::CW;
  __shared__ T Ps[2 * 3 * PT * CW];  // [plane buffer][Ex Ey Ez][PT]
  __shared__ T Hs[5 * HT * CW];      // [plane buffer][Hx Hy][HT], then Hz [HT]
  __shared__ T axs[4 * PW + 4 * PH];  // p d ip id along x over the tile, then y
  __shared__ double lds_red[kFusedVals * (NT / 64)];
  __shared__ double res[kFusedVals];
  V* P = reinterpret_cast<V*>(Ps);
  V* H = reinterpret_cast<V*>(Hs);
  const int b = blockIdx.x;
  const int xcd = b & 7, loc = b >> 3;
  const int col = cm.c[loc % cm.n];
  const int tl = xcd * ft.per_xcd + loc / cm.n;
  // a converged column keeps x, r and p as they are: its blocks do nothing
  // (their partial sums are not read for it any more)
  if (st[col].status != 0) return;
  double acc[kFusedVals];
#pragma clang loop unroll(full)
  for (int v = 0; v < kFusedVals; ++v) acc[v] = 0;
  if (tl < ft.ntiles * ft.nkz) {
    const int chunk = tl % ft.nkz, tile = tl / ft.nkz;
    const int i0 = (tile % ft.ntx) * TX, j0 = (tile / ft.ntx) * TY;
    const int k0 = chunk * ft.KZ, k1 = min(nz, k0 + ft.KZ);
    const V alpha = FV<V>::mk(st[col].alpha_re, st[col].alpha_im);
    const V alpha1 = FV<V>::mk(st[col].alpha1_re, st[col].alpha1_im);
    const V beta = FV<V>::mk(st[col].beta_re, st[col].beta_im);
    const V z = FV<V>::mk(zr, zi);
    const int64_t co = col * ldE;
    const int64_t len = g.len, X = g.X, Y = g.Y, XY = (int64_t)g.X * g.Y;
    const T inv_v0 = (T)g.inv_v0;
    for (int u = threadIdx.x; u < 4 * PW; u += NT) {
      const int which = u / PW, m = u - which * PW, ix = i0 - 1 + m;
      const T* tab = which == 0 ? ax.p[0] : which == 1 ? ax.d[0] : which == 2 ? ax.ip[0] : ax.id[0];
      axs[u] = (ix >= 0 && ix < g.X) ? tab[ix] : T(0);
    }
    for (int u = threadIdx.x; u < 4 * PH; u += NT) {
      const int which = u / PH, m = u - which * PH, ix = j0 - 1 + m;
      const T* tab = which == 0 ? ax.p[1] : which == 1 ? ax.d[1] : which == 2 ? ax.ip[1] : ax.id[1];
      axs[4 * PW + u] = (ix >= 0 && ix < g.Y) ? tab[ix] : T(0);
    }
    // plane slots: slot u of this thread is p-tile entry threadIdx.x + u NT;
    // `own` marks the tile's interior cells, which this block updates, `pad`
    // the padding positions i = nx or j = ny that border them (never unknowns,
    // always zero): the block stores zeros there too, so that every row of a
    // vector is written as whole cache lines (a line left partly unwritten
    // costs a read-modify-write in memory)
    int64_t off[NL];
    bool okxy[NL], own[NL], pad[NL];
#pragma clang loop unroll(full)
    for (int u = 0; u < NL; ++u) {
      const int idx = threadIdx.x + u * NT;
      const int s = idx / PT, rem = idx - s * PT;
      const int lj = rem / PW, li = rem - lj * PW;
      const int i = i0 - 1 + li, j = j0 - 1 + lj;
      okxy[u] = idx < 3 * PT && i >= 0 && j >= 0 && i < X && j < Y;
      own[u] = idx < 3 * PT && li >= 1 && li <= TX && lj >= 1 && lj <= TY && i < nx && j < ny;
      pad[u] = idx < 3 * PT && li >= 1 && lj >= 1 && i <= nx && j <= ny && (i == nx || j == ny) &&
               (li <= TX || i == nx) && (lj <= TY || j == ny);
      off[u] = co + s * len + (int64_t)j * X + i;
    }
    V rv[NL], qv[NL], pv[NL], xv[NL], p2v[NL];
    // Loads only: out-of-box slots read element 0 and are zeroed where the
    // values are used (stash), so no instruction needs the loaded values
    // before the two stencils of the current plane have run (a select right
    // after a load would make the wave wait for it at once).
    auto fetch = [&](int kk, bool live = true) __attribute__((always_inline)) {
      const bool okz = live && kk >= 0 && kk < g.Z;
      const bool ownz = kk >= k0 && kk < k1;
#pragma clang loop unroll(full)
      for (int u = 0; u < NL; ++u) {
        const bool ok = okz && okxy[u];
        const bool ox = ownz && own[u];
        const int64_t gi = ok ? off[u] + kk * XY : 0;
        const int64_t gx = ox ? off[u] + kk * XY : 0;
        rv[u] = rin[gi];
        qv[u] = qin[gi];
        pv[u] = pin[gi];
        if (XU) {  // owned slots only
          xv[u] = x[gx];
          p2v[u] = p2in[gx];
        }
      }
    };
    // the wave waits for the loads of fetch() here on every path (also where
    // the plane is not needed), so no register of theirs is still pending
    // when the next fetch reuses it
    auto settle = [&]() __attribute__((always_inline)) {
#pragma clang loop unroll(full)
      for (int u = 0; u < NL; ++u) {
        FV<V>::use(rv[u]);
        FV<V>::use(qv[u]);
        FV<V>::use(pv[u]);
        if (XU) {
          FV<V>::use(xv[u]);
          FV<V>::use(p2v[u]);
        }
      }
    };
    // vector updates of plane kk into p buffer `buf` (and HBM for owned cells)
    auto stash = [&](int buf, int kk) __attribute__((always_inline)) {
      const bool okz = kk >= 0 && kk < g.Z;
      const bool ownz = kk >= k0 && kk < k1;
#pragma clang loop unroll(full)
      for (int u = 0; u < NL; ++u) {
        const int idx = threadIdx.x + u * NT;
        const bool ok = okz && okxy[u];
        const V r0 = ok ? rv[u] : V(0), q0 = ok ? qv[u] : V(0), p0 = ok ? pv[u] : V(0);
        const V rn = r0 - alpha * q0;
        const V pn = rn + beta * p0;
        if (idx < 3 * PT) P[buf * 3 * PT + idx] = pn;
        if (ownz && own[u]) {
          const int64_t gi = off[u] + kk * XY;
          rout[gi] = rn;
          pout[gi] = pn;
          // x_i = x_{i-2} + alpha_{i-2} p_{i-2} + alpha_{i-1} p_{i-1} on the passes that
          // update x (every other one)
          if (XU) x[gi] = (xv[u] + alpha1 * p2v[u]) + alpha * p0;
          FV<V>::bil(acc + 0, rn, rn);
          acc[2] += FV<V>::nrm(rn);
          FV<V>::bil(acc + 3, q0, pn);
        } else if (ownz && pad[u]) {
          const int64_t gi = off[u] + kk * XY;
          rout[gi] = V(0);
          pout[gi] = V(0);
          qout[gi] = V(0);
          if (XU) x[gi] = V(0);
        }
      }
    };
    // output positions of this thread
    int64_t eoff[NE];
    int eli[NE], elj[NE];
    bool eok[NE];
#pragma clang loop unroll(full)
    for (int u = 0; u < NE; ++u) {
      const int idx = threadIdx.x + u * NT;
      elj[u] = idx / TX;
      eli[u] = idx - elj[u] * TX;
      eok[u] = idx < TX * TY && i0 + eli[u] < nx && j0 + elj[u] < ny;
      eoff[u] = (int64_t)(j0 + elj[u]) * X + i0 + eli[u];
    }
    V av[NE][3];
    uint8_t mv[NE][3];
    T zip = 0, zid = 0, zp = 0, zd_ = 0;  // ip, id, p, d along z at plane k
    auto fetch_e = [&](int k) __attribute__((always_inline)) {
      zip = ax.ip[2][k];  // 0 <= k < nz: in range
      zid = ax.id[2][k];
      zp = ax.p[2][k];
      zd_ = ax.d[2][k];
#pragma clang loop unroll(full)
      for (int u = 0; u < NE; ++u)
#pragma clang loop unroll(full)
        for (int s = 0; s < 3; ++s) {
          // used only where eok (e_plane skips the others): no select
          const int64_t gi = eok[u] ? s * len + k * XY + eoff[u] : 0;
          av[u][s] = a11[gi];
          mv[u][s] = emask[gi];
        }
    };
    // h = a22^-1 cp(p) on plane kk from p planes kk (buffer a) and kk+1 (bn)
    // ipz: ip along z at plane kk (0 outside [0, nz))
    auto h_plane = [&](int kk, T ipz, int a, int bn, int hb, bool only_xy)
                       __attribute__((always_inline)) {
      const int ncomp = only_xy ? 2 : 3;
      const bool okz = kk >= 0 && kk < nz;
      const V* Pa = P + a * 3 * PT;
      const V* Pb = P + bn * 3 * PT;
      for (int idx = threadIdx.x; idx < ncomp * HT; idx += NT) {
        const int s = idx / HT, rem = idx - s * HT;
        const int hj = rem / HW, hi = rem - hj * HW;
        const int i = i0 - 1 + hi, j = j0 - 1 + hj;
        V v(0);
        // magnetic unknowns feeding an electric one lie in [0,nx) x [0,ny) x [0,nz)
        if (okz && i >= 0 && j >= 0 && i < nx && j < ny) {
          const int pl = hj * PW + hi;  // p-tile index of (i, j)
          const T ipx = axs[2 * PW + hi], ipy = axs[4 * PW + 2 * PH + hj];
          V c;
          if (s == 0)  // Hx: dEy/dz - dEz/dy
            c = (Pb[PT + pl] - Pa[PT + pl]) * ipz - (Pa[2 * PT + pl + PW] - Pa[2 * PT + pl]) * ipy;
          else if (s == 1)  // Hy: dEz/dx - dEx/dz
            c = (Pa[2 * PT + pl + 1] - Pa[2 * PT + pl]) * ipx - (Pb[pl] - Pa[pl]) * ipz;
          else  // Hz: dEx/dy - dEy/dx
            c = (Pa[pl + PW] - Pa[pl]) * ipy - (Pa[PT + pl + 1] - Pa[PT + pl]) * ipx;
          v = a22s * c;
        }
        H[(s < 2 ? hb * 2 + s : 4) * HT + rem] = v;
      }
    };
    // q = W_e (a11 p - z curl_d h) on plane k
    auto e_plane = [&](int k, int pa, int hb) __attribute__((always_inline)) {
      const V* Hc = H + hb * 2 * HT;        // Hx, Hy of plane k
      const V* Hp = H + (1 - hb) * 2 * HT;  // Hx, Hy of plane k-1
      const V* Hz = H + 4 * HT;
      const V* Pc = P + pa * 3 * PT;
      const T idz = zid, pz = zp, dz = zd_;
#pragma clang loop unroll(full)
      for (int u = 0; u < NE; ++u) {
        if (!eok[u]) continue;
        const int li = eli[u], lj = elj[u];
        const int hl = (lj + 1) * HW + (li + 1);  // h-tile index of (i, j)
        const int pl = (lj + 1) * PW + (li + 1);  // p-tile index of (i, j)
        const T pxv = axs[li + 1], dxv = axs[PW + li + 1], idxv = axs[3 * PW + li + 1];
        const T pyv = axs[4 * PW + lj + 1], dyv = axs[4 * PW + PH + lj + 1],
                idyv = axs[4 * PW + 3 * PH + lj + 1];
        const int64_t base = co + k * XY + eoff[u];
#pragma clang loop unroll(full)
        for (int s = 0; s < 3; ++s) {
          const V pn = Pc[s * PT + pl];
          V qn(0);
          if (mv[u][s] == 1) {
            V cd;
            T w;
            if (s == 0) {  // dHz/dy - dHy/dz
              cd = (Hz[hl] - Hz[hl - HW]) * idyv - (Hc[HT + hl] - Hp[HT + hl]) * idz;
              w = pxv * dyv * dz;
            } else if (s == 1) {  // dHx/dz - dHz/dx
              cd = (Hc[hl] - Hp[hl]) * idz - (Hz[hl] - Hz[hl - 1]) * idxv;
              w = dxv * pyv * dz;
            } else {  // dHy/dx - dHx/dy
              cd = (Hc[HT + hl] - Hc[HT + hl - 1]) * idxv - (Hc[hl] - Hc[hl - HW]) * idyv;
              w = dxv * dyv * pz;
            }
            qn = (av[u][s] * pn - z * cd) * (w * inv_v0);
          }
          qout[s * len + base] = qn;
          FV<V>::bil(acc + 5, pn, qn);
          FV<V>::bil(acc + 7, qn, qn);
        }
      }
    };
    int cur = 0, hb = 0;
    fetch(k0 - 1);
    stash(1, k0 - 1);
    fetch(k0);
    stash(0, k0);
    fetch(k0 + 1);
    __syncthreads();
    h_plane(k0 - 1, k0 >= 1 ? ax.ip[2][k0 - 1] : T(0), 1, 0, 1, true);
    __syncthreads();
    stash(1, k0 + 1);  // plane k0+1 replaces k0-1
    __syncthreads();
    for (int k = k0; k < k1; ++k) {
      const bool more = k + 2 <= k1;
      // a11 and the mask of plane k first, then plane k+2 of r, q, p, x: the
      // loads complete in issue order, so e_plane's wait for a11 leaves the
      // plane k+2 loads in flight behind both stencils.  They are issued even
      // past the chunk (as reads of element 0): no branch joins in front of
      // the stencils.
      fetch_e(k);
      fetch(k + 2, more);
      h_plane(k, zip, cur, 1 - cur, hb, false);
      __syncthreads();
      e_plane(k, cur, hb);
      __syncthreads();
      settle();
      if (more) {
        stash(cur, k + 2);  // plane k+2 replaces k
        __syncthreads();
      }
      cur = 1 - cur;
      hb = 1 - hb;
    }
  }
  // block sums, laid out [block][kFusedVals]
  block_sum<kFusedVals>(acc, lds_red, res);
  __syncthreads();
  if (threadIdx.x < kFusedVals) partial[(int64_t)b * kFusedVals + threadIdx.x] = res[threadIdx.x];
}

// One COCG iteration in one pass on a 2-D grid (Ez polarisation: Ez on the
// nodes, Hx and Hy on the edges), with the recurrences and bilinear sums of
// k_cocg_fused3 (so k_cocg_scalar_fused and k_x_fixup serve both).  A block
// takes an xy tile of TX x TY electric positions of one right-hand side
// (blocks mapped to tiles and columns as in k_cocg_fused3, one z plane): it
// forms p_i on the tile with a one-cell halo in LDS (writing r_i, p_i and, on
// the passes that update it, x on the tile), then h = a22^-1 cp(p_i) on the
// tile with a low-side halo in LDS, then q_i = S p_i on the tile.  Magnetic
// coefficients per sample (UNI false: graded absorbers) or uniform; both
// masks are read.
template <typename T>
__device__ inline cplx<T> a22_times(cplx<T> a, cplx<T> c) { return a * c; }
template <typename T>
__device__ inline T a22_times(cplx<T> a, T c) { return a.re * c; }

template <typename T, typename V, int TX, int TY, bool XU, bool UNI>
__global__ void __launch_bounds__(TX * TY)
    k_cocg_fused2(const V* __restrict__ rin, const V* __restrict__ qin, const V* __restrict__ pin,
                  const V* __restrict__ p2in, V* __restrict__ rout, V* __restrict__ qout,
                  V* __restrict__ pout, V* __restrict__ x, const ColState* __restrict__ st,
                  const V* __restrict__ a11, const cplx<T>* __restrict__ a22inv, cplx<T> a22s,
                  const uint8_t* __restrict__ emask, const uint8_t* __restrict__ hmask,
                  Axes<T> ax, Geo g, int64_t ldE, int nx, int ny, FusedTiling ft, ColMap cm,
                  double zr, double zi, double* __restrict__ partial) {
  constexpr int NT = TX * TY;
  constexpr int PW = TX + 2, PH = TY + 2, PT = PW * PH;  // p tile with halo
  constexpr int HW = TX + 1, HH = TY + 1, HT = HW * HH;  // h tile, low-side halo
  constexpr int CW = FV<V>::CW;
  __shared__ T Ps[PT * CW];
  __shared__ T Hs[2 * HT * CW];  // Hx, Hy
  __shared__ double lds_red[kFusedVals * (NT / 64)];
  __shared__ double res[kFusedVals];
  V* P = reinterpret_cast<V*>(Ps);
  V* H = reinterpret_cast<V*>(Hs);
  const int b = blockIdx.x;
  const int xcd = b & 7, loc = b >> 3;
  const int col = cm.c[loc % cm.n];
  const int tl = xcd * ft.per_xcd + loc / cm.n;
  if (st[col].status != 0) return;  // a converged column keeps x, r and p
  double acc[kFusedVals];
#pragma clang loop unroll(full)
  for (int v = 0; v < kFusedVals; ++v) acc[v] = 0;
  if (tl < ft.ntiles) {
    const int i0 = (tl % ft.ntx) * TX, j0 = (tl / ft.ntx) * TY;
    const V alpha = FV<V>::mk(st[col].alpha_re, st[col].alpha_im);
    const V alpha1 = FV<V>::mk(st[col].alpha1_re, st[col].alpha1_im);
    const V beta = FV<V>::mk(st[col].beta_re, st[col].beta_im);
    const V z = FV<V>::mk(zr, zi);
    const int64_t co = col * ldE;
    const int X = g.X, Y = g.Y;
    // r_i, p_i on the tile and its halo (electric unknowns lie at i < nx,
    // j < ny: the tile's own positions are those)
    for (int idx = threadIdx.x; idx < PT; idx += NT) {
      const int lj = idx / PW, li = idx - lj * PW;
      const int i = i0 - 1 + li, j = j0 - 1 + lj;
      const bool ok = i >= 0 && j >= 0 && i < X && j < Y;
      const bool own = li >= 1 && li <= TX && lj >= 1 && lj <= TY && i < nx && j < ny;
      const int64_t gi = co + (ok ? (int64_t)j * X + i : 0);
      const V r0 = ok ? rin[gi] : V(0), q0 = ok ? qin[gi] : V(0), p0 = ok ? pin[gi] : V(0);
      const V rn = r0 - alpha * q0;
      const V pn = rn + beta * p0;
      P[idx] = pn;
      if (own) {
        rout[gi] = rn;
        pout[gi] = pn;
        if (XU) x[gi] = (x[gi] + alpha1 * p2in[gi]) + alpha * p0;
        FV<V>::bil(acc + 0, rn, rn);
        acc[2] += FV<V>::nrm(rn);
        FV<V>::bil(acc + 3, q0, pn);
      }
    }
    __syncthreads();
    // h = a22^-1 cp(p_i): Hx = -dEz/dy, Hy = dEz/dx
    for (int idx = threadIdx.x; idx < 2 * HT; idx += NT) {
      const int s = idx / HT, rem = idx - s * HT;
      const int hj = rem / HW, hi = rem - hj * HW;
      const int i = i0 - 1 + hi, j = j0 - 1 + hj;
      V v(0);
      if (i >= 0 && j >= 0 && i < X && j < Y) {
        const int64_t hg = (int64_t)s * g.len + (int64_t)j * X + i;
        if (hmask[hg] == 1) {
          const int pl = hj * PW + hi;  // p-tile index of (i, j)
          const V c = s == 0 ? (P[pl] - P[pl + PW]) * ax.ip[1][j] : (P[pl + 1] - P[pl]) * ax.ip[0][i];
          v = a22_times(UNI ? a22s : a22inv[hg], c);
        }
      }
      H[s * HT + rem] = v;
    }
    __syncthreads();
    // q_i = W_e (a11 p_i - z curl_d h) on the tile
    const T inv_v0 = (T)g.inv_v0;
    for (int idx = threadIdx.x; idx < TX * TY; idx += NT) {
      const int lj = idx / TX, li = idx - lj * TX;
      const int i = i0 + li, j = j0 + lj;
      if (i >= nx || j >= ny) continue;
      const int64_t e = (int64_t)j * X + i;
      const int hl = (lj + 1) * HW + (li + 1);  // h-tile index of (i, j)
      const V pn = P[(lj + 1) * PW + (li + 1)];
      V qn(0);
      if (emask[e] == 1) {
        const V cd = (H[HT + hl] - H[HT + hl - 1]) * ax.id[0][i] - (H[hl] - H[hl - HW]) * ax.id[1][j];
        const T w = ax.d[0][i] * ax.d[1][j] * ax.p[2][0] * inv_v0;
        qn = (a11[e] * pn - z * cd) * w;
      }
      qout[co + e] = qn;
      FV<V>::bil(acc + 5, pn, qn);
      FV<V>::bil(acc + 7, qn, qn);
    }
  }
  block_sum<kFusedVals>(acc, lds_red, res);
  __syncthreads();
  if (threadIdx.x < kFusedVals) partial[(int64_t)b * kFusedVals + threadIdx.x] = res[threadIdx.x];
}

// alpha_i = rho_i / sigma_i and, from r_{i+1} = r_i - alpha_i q_i,
//   rho_{i+1} = rho_i - 2 alpha_i r_i^T q_i + alpha_i^2 omega_i,
//   r_i^T q_i = sigma_i - beta_i p_{i-1}^T q_i = sigma_i - beta_i pi_i
// (S symmetric: p_{i-1}^T S p_i = q_{i-1}^T p_i), beta_{i+1} = rho_{i+1} / rho_i.
// Convergence is tested on the exact ||r_i||^2 of the pass; a finished column
// gets alpha = beta = 0, which freezes x and r in later passes.
// Block b of the pass served mapped column ((b >> 3) % cm.n); only the mapped
// columns are updated.  The sums run in a fixed order (deterministic).
template <int NB>
__global__ void __launch_bounds__(256)
    k_cocg_scalar_fused(ColState* __restrict__ st, const double* __restrict__ partial,
                        int per_xcd, ColMap cm, double tol2) {
  constexpr int NV = kFusedVals * NB;
  __shared__ double tot[NV];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nv = kFusedVals * cm.n;
  for (int pr = wid; pr < nv; pr += 4) {
    const int c = pr / kFusedVals, v = pr - c * kFusedVals;
    double sum = 0;
    for (int t = lane; t < 8 * per_xcd; t += 64) {
      const int b = (t & 7) + 8 * (c + cm.n * (t >> 3));
      sum += partial[(int64_t)b * kFusedVals + v];
    }
    sum = wave_sum(sum);
    if (lane == 0) tot[pr] = sum;
  }
  __syncthreads();
  if (threadIdx.x >= cm.n) return;
  const double* t = tot + threadIdx.x * kFusedVals;
  const int c = cm.c[threadIdx.x];
  ColState s = st[c];
  const zd beta_old(s.beta_re, s.beta_im);
  if (s.status == 0) {  // the alpha this pass used: the next x update needs it
    s.alpha1_re = s.alpha_re;
    s.alpha1_im = s.alpha_im;
  }
  s.alpha_re = s.alpha_im = s.beta_re = s.beta_im = 0;
  if (s.status == 0) {
    s.iters += 1;
    const zd rho(t[0], t[1]), pi(t[3], t[4]), sigma(t[5], t[6]), omega(t[7], t[8]);
    s.rr = t[2];
    if (s.rr <= tol2 * s.bb) {
      s.status = 1;
    } else if ((sigma.re == 0 && sigma.im == 0) || (rho.re == 0 && rho.im == 0)) {
      s.status = 2;
    } else {
      const zd a = cdiv(rho, sigma);
      const zd tau = sigma - beta_old * pi;
      const zd rho_next = rho - zd(2.0, 0.0) * a * tau + a * a * omega;
      const zd bn = cdiv(rho_next, rho);
      s.alpha_re = a.re;
      s.alpha_im = a.im;
      s.beta_re = bn.re;
      s.beta_im = bn.im;
      s.rho_re = rho_next.re;
      s.rho_im = rho_next.im;
    }
  }
  st[c] = s;
}

enum { kInit = 0, kAlpha = 1, kBeta = 2 };

template <int NB>
__global__ void __launch_bounds__(kBlock)
    k_cocg_scalar(ColState* __restrict__ st, const double* __restrict__ partial, int nblk,
                  int mode, double tol2) {
  __shared__ double lds[kMaxVals * (kBlock / 64)];
  __shared__ double tot[kMaxVals];
  constexpr int NV = 3 * NB;
  const int nv = mode == kAlpha ? 2 * NB : 3 * NB;
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x)
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (v < nv) acc[v] += partial[(int64_t)b * nv + v];
  block_sum<NV>(acc, lds, tot);
  __syncthreads();
  if (threadIdx.x >= NB) return;
  const int c = threadIdx.x;
  ColState s = st[c];
  if (mode == kInit) {
    s.rho_re = tot[3 * c];
    s.rho_im = tot[3 * c + 1];
    s.bb = tot[3 * c + 2];
    s.rr = s.bb;
    s.alpha_re = s.alpha_im = s.beta_re = s.beta_im = 0;
    s.alpha1_re = s.alpha1_im = 0;
    s.status = s.bb > 0 ? 0 : 1;
    s.iters = 0;
  } else if (mode == kAlpha) {
    s.alpha_re = s.alpha_im = 0;
    if (s.status == 0) {
      zd pq(tot[2 * c], tot[2 * c + 1]);
      if (pq.re == 0 && pq.im == 0) {
        s.status = 2;
      } else {
        zd a = cdiv(zd(s.rho_re, s.rho_im), pq);
        s.alpha_re = a.re;
        s.alpha_im = a.im;
      }
    }
  } else {
    s.beta_re = s.beta_im = 0;
    if (s.status == 0) {
      s.iters += 1;
      s.rr = tot[3 * c + 2];
      zd rho_new(tot[3 * c], tot[3 * c + 1]);
      if (s.rr <= tol2 * s.bb) {
        s.status = 1;
      } else if (s.rho_re == 0 && s.rho_im == 0) {
        s.status = 2;
      } else {
        zd b = cdiv(rho_new, zd(s.rho_re, s.rho_im));
        s.beta_re = b.re;
        s.beta_im = b.im;
        s.rho_re = rho_new.re;
        s.rho_im = rho_new.im;
      }
    }
  }
  st[c] = s;
}

template <typename T>
__global__ void k_copy_cols(cplx<T>* __restrict__ dst, const cplx<T>* __restrict__ src,
                            int64_t n, int64_t ld, int ncopy, int ntot) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= n) return;
  for (int c = 0; c < ntot; ++c)
    dst[c * ld + g] = (c < ncopy && src) ? src[c * ld + g] : cplx<T>(0, 0);
}

// The one-pass iteration updates x on odd passes only (x_i = x_{i-2} +
// alpha_{i-2} p_{i-2} + alpha_{i-1} p_{i-1}).  A column whose last pass L was
// even holds x_{L-1}: add alpha_{L-1} p_{L-1} (p_{L-1} sits in pb[L % 3]; the
// alpha that pass L used is alpha1 of its state).
template <typename V>
__global__ void k_x_fixup(V* __restrict__ x, const V* __restrict__ pb0, const V* __restrict__ pb1,
                          const V* __restrict__ pb2, const ColState* __restrict__ st, int64_t n,
                          int ncol) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < n * ncol;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(g / n);
    const int iters = st[c].iters;
    if (iters < 1 || ((iters - 1) & 1)) continue;  // no pass, or the last one was odd
    const int L = iters - 1;
    const V* pp = L % 3 == 0 ? pb0 : L % 3 == 1 ? pb1 : pb2;
    x[g] = x[g] + FV<V>::mk(st[c].alpha1_re, st[c].alpha1_im) * pp[g];
  }
}

// ---------------------------------------------------------------- solver

namespace {
struct Workspace {
  DevBuf x, r, p, q, h, r2, p2, q2, p3, partial, st;
  std::vector<ColState> host;
};
thread_local Workspace g_ws;
}  // namespace

void cocg_release_workspace() {
  for (DevBuf* b : {&g_ws.x, &g_ws.r, &g_ws.p, &g_ws.q, &g_ws.h, &g_ws.r2, &g_ws.p2, &g_ws.q2,
                    &g_ws.p3})
    b->release();
}

template <typename T, int NB>
static int cocg_chunk(const SchurOp<T>& S, const cplx<T>* bhat, cplx<T>* x1, int nbc,
                      const SolveOpts& o, SolveStats& stt, hipStream_t s) {
  const yr_operator* op = S.op;
  Geo g = geo_of(op);
  const int64_t nE = op->ne_slots * op->len, nH = op->nh_slots * op->len;
  Workspace& w = g_ws;
  YR_CALL(w.x.reserve(NB * nE * sizeof(cplx<T>)));
  YR_CALL(w.r.reserve(NB * nE * sizeof(cplx<T>)));
  YR_CALL(w.p.reserve(NB * nE * sizeof(cplx<T>)));
  YR_CALL(w.q.reserve(NB * nE * sizeof(cplx<T>)));
  // one-pass iteration where it applies: k_cocg_fused3 (3-D, uniform
  // magnetic materials), k_cocg_fused2 (2-D, any materials)
  using FC = FusedCfg<T>;
  constexpr int F2X = 64, F2Y = 8;  // 2-D tile: one wavefront per row
  const bool fused3 = op->dim == 3 && op->uniform_h && o.matvec != 1;
  const bool fused2 = op->dim == 2 && o.matvec != 1;
  const bool fused = fused3 || fused2;
  if (!fused) YR_CALL(w.h.reserve(NB * nH * sizeof(cplx<T>)));  // H intermediate of two sweeps
  // grid of one pass over `ncol` columns: z chunks so that the blocks (one
  // per compute unit: their LDS) fill the 256 units without a second round,
  // each chunk as long as possible (its two halo planes are re-read); 2-D:
  // one block per tile and column
  auto plan = [&](int ncol, FusedTiling& t) -> unsigned {
    if (fused2) {
      t.ntx = (op->nx + F2X - 1) / F2X;
      t.nty = (op->ny + F2Y - 1) / F2Y;
      t.ntiles = t.ntx * t.nty;
      t.KZ = t.nkz = 1;
      t.per_xcd = (t.ntiles + 7) / 8;
      return (unsigned)(8 * ncol * t.per_xcd);
    }
    t.ntx = (op->nx + FC::TX - 1) / FC::TX;
    t.nty = (op->ny + FC::TY - 1) / FC::TY;
    t.ntiles = t.ntx * t.nty;
    int nkz = std::min(std::max(1, 256 / (t.ntiles * ncol)), std::max(1, op->nz / 8));
    if (FC::NT == 1024) {
      // one workgroup per compute unit at a time: a pass takes
      // ceil(blocks / 256) rounds of (chunk planes + 2 halo planes); take
      // the chunk count that minimises that product, the fewer chunks on a
      // tie (256^3 with 13 of 16 columns active: 4 chunks, 3328 blocks, 13
      // full rounds, instead of 1 chunk, 832 blocks and a quarter-full 4th)
      int64_t best = -1;
      for (int c = 1; c <= std::max(1, op->nz / 8); ++c) {
        const int kz = (op->nz + c - 1) / c, nk = (op->nz + kz - 1) / kz;
        const int64_t blocks = 8LL * ncol * ((t.ntiles * nk + 7) / 8);
        const int64_t cost = (blocks + 255) / 256 * (kz + 2);
        if (best < 0 || cost < best) {
          best = cost;
          nkz = c;
        }
      }
    }
    t.KZ = (op->nz + nkz - 1) / nkz;
    t.nkz = (op->nz + t.KZ - 1) / t.KZ;
    t.per_xcd = (t.ntiles * t.nkz + 7) / 8;
    return (unsigned)(8 * ncol * t.per_xcd);
  };
  static_assert(NB <= kMaxCols, "column map too small");
  FusedTiling ft{};
  unsigned gF = 0, gF_max = 0;
  ColMap cm{};
  cm.n = nbc;
  for (int c = 0; c < nbc; ++c) cm.c[c] = c;
  if (fused) {
    for (int n = 1; n <= nbc; ++n) gF_max = std::max(gF_max, plan(n, ft));
    gF = plan(nbc, ft);
    YR_CALL(w.r2.reserve(NB * nE * sizeof(cplx<T>)));
    YR_CALL(w.p2.reserve(NB * nE * sizeof(cplx<T>)));
    YR_CALL(w.p3.reserve(NB * nE * sizeof(cplx<T>)));
    YR_CALL(w.q2.reserve(NB * nE * sizeof(cplx<T>)));
  }
  YR_CALL(w.partial.reserve(std::max<size_t>((size_t)kRedBlocksMax * 3 * NB,
                                             (size_t)gF_max * kFusedVals) * sizeof(double)));
  YR_CALL(w.st.reserve(NB * sizeof(ColState)));
  cplx<T>* x = w.x.as<cplx<T>>();
  cplx<T>* r = w.r.as<cplx<T>>();
  cplx<T>* p = w.p.as<cplx<T>>();
  cplx<T>* q = w.q.as<cplx<T>>();
  cplx<T>* h = w.h.as<cplx<T>>();
  double* part = w.partial.as<double>();
  ColState* st = w.st.as<ColState>();
  Axes<T> ax = op->axes<T>();
  const uint8_t* em = op->emask.as<uint8_t>();
  const uint8_t* hm = op->hmask.as<uint8_t>();

  k_copy_cols<T><<<grid_for(nE), kBlock, 0, s>>>(r, bhat, nE, nE, nbc, NB);
  k_copy_cols<T><<<grid_for(nE), kBlock, 0, s>>>(x, nullptr, nE, nE, 0, NB);
  k_copy_cols<T><<<grid_for(nE), kBlock, 0, s>>>(p, nullptr, nE, nE, 0, NB);
  cplx<T>* rb[2] = {r, fused ? w.r2.as<cplx<T>>() : r};
  // p rotates over three buffers in the one-pass iteration: pass i reads
  // p_{i-1} from pb[i % 3] and p_{i-2} from pb[(i + 2) % 3] and writes p_i to
  // pb[(i + 1) % 3] (p_{-1} = p_{-2} = 0)
  cplx<T>* pb[3] = {p, fused ? w.p2.as<cplx<T>>() : p, fused ? w.p3.as<cplx<T>>() : p};
  cplx<T>* qb[2] = {q, fused ? w.q2.as<cplx<T>>() : q};
  if (fused) {  // positions no pass writes (i = nx, j = ny, k = nz) stay zero
    k_copy_cols<T><<<grid_for(nE), kBlock, 0, s>>>(q, nullptr, nE, nE, 0, NB);
    k_copy_cols<T><<<grid_for(nE), kBlock, 0, s>>>(rb[1], nullptr, nE, nE, 0, NB);
    k_copy_cols<T><<<grid_for(nE), kBlock, 0, s>>>(pb[1], nullptr, nE, nE, 0, NB);
    k_copy_cols<T><<<grid_for(nE), kBlock, 0, s>>>(pb[2], nullptr, nE, nE, 0, NB);
    k_copy_cols<T><<<grid_for(nE), kBlock, 0, s>>>(qb[1], nullptr, nE, nE, 0, NB);
  }
  int cur = 0;
  const unsigned gE = red_grid(nE), gL = red_grid(op->len);
  k_cocg_update<T, NB><<<gE, kBlock, 0, s>>>(x, r, p, q, st, nE, nE, 0, part);
  k_cocg_scalar<NB><<<1, kBlock, 0, s>>>(st, part, gE, kInit, o.tol * o.tol);
  YR_TRY_HIP(hipGetLastError());
  // real shift: the system and its right-hand sides are real, so the one-pass
  // kernel runs in real arithmetic on real views of the same buffers (half
  // the bytes of the complex iteration)
  const bool real = fused && S.z.im == 0;
  T *rr[2] = {nullptr, nullptr}, *pr[3] = {nullptr, nullptr, nullptr}, *qr[2] = {nullptr, nullptr},
    *xr = nullptr;
  if (real) {
    const int64_t nr = NB * nE;
    rr[0] = w.r2.as<T>();
    rr[1] = w.r.as<T>();
    pr[0] = w.p.as<T>();
    pr[1] = w.p2.as<T>();
    pr[2] = w.p3.as<T>();
    qr[0] = w.q.as<T>();
    qr[1] = w.q2.as<T>();
    xr = w.x.as<T>();
    k_real_part<T><<<grid_for(nr), kBlock, 0, s>>>(r, rr[0], nr);  // before r is reused
    for (T* b : {rr[1], pr[0], pr[1], pr[2], qr[0], qr[1], xr})
      k_zero_real<T><<<grid_for(nr), kBlock, 0, s>>>(b, nr);
    YR_TRY_HIP(hipGetLastError());
  }
  const double zr = S.z.re, zi = S.z.im;
  const cplx<T>* a22 = op->uniform_h ? nullptr : S.a22inv.template as<cplx<T>>();
  w.host.resize(NB);
  int it = 0;
  bool done = false;
  for (; it < o.max_iter && !done; ++it) {
    if (fused) {
      {
        ProfScope ps(real ? "cocg_fused_real" : "cocg_fused", s);
        const int p1 = it % 3, p0 = (it + 1) % 3, p2 = (it + 2) % 3;  // p_{i-1}, p_i, p_{i-2}
        // x is updated on odd passes only, with the p and alpha of two passes
        auto launch = [&](auto xu) {
          constexpr bool XU = decltype(xu)::value;
          if (fused2) {
            const cplx<T>* a22v = op->uniform_h ? nullptr : S.a22inv.template as<cplx<T>>();
            const uint8_t* hm2 = op->hmask.as<uint8_t>();
            if (real) {
              auto* k = op->uniform_h ? k_cocg_fused2<T, T, F2X, F2Y, XU, true>
                                      : k_cocg_fused2<T, T, F2X, F2Y, XU, false>;
              k<<<gF, F2X * F2Y, 0, s>>>(rr[cur], qr[cur], pr[p1], pr[p2], rr[1 - cur], qr[1 - cur],
                                         pr[p0], xr, st, S.a11r.template as<T>(), a22v, S.a22inv_s,
                                         em, hm2, ax, g, nE, op->nx, op->ny, ft, cm, zr, 0.0, part);
            } else {
              auto* k = op->uniform_h ? k_cocg_fused2<T, cplx<T>, F2X, F2Y, XU, true>
                                      : k_cocg_fused2<T, cplx<T>, F2X, F2Y, XU, false>;
              k<<<gF, F2X * F2Y, 0, s>>>(rb[cur], qb[cur], pb[p1], pb[p2], rb[1 - cur], qb[1 - cur],
                                         pb[p0], x, st, S.a11.template as<cplx<T>>(), a22v,
                                         S.a22inv_s, em, hm2, ax, g, nE, op->nx, op->ny, ft, cm, zr,
                                         zi, part);
            }
            return;
          }
          if (real)
            k_cocg_fused3<T, T, FC::TX, FC::TY, FC::NT, XU><<<gF, FC::NT, 0, s>>>(
                rr[cur], qr[cur], pr[p1], pr[p2], rr[1 - cur], qr[1 - cur], pr[p0], xr, st,
                S.a11r.template as<T>(), S.a22inv_s.re, em, ax, g, nE, op->nx, op->ny, op->nz,
                ft, cm, zr, 0.0, part);
          else
            k_cocg_fused3<T, cplx<T>, FC::TX, FC::TY, FC::NT, XU><<<gF, FC::NT, 0, s>>>(
                rb[cur], qb[cur], pb[p1], pb[p2], rb[1 - cur], qb[1 - cur], pb[p0], x, st,
                S.a11.template as<cplx<T>>(), S.a22inv_s, em, ax, g, nE, op->nx, op->ny, op->nz,
                ft, cm, zr, zi, part);
        };
        if (it & 1) launch(std::true_type{});
        else launch(std::false_type{});
      }
      k_cocg_scalar_fused<NB><<<1, 256, 0, s>>>(st, part, ft.per_xcd, cm, o.tol * o.tol);
      cur = 1 - cur;
    } else {
    {
      ProfScope ps("schur_h", s);
      if (op->uniform_h)
        k_schur_h<T, NB, true><<<gL, kBlock, 0, s>>>(r, p, st, h, a22, S.a22inv_s, hm, ax, g, nE,
                                                    nH, 1);
      else
        k_schur_h<T, NB, false><<<gL, kBlock, 0, s>>>(r, p, st, h, a22, S.a22inv_s, hm, ax, g, nE,
                                                     nH, 1);
    }
    {
      ProfScope ps("schur_e", s);
      k_schur_e<T, NB><<<gL, kBlock, 0, s>>>(r, p, st, h, q, S.a11.template as<cplx<T>>(), em, ax, g,
                                            nE, nH, zr, zi, 1, part);
    }
    k_cocg_scalar<NB><<<1, kBlock, 0, s>>>(st, part, gL, kAlpha, o.tol * o.tol);
    {
      ProfScope ps("cocg_update", s);
      k_cocg_update<T, NB><<<gE, kBlock, 0, s>>>(x, r, p, q, st, nE, nE, 1, part);
    }
    k_cocg_scalar<NB><<<1, kBlock, 0, s>>>(st, part, gE, kBeta, o.tol * o.tol);
    }
    if ((it + 1) % o.check_every == 0 || it + 1 == o.max_iter) {
      YR_TRY_HIP(hipMemcpyAsync(w.host.data(), st, NB * sizeof(ColState), hipMemcpyDeviceToHost, s));
      YR_TRY_HIP(hipStreamSynchronize(s));
      done = true;
      for (int c = 0; c < NB; ++c) done = done && w.host[c].status != 0;
      if (fused && !done) {  // next passes: the columns still iterating
        ColMap nm{};
        for (int c = 0; c < nbc; ++c)
          if (w.host[c].status == 0) nm.c[nm.n++] = c;
        if (nm.n != cm.n) {
          cm = nm;
          gF = plan(cm.n, ft);
        }
      }
    }
  }
  YR_TRY_HIP(hipGetLastError());
  YR_TRY_HIP(hipMemcpyAsync(w.host.data(), st, NB * sizeof(ColState), hipMemcpyDeviceToHost, s));
  YR_TRY_HIP(hipStreamSynchronize(s));
  stt.iters += it;
  if (fused) {  // a column's passes stop when it converges
    for (int c = 0; c < nbc; ++c) stt.matvecs += w.host[c].iters;
  } else {
    stt.matvecs += (int64_t)it * nbc;
  }
  bool ok = true;
  for (int c = 0; c < nbc; ++c) {
    const ColState& cs = w.host[c];
    double rel = cs.bb > 0 ? std::sqrt(cs.rr / cs.bb) : 0.0;
    if (rel > stt.relres_max) stt.relres_max = rel;
    if (cs.iters > stt.col_iters_max) stt.col_iters_max = cs.iters;
    if (cs.status != 1) ok = false;
  }
  if (fused) {
    const int64_t nx_all = (int64_t)nbc * nE;
    const unsigned gx = (unsigned)std::min<int64_t>(grid_for(nx_all), 65536);
    if (real)
      k_x_fixup<T><<<gx, kBlock, 0, s>>>(xr, pr[0], pr[1], pr[2], st, nE, nbc);
    else
      k_x_fixup<cplx<T>><<<gx, kBlock, 0, s>>>(x, pb[0], pb[1], pb[2], st, nE, nbc);
    YR_TRY_HIP(hipGetLastError());
  }
  if (real) {
    k_to_complex<T><<<grid_for((int64_t)nbc * nE), kBlock, 0, s>>>(xr, x1, (int64_t)nbc * nE);
    YR_TRY_HIP(hipGetLastError());
  } else {
    YR_TRY_HIP(hipMemcpyAsync(x1, x, (size_t)nbc * nE * sizeof(cplx<T>), hipMemcpyDeviceToDevice, s));
  }
  YR_REQUIRE(ok, YR_ENOCONV, "shifted solve did not reach the residual tolerance");
  return YR_OK;
}

template <typename T>
static int cocg_chunk_any(const SchurOp<T>& S, const cplx<T>* b, cplx<T>* x, int nbc,
                          const SolveOpts& o, SolveStats& st, hipStream_t s) {
  if (nbc == 1) return cocg_chunk<T, 1>(S, b, x, nbc, o, st, s);
  if (nbc <= 2) return cocg_chunk<T, 2>(S, b, x, nbc, o, st, s);
  if (nbc <= 4) return cocg_chunk<T, 4>(S, b, x, nbc, o, st, s);
  if (nbc <= 8) return cocg_chunk<T, 8>(S, b, x, nbc, o, st, s);
  return cocg_chunk<T, 16>(S, b, x, nbc, o, st, s);
}

template <typename T>
int cocg_solve(const SchurOp<T>& S, const cplx<T>* bhat, cplx<T>* x1, int nb, const SolveOpts& o,
               SolveStats& st, hipStream_t s) {
  const int64_t nE = S.op->ne_slots * S.op->len;
  for (int c0 = 0; c0 < nb; c0 += 16) {
    int nbc = nb - c0 < 16 ? nb - c0 : 16;
    const cplx<T>* b = bhat + c0 * nE;
    cplx<T>* x = x1 + c0 * nE;
    const SolveStats before = st;
    int rc = cocg_chunk_any<T>(S, b, x, nbc, o, st, s);
    // The 2-D one-pass form takes the next r^T r from the previous pass's
    // sums and needs a few per cent more iterations than the two-sweep form
    // on hard solves (the iris guide at M = 1.02: 19,448 vs 17,880 over a
    // q = 40 reduction); a chunk that reaches the cap that way is solved
    // again with two sweeps (its work counts, its residual does not).
    if (rc == YR_ENOCONV && S.op->dim == 2 && o.matvec == 0) {
      SolveStats retry = before;
      retry.iters += st.iters - before.iters;
      retry.matvecs += st.matvecs - before.matvecs;
      st = retry;
      SolveOpts o2 = o;
      o2.matvec = 1;
      rc = cocg_chunk_any<T>(S, b, x, nbc, o2, st, s);
    }
    if (rc != YR_OK) return rc;
  }
  return YR_OK;
}

// ---------------------------------------------------------------- right-hand sides

template <typename T, bool UNI>
__global__ void k_rhs_h(const zd* __restrict__ v, int64_t ldv, double hscale, int nb,
                        cplx<T>* __restrict__ gout, const double* __restrict__ mu,
                        const double* __restrict__ sm, const cplx<T>* __restrict__ a22inv,
                        cplx<T> a22s, const uint8_t* __restrict__ hmask, Axes<T> ax, Geo g,
                        double dt) {
  const int64_t nE = g.ne_slots * g.len, nH = g.nh_slots * g.len;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < g.len;
       t += (int64_t)gridDim.x * blockDim.x) {
    int i, j, k;
    decode(t, g, i, j, k);
    for (int s = 0; s < g.nh_slots; ++s) {
      int64_t gi = s * g.len + t;
      for (int c = 0; c < nb; ++c) {
        cplx<T> out(0, 0);
        if (hmask[gi] == 1) {
          const zd* vc = v + c * ldv;
          auto ev = [&](int sl, int64_t idx) { return cplx<T>(vc[sl * g.len + idx]); };
          cplx<T> cpv = curl_p<cplx<T>>(g, ax, s, t, i, j, k, ev);
          T pm = (T)(mu[gi] / dt + 0.5 * sm[gi]);
          cplx<T> v2 = cplx<T>(vc[nE + gi]) * (T)hscale;
          cplx<T> a = UNI ? a22s : a22inv[gi];
          out = a * (v2 * pm - cpv);
        }
        gout[c * nH + gi] = out;
      }
    }
  }
}

template <typename T>
__global__ void k_rhs_e(const zd* __restrict__ v, int64_t ldv, const cplx<T>* __restrict__ gin,
                        int nb, cplx<T>* __restrict__ bhat, const double* __restrict__ eps,
                        const double* __restrict__ sig, const uint8_t* __restrict__ emask,
                        Axes<T> ax, Geo g, double dt) {
  const int64_t nE = g.ne_slots * g.len, nH = g.nh_slots * g.len;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < g.len;
       t += (int64_t)gridDim.x * blockDim.x) {
    int i, j, k;
    decode(t, g, i, j, k);
    for (int s = 0; s < g.ne_slots; ++s) {
      int64_t gi = s * g.len + t;
      for (int c = 0; c < nb; ++c) {
        cplx<T> out(0, 0);
        if (emask[gi] == 1) {
          const cplx<T>* gc = gin + c * nH;
          auto hv = [&](int sl, int64_t idx) { return gc[sl * g.len + idx]; };
          cplx<T> cd = curl_d<cplx<T>>(g, ax, s, t, i, j, k, hv);
          T pe = (T)(eps[gi] / dt + 0.5 * sig[gi]);
          out = (cplx<T>(v[c * ldv + gi]) * pe + cd) * w_e<T>(g, ax, s, i, j, k);
        }
        bhat[c * nE + gi] = out;
      }
    }
  }
}

template <typename T, bool UNI>
__global__ void k_recover_pack(const cplx<T>* __restrict__ x1, const cplx<T>* __restrict__ gin,
                               int nb, double hs_out, zd* __restrict__ out, int64_t ldo,
                               const cplx<T>* __restrict__ a22inv, cplx<T> a22s,
                               const uint8_t* __restrict__ hmask, Axes<T> ax, Geo g, double zr,
                               double zi) {
  const int64_t nE = g.ne_slots * g.len, nH = g.nh_slots * g.len;
  const cplx<T> z((T)zr, (T)zi);
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < g.len;
       t += (int64_t)gridDim.x * blockDim.x) {
    int i, j, k;
    decode(t, g, i, j, k);
    for (int c = 0; c < nb; ++c)
      for (int s = 0; s < g.ne_slots; ++s) {
        int64_t gi = s * g.len + t;
        cplx<T> v = x1[c * nE + gi];
        out[c * ldo + gi] = zd(v.re, v.im);
      }
    for (int s = 0; s < g.nh_slots; ++s) {
      int64_t gi = s * g.len + t;
      for (int c = 0; c < nb; ++c) {
        cplx<T> x2(0, 0);
        if (hmask[gi] == 1) {
          const cplx<T>* xc = x1 + c * nE;
          auto ev = [&](int sl, int64_t idx) { return xc[sl * g.len + idx]; };
          cplx<T> a = UNI ? a22s : a22inv[gi];
          x2 = z * (a * curl_p<cplx<T>>(g, ax, s, t, i, j, k, ev));
          if (gin) x2 = x2 + gin[c * nH + gi];
        }
        out[c * ldo + nE + gi] = zd(hs_out * (double)x2.re, hs_out * (double)x2.im);
      }
    }
  }
}

template <typename T>
int rhs_magnetic(const SchurOp<T>& S, const zd* v, int64_t ldv, double hscale, int nb,
                 cplx<T>* gout, hipStream_t s) {
  const yr_operator* op = S.op;
  Geo g = geo_of(op);
  Axes<T> ax = op->axes<T>();
  const cplx<T>* a22 = op->uniform_h ? nullptr : S.a22inv.template as<cplx<T>>();
  if (op->uniform_h)
    k_rhs_h<T, true><<<red_grid(op->len), kBlock, 0, s>>>(
        v, ldv, hscale, nb, gout, op->mu_h.as<double>(), op->sigm_h.as<double>(), a22,
        S.a22inv_s, op->hmask.as<uint8_t>(), ax, g, S.dt);
  else
    k_rhs_h<T, false><<<red_grid(op->len), kBlock, 0, s>>>(
        v, ldv, hscale, nb, gout, op->mu_h.as<double>(), op->sigm_h.as<double>(), a22,
        S.a22inv_s, op->hmask.as<uint8_t>(), ax, g, S.dt);
  YR_TRY_HIP(hipGetLastError());
  return YR_OK;
}

template <typename T>
int rhs_electric(const SchurOp<T>& S, const zd* v, int64_t ldv, const cplx<T>* gin, int nb,
                 cplx<T>* bhat, hipStream_t s) {
  const yr_operator* op = S.op;
  k_rhs_e<T><<<red_grid(op->len), kBlock, 0, s>>>(v, ldv, gin, nb, bhat, op->eps_e.as<double>(),
                                                 op->sig_e.as<double>(), op->emask.as<uint8_t>(),
                                                 op->axes<T>(), geo_of(op), S.dt);
  YR_TRY_HIP(hipGetLastError());
  return YR_OK;
}

template <typename T>
int recover_pack(const SchurOp<T>& S, const cplx<T>* x1, const cplx<T>* gin, int nb,
                 double hs_out, zd* out, int64_t ldo, hipStream_t s) {
  const yr_operator* op = S.op;
  const cplx<T>* a22 = op->uniform_h ? nullptr : S.a22inv.template as<cplx<T>>();
  if (op->uniform_h)
    k_recover_pack<T, true><<<red_grid(op->len), kBlock, 0, s>>>(
        x1, gin, nb, hs_out, out, ldo, a22, S.a22inv_s, op->hmask.as<uint8_t>(), op->axes<T>(),
        geo_of(op), S.z.re, S.z.im);
  else
    k_recover_pack<T, false><<<red_grid(op->len), kBlock, 0, s>>>(
        x1, gin, nb, hs_out, out, ldo, a22, S.a22inv_s, op->hmask.as<uint8_t>(), op->axes<T>(),
        geo_of(op), S.z.re, S.z.im);
  YR_TRY_HIP(hipGetLastError());
  return YR_OK;
}

template <typename T, int NB>
static int schur_apply_chunk(const SchurOp<T>& S, const cplx<T>* x, cplx<T>* y, hipStream_t s) {
  const yr_operator* op = S.op;
  Geo g = geo_of(op);
  const int64_t nE = op->ne_slots * op->len, nH = op->nh_slots * op->len;
  Workspace& w = g_ws;
  YR_CALL(w.p.reserve(NB * nE * sizeof(cplx<T>)));
  YR_CALL(w.h.reserve(NB * nH * sizeof(cplx<T>)));
  YR_CALL(w.partial.reserve((size_t)kRedBlocksMax * 3 * NB * sizeof(double)));
  YR_CALL(w.st.reserve(NB * sizeof(ColState)));
  cplx<T>* p = w.p.as<cplx<T>>();
  const unsigned gL = red_grid(op->len);
  const cplx<T>* a22 = op->uniform_h ? nullptr : S.a22inv.template as<cplx<T>>();
  Axes<T> ax = op->axes<T>();
  // p = 0, r = x, beta unused -> h = a22^-1 cp(x), y = S x
  k_copy_cols<T><<<grid_for(nE), kBlock, 0, s>>>(p, nullptr, nE, nE, 0, NB);
  if (op->uniform_h)
    k_schur_h<T, NB, true><<<gL, kBlock, 0, s>>>(x, p, w.st.as<ColState>(), w.h.as<cplx<T>>(),
                                                a22, S.a22inv_s, op->hmask.as<uint8_t>(), ax, g,
                                                nE, nH, 0);
  else
    k_schur_h<T, NB, false><<<gL, kBlock, 0, s>>>(x, p, w.st.as<ColState>(), w.h.as<cplx<T>>(),
                                                 a22, S.a22inv_s, op->hmask.as<uint8_t>(), ax, g,
                                                 nE, nH, 0);
  k_schur_e<T, NB><<<gL, kBlock, 0, s>>>(x, p, w.st.as<ColState>(), w.h.as<cplx<T>>(), y,
                                        S.a11.template as<cplx<T>>(), op->emask.as<uint8_t>(), ax, g, nE,
                                        nH, S.z.re, S.z.im, 0, w.partial.as<double>());
  YR_TRY_HIP(hipGetLastError());
  return YR_OK;
}

template <typename T>
int schur_apply(const SchurOp<T>& S, const cplx<T>* x, cplx<T>* y, int nb, hipStream_t s) {
  const int64_t nE = S.op->ne_slots * S.op->len;
  for (int c = 0; c < nb; ++c) YR_CALL((schur_apply_chunk<T, 1>(S, x + c * nE, y + c * nE, s)));
  return YR_OK;
}

template struct SchurOp<float>;
template struct SchurOp<double>;
template int cocg_solve<float>(const SchurOp<float>&, const cplx<float>*, cplx<float>*, int,
                               const SolveOpts&, SolveStats&, hipStream_t);
template int cocg_solve<double>(const SchurOp<double>&, const cplx<double>*, cplx<double>*, int,
                                const SolveOpts&, SolveStats&, hipStream_t);
template int rhs_magnetic<float>(const SchurOp<float>&, const zd*, int64_t, double, int,
                                 cplx<float>*, hipStream_t);
template int rhs_magnetic<double>(const SchurOp<double>&, const zd*, int64_t, double, int,
                                  cplx<double>*, hipStream_t);
template int rhs_electric<float>(const SchurOp<float>&, const zd*, int64_t, const cplx<float>*,
                                 int, cplx<float>*, hipStream_t);
template int rhs_electric<double>(const SchurOp<double>&, const zd*, int64_t,
                                  const cplx<double>*, int, cplx<double>*, hipStream_t);
template int recover_pack<float>(const SchurOp<float>&, const cplx<float>*, const cplx<float>*,
                                 int, double, zd*, int64_t, hipStream_t);
template int recover_pack<double>(const SchurOp<double>&, const cplx<double>*,
                                  const cplx<double>*, int, double, zd*, int64_t, hipStream_t);
template int schur_apply<float>(const SchurOp<float>&, const cplx<float>*, cplx<float>*, int,
                                hipStream_t);
template int schur_apply<double>(const SchurOp<double>&, const cplx<double>*, cplx<double>*, int,
                                 hipStream_t);

}  // namespace yr
