// Discrete adjoint of the full-order leapfrog eq. (MNAform) for objectives of
// the probe outputs y^n = L^T x^n (not in the paper; derived from the same
// equations).  With lambda^{N+1} = 0 and g^n = L dJ/dy^n, for n = N..1
//   (R+F)^T lambda^n = (R-F)^T lambda^{n+1} + g^n.
// (R+F)^T is block upper triangular, so each adjoint step solves the magnetic
// rows first and then the electric rows.  With mu_h = -lambda_h this is
//   mu_h^n     = da mu_h^{n+1} + db cp(lambda_e^{n+1})
//   lambda_e^n = ca lambda_e^{n+1} + cb curl_d(mu_h^n) + cb g_e^n / W_e,
// i.e. the forward half steps of the leapfrog run in reverse order: the
// stencil kernels of the forward sweep are reused unchanged (the transposed
// stencil of K^T is the other curl).  Gradients with respect to the
// per-sample field-form diagonals:
//   dJ/deps_e   = -W_e sum_n lambda_e^n (E^n - E^{n-1}) / dt
//   dJ/dsigma_e = -W_e sum_n lambda_e^n (E^n + E^{n-1}) / 2
// and to per-cell eps_r, sigma_e through the averaging weights.  The forward
// states are recomputed segment by segment from checkpoints taken every
// `ckpt` steps, so memory is nsteps/ckpt field buffers + ckpt electric halves.
#include <cmath>
#include <vector>

#include "fdtd_kernels.hpp"
#include "stencil.hpp"

namespace yr {

template <typename T>
__global__ void k_adj_grad(const T* __restrict__ lam, const T* __restrict__ En,
                           const T* __restrict__ Em, T* __restrict__ ge, T* __restrict__ gs,
                           Axes<T> ax, Geo g, T inv_dt) {
  const int64_t n = g.ne_slots * g.len;
  for (int64_t gi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; gi < n;
       gi += (int64_t)gridDim.x * blockDim.x) {
    T l = lam[gi];
    if (l == (T)0) continue;
    int s = (int)(gi / g.len);
    int64_t t = gi - s * g.len;
    int i, j, k;
    decode(t, g, i, j, k);
    T we = w_e<T>(g, ax, s, i, j, k);
    T en = En[gi], em = Em[gi];
    ge[gi] -= we * l * (en - em) * inv_dt;
    gs[gi] -= we * l * (en + em) * (T)0.5;
  }
}

template <typename T>
__global__ void k_accumulate(double* __restrict__ G, T* __restrict__ g, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) {
    G[i] += (double)g[i];
    g[i] = 0;
  }
}

// per-cell gradients: sum over the electric samples of the cell, weighted by
// the cell's share in each sample's dual-area average
__global__ void k_cell_grad(const double* __restrict__ Ge, const double* __restrict__ Gs,
                            const uint8_t* __restrict__ emask, Axes<double> ax, int dim, int nx,
                            int ny, int nz, int X, int Y, int64_t len, double eps0,
                            double* __restrict__ out_e, double* __restrict__ out_s) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t ncell = (int64_t)nx * ny * nz;
  if (c >= ncell) return;
  int i = (int)(c % nx);
  int64_t r = c / nx;
  int j = (int)(r % ny);
  int k = (int)(r / ny);
  const double *px = ax.p[0], *py = ax.p[1], *pz = ax.p[2];
  const double *dx = ax.d[0], *dy = ax.d[1], *dz = ax.d[2];
  double se = 0, ss = 0;
  auto add = [&](int slot, int ii, int jj, int kk, double a) {
    int64_t gi = slot * len + ((int64_t)kk * Y + jj) * X + ii;
    if (emask[gi] == 1) {
      se += a * Ge[gi];
      ss += a * Gs[gi];
    }
  };
  if (dim == 2) {
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        add(0, i + a, j + b, 0, px[i] * py[j] / (4.0 * dx[i + a] * dy[j + b]));
  } else {
    for (int b = 0; b < 2; ++b)
      for (int cc = 0; cc < 2; ++cc) {
        add(0, i, j + b, k + cc, py[j] * pz[k] / (4.0 * dy[j + b] * dz[k + cc]));
        add(1, i + b, j, k + cc, px[i] * pz[k] / (4.0 * dx[i + b] * dz[k + cc]));
        add(2, i + b, j + cc, k, px[i] * py[j] / (4.0 * dx[i + b] * dy[j + cc]));
      }
  }
  out_e[c] = eps0 * se;
  out_s[c] = ss;
}

template <typename T>
static int run_adjoint(yr_operator* op, double dt, int64_t N, const std::vector<PortEntry>& srcE,
                       int nsrc, const T* u, const std::vector<PortEntry>& prbE, int nprb,
                       const T* dJdy, int64_t K, double* out_e, double* out_s, hipStream_t s) {
  const int64_t nE = op->ne_slots * op->len;
  const int64_t F = (op->ne_slots + op->nh_slots) * op->len;
  const int64_t nck = (N + K - 1) / K;
  DevBuf ck, seg, cur, lam, ge, gs, Ge, Gs, sbuf, abuf, pbuf;
  YR_CALL(ck.reserve((size_t)nck * F * sizeof(T)));
  YR_CALL(seg.reserve((size_t)(K + 1) * nE * sizeof(T)));
  YR_CALL(cur.reserve((size_t)F * sizeof(T)));
  YR_CALL(lam.reserve((size_t)F * sizeof(T)));
  YR_CALL(ge.reserve((size_t)nE * sizeof(T)));
  YR_CALL(gs.reserve((size_t)nE * sizeof(T)));
  YR_CALL(Ge.reserve((size_t)nE * 8));
  YR_CALL(Gs.reserve((size_t)nE * 8));
  SrcList<T> sl{};
  SrcList<T> al{};
  PrbList<T> none{};
  YR_CALL(stage_src<T>(sbuf, srcE, nsrc, (int)e_blocks(op), sl, s));
  std::vector<PortEntry> adj = prbE;  // adjoint sources g_e / W_e at the probe samples
  for (auto& e : adj) e.w = e.w / host_we(op, e.slot);
  YR_CALL(stage_src<T>(abuf, adj, nprb, (int)e_blocks(op), al, s));
  YR_CALL(stage_prb<T>(pbuf, std::vector<PortEntry>(), 0, none, s));
  T* c = cur.as<T>();
  T* l = lam.as<T>();
  YR_TRY_HIP(hipMemsetAsync(c, 0, F * sizeof(T), s));
  YR_TRY_HIP(hipMemsetAsync(l, 0, F * sizeof(T), s));
  YR_TRY_HIP(hipMemsetAsync(ge.p, 0, nE * sizeof(T), s));
  YR_TRY_HIP(hipMemsetAsync(gs.p, 0, nE * sizeof(T), s));
  YR_TRY_HIP(hipMemsetAsync(Ge.p, 0, nE * 8, s));
  YR_TRY_HIP(hipMemsetAsync(Gs.p, 0, nE * 8, s));
  // forward sweep, checkpoints every K steps
  for (int64_t q = 0; q < nck; ++q) {
    YR_TRY_HIP(hipMemcpyAsync(ck.as<T>() + q * F, c, F * sizeof(T), hipMemcpyDeviceToDevice, s));
    const int64_t n1 = std::min(N, (q + 1) * K);
    for (int64_t n = q * K; n < n1; ++n) {
      launch_e<T>(op, c, sl, sl.n ? u + n * nsrc : nullptr, s);
      launch_h<T>(op, c, none, nullptr, s);
    }
  }
  Axes<T> ax = op->axes<T>();
  Geo g = geo_of(op);
  const T inv_dt = (T)(1.0 / dt);
  const unsigned gE = (unsigned)std::min<int64_t>(grid_for(nE), 8192);
  for (int64_t q = nck - 1; q >= 0; --q) {
    const int64_t n0 = q * K, n1 = std::min(N, n0 + K);
    T* E = seg.as<T>();
    YR_TRY_HIP(hipMemcpyAsync(c, ck.as<T>() + q * F, F * sizeof(T), hipMemcpyDeviceToDevice, s));
    YR_TRY_HIP(hipMemcpyAsync(E, c, nE * sizeof(T), hipMemcpyDeviceToDevice, s));
    for (int64_t n = n0; n < n1; ++n) {
      launch_e<T>(op, c, sl, sl.n ? u + n * nsrc : nullptr, s);
      launch_h<T>(op, c, none, nullptr, s);
      YR_TRY_HIP(hipMemcpyAsync(E + (n - n0 + 1) * nE, c, nE * sizeof(T), hipMemcpyDeviceToDevice, s));
    }
    for (int64_t n = n1; n > n0; --n) {
      launch_h<T>(op, l, none, nullptr, s);                        // mu_h^n
      launch_e<T>(op, l, al, dJdy + (n - 1) * nprb, s);           // lambda_e^n
      k_adj_grad<T><<<gE, kBlock, 0, s>>>(l, E + (n - n0) * nE, E + (n - n0 - 1) * nE, ge.as<T>(),
                                          gs.as<T>(), ax, g, inv_dt);
    }
    k_accumulate<T><<<grid_for(nE), kBlock, 0, s>>>(Ge.as<double>(), ge.as<T>(), nE);
    k_accumulate<T><<<grid_for(nE), kBlock, 0, s>>>(Gs.as<double>(), gs.as<T>(), nE);
    YR_TRY_HIP(hipGetLastError());
  }
  const int64_t ncell = (int64_t)op->nx * op->ny * op->nz;
  const double eps0 = 1.0 / (1.25663706212e-6 * 299792458.0 * 299792458.0);
  k_cell_grad<<<grid_for(ncell), kBlock, 0, s>>>(Ge.as<double>(), Gs.as<double>(),
                                                 op->emask.as<uint8_t>(), op->axes<double>(),
                                                 op->dim, op->nx, op->ny, op->nz, op->X, op->Y,
                                                 op->len, eps0, out_e, out_s);
  YR_TRY_HIP(hipGetLastError());
  YR_TRY_HIP(hipStreamSynchronize(s));  // the local buffers are freed on return
  return YR_OK;
}

}  // namespace yr

using namespace yr;

extern "C" int fdtd_adjoint(yr_operator* op, yr_dtype dtype, double dt, int64_t nsteps,
                            const yr_ports* src, const void* u, const yr_ports* probes,
                            const void* dJdy, int64_t ckpt_every, double* grad_eps_r,
                            double* grad_sigma_e, void* stream_) {
  YR_REQUIRE(op && grad_eps_r && grad_sigma_e, YR_EINVAL, "null argument");
  YR_REQUIRE(dtype == YR_F32 || dtype == YR_F64, YR_EINVAL, "bad dtype");
  YR_REQUIRE(nsteps > 0 && ckpt_every > 0, YR_EINVAL, "nsteps and ckpt_every must be > 0");
  YR_REQUIRE(dt > 0 && dt <= op->dt_max * (1 + 1e-12), YR_EUNSTABLE,
             "dt exceeds the CFL limit: the leapfrog would be unstable");
  YR_REQUIRE(probes && probes->n > 0 && dJdy, YR_EINVAL, "the objective needs probes and dJ/dy");
  int nsrc = src ? src->n : 0;
  YR_REQUIRE(nsrc == 0 || u, YR_EINVAL, "sources given without a waveform buffer");
  std::vector<PortEntry> se, pe;
  YR_CALL(resolve_ports(op, src, se, kBlock));
  YR_CALL(resolve_ports(op, probes, pe, kBlock));
  hipStream_t s = static_cast<hipStream_t>(stream_);
  YR_CALL(op_wait_idle(op));
  YR_CALL(ensure_coefficients(op, dt, dtype, s));
  int64_t K = std::min(ckpt_every, nsteps);
  if (dtype == YR_F64)
    return run_adjoint<double>(op, dt, nsteps, se, nsrc, (const double*)u, pe, probes->n,
                               (const double*)dJdy, K, grad_eps_r, grad_sigma_e, s);
  return run_adjoint<float>(op, dt, nsteps, se, nsrc, (const float*)u, pe, probes->n,
                            (const float*)dJdy, K, grad_eps_r, grad_sigma_e, s);
}
