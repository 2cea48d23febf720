// mor_reduce: structure-preserving (SPRIM) reduction of eq. (MNAform) with
// complex frequency hopping (Sec. II-C, IV-A, IV-B), and the reduced-model
// object's accessors.
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "krylov.hpp"
#include "orth.hpp"
#include "rom.hpp"

namespace yr {

namespace {
constexpr double kPi = 3.14159265358979323846;
constexpr double kMu0 = 1.25663706212e-6;
constexpr double kC0 = 299792458.0;
const double kEta0 = kMu0 * kC0;  // sqrt(mu0/eps0) = mu0 c0

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

template <typename T>
__global__ void k_fill_zero(cplx<T>* __restrict__ a, int64_t n) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g < n) a[g] = cplx<T>(0, 0);
}

template <typename T>
__global__ void k_scatter_real(cplx<T>* __restrict__ a, const int64_t* __restrict__ idx,
                               const double* __restrict__ val, int n) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) a[idx[g]] = a[idx[g]] + cplx<T>((T)val[g], 0);
}

// real parts (and imaginary parts when `both`) of complex columns -> real columns
__global__ void k_split(const zd* __restrict__ P, int64_t ldp, int64_t row0, int64_t nrows,
                        int ncol, int both, double* __restrict__ V, int64_t ldv) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= nrows) return;
  int o = 0;
  for (int c = 0; c < ncol; ++c) {
    zd v = P[c * ldp + row0 + g];
    V[(o++) * ldv + g] = v.re;
    if (both) V[(o++) * ldv + g] = v.im;
  }
}

// out_c = K v_c = -W_e curl_d(v_c) on electric unknowns (FP64, v: magnetic columns)
__global__ void k_apply_K(const double* __restrict__ V2, int64_t ldh, int ncol,
                          double* __restrict__ out, int64_t lde, const uint8_t* __restrict__ emask,
                          Axes<double> ax, Geo g) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < g.len;
       t += (int64_t)gridDim.x * blockDim.x) {
    int i, j, k;
    decode(t, g, i, j, k);
    for (int s = 0; s < g.ne_slots; ++s) {
      int64_t gi = s * g.len + t;
      for (int c = 0; c < ncol; ++c) {
        double v = 0;
        if (emask[gi] == 1) {
          const double* hc = V2 + c * ldh;
          auto hv = [&](int sl, int64_t idx) { return hc[sl * g.len + idx]; };
          v = -w_e<double>(g, ax, s, i, j, k) * curl_d<double>(g, ax, s, t, i, j, k, hv);
        }
        out[c * lde + gi] = v;
      }
    }
  }
}

// diagonal weights of eq. (matrix): W_e * material (electric) or W_f * material
__global__ void k_weights(double* __restrict__ out, const double* __restrict__ mat,
                          const uint8_t* __restrict__ mask, int electric, Axes<double> ax, Geo g) {
  int64_t n = (electric ? g.ne_slots : g.nh_slots) * g.len;
  int64_t gi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gi >= n) return;
  if (mask[gi] != 1) {
    out[gi] = 0;
    return;
  }
  int s = (int)(gi / g.len);
  int64_t t = gi - s * g.len;
  int i, j, k;
  decode(t, g, i, j, k);
  double w = electric ? w_e<double>(g, ax, s, i, j, k) : w_h<double>(g, ax, s, i, j, k);
  out[gi] = w * mat[gi];
}

// W_e * scale * (dual-area mean of a per-cell field) on the electric unknowns:
// the diagonal of dD/dtheta for a material change given per cell
__global__ void k_direction_e(double* __restrict__ out, const double* __restrict__ cells,
                              const uint8_t* __restrict__ emask, Axes<double> ax, Geo g, int nx,
                              int ny, double scale) {
  const int64_t n = g.ne_slots * g.len;
  int64_t gi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (gi >= n) return;
  if (emask[gi] != 1) {
    out[gi] = 0;
    return;
  }
  int s = (int)(gi / g.len);
  int64_t t = gi - s * g.len;
  int i, j, k;
  decode(t, g, i, j, k);
  const double *px = ax.p[0], *py = ax.p[1], *pz = ax.p[2];
  double ws = 0, v = 0;
  auto cell = [&](int a, int b, int c) { return cells[((int64_t)c * ny + b) * nx + a]; };
  for (int qq = 0; qq < 4; ++qq) {
    int a0 = qq & 1, b0 = qq >> 1;
    double wgt, val;
    if (g.dim == 2 || s == 2) {
      wgt = px[i - 1 + a0] * py[j - 1 + b0];
      val = cell(i - 1 + a0, j - 1 + b0, k);
    } else if (s == 0) {
      wgt = py[j - 1 + a0] * pz[k - 1 + b0];
      val = cell(i, j - 1 + a0, k - 1 + b0);
    } else {
      wgt = px[i - 1 + a0] * pz[k - 1 + b0];
      val = cell(i - 1 + a0, j, k - 1 + b0);
    }
    ws += wgt;
    v += wgt * val;
  }
  out[gi] = w_e<double>(g, ax, s, i, j, k) * scale * v / ws;
}

__global__ void k_gather_rows(const double* __restrict__ V, int64_t ld, int ncol,
                              const int64_t* __restrict__ rows, int nrows, double* __restrict__ out) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nrows * ncol) return;
  int r = g % nrows, c = g / nrows;
  out[g] = V[c * ld + rows[r]];
}

static int download_sym(const double* dev, int q, std::vector<double>& out, bool sym) {
  out.resize((size_t)q * q);
  if (q == 0) return YR_OK;
  YR_TRY_HIP(hipMemcpy(out.data(), dev, (size_t)q * q * 8, hipMemcpyDeviceToHost));
  if (sym)
    for (int a = 0; a < q; ++a)
      for (int b = 0; b < a; ++b) {
        double m = 0.5 * (out[a + b * q] + out[b + a * q]);
        out[a + b * q] = out[b + a * q] = m;
      }
  return YR_OK;
}

// rows^T of V at the port entries, combined with weights: out[q x nports]
static int port_projection(const yr_operator* op, const double* V, int64_t ld, int q,
                           const std::vector<PortEntry>& ents, int nports, bool scale_we,
                           std::vector<double>& out) {
  out.assign((size_t)q * nports, 0.0);
  if (ents.empty() || q == 0) return YR_OK;
  std::vector<int64_t> rows;
  for (const auto& e : ents) rows.push_back(e.slot);
  DevBuf drows, dout;
  YR_CALL(drows.reserve(rows.size() * 8));
  YR_CALL(dout.reserve(rows.size() * q * 8));
  YR_TRY_HIP(hipMemcpy(drows.p, rows.data(), rows.size() * 8, hipMemcpyHostToDevice));
  int n = (int)rows.size();
  k_gather_rows<<<grid_for((int64_t)n * q), kBlock>>>(V, ld, q, drows.as<int64_t>(), n,
                                                      dout.as<double>());
  YR_TRY_HIP(hipGetLastError());
  std::vector<double> h((size_t)n * q);
  YR_TRY_HIP(hipMemcpy(h.data(), dout.p, h.size() * 8, hipMemcpyDeviceToHost));
  for (int e = 0; e < n; ++e) {
    double w = ents[e].w * (scale_we ? host_we(op, ents[e].slot) : 1.0);
    for (int c = 0; c < q; ++c) out[c + (size_t)ents[e].port * q] += w * h[e + (size_t)c * n];
  }
  return YR_OK;
}

template <typename T>
static int reduce_impl(yr_operator* op, const std::vector<PortEntry>& src, int nsrc,
                       const std::vector<PortEntry>& prb, int nprb, int q, const yr_mor_opts& o,
                       yr_rom* rom) {
  hipStream_t s = nullptr;
  const int64_t nE = op->ne_slots * op->len, nH = op->nh_slots * op->len, N = nE + nH;
  const int L = o.L, b = nsrc;
  const bool pair = o.pair_only != 0;
  // real columns per point: the pair's q/2 complex vectors give all q
  const int k = pair ? q / 2 : q / (2 * L + 1);
  const int nblk = k / b;
  const int npts = pair ? 1 : L + 1;
  rom->nE = nE;
  rom->nH = nH;
  rom->nsrc = nsrc;
  rom->nprb = nprb;
  // SPRIM split for FP32 solves: the Krylov vectors carry ~1e-4 relative
  // error and deflation works at defl_tol >= 1e-7, which a CholQR2 on the FP64
  // Gram matrix of all raw columns resolves: two passes over V1 and V2 instead
  // of CGS2 of every block against all earlier ones.  FP64 solves (deflation
  // down to 1e-10) keep the blockwise CGS2.
  const bool gram_split = o.solve_dtype == YR_F32 && o.defl_tol >= 1e-7;
  // With one point (the conjugate pair) and the raw split, the point basis P
  // holds every column until the end: V1 and V2 are allocated and filled
  // after the solver's vectors are freed, so the two never coexist (at 256^3
  // cells, 16 ports and q = 128: 104 GB of P + 52 GB of solver vectors, then
  // 104 GB of P + 104 GB of V1 and V2, instead of all at once).
  const bool defer_split = gram_split && npts == 1;
  if (!defer_split) {
    YR_CALL(rom->V1.reserve((size_t)nE * q * 8));
    YR_CALL(rom->V2.reserve((size_t)nH * q * 8));
  }
  DevBuf P, bhat, x1, g;
  YR_CALL(P.reserve((size_t)N * k * sizeof(zd)));  // blocks fill [0, k) at most
  YR_CALL(bhat.reserve((size_t)nE * b * sizeof(cplx<T>)));
  YR_CALL(x1.reserve((size_t)nE * b * sizeof(cplx<T>)));
  YR_CALL(g.reserve((size_t)nH * b * sizeof(cplx<T>)));
  zd* Pb = P.as<zd>();
  double* V1 = rom->V1.as<double>();
  double* V2 = rom->V2.as<double>();
  // B_e scatter lists
  std::vector<int64_t> sidx;
  std::vector<double> sval;
  for (const auto& e : src) {
    sidx.push_back((int64_t)e.port * nE + e.slot);
    sval.push_back(e.w * host_we(op, e.slot));
  }
  DevBuf dsidx, dsval;
  YR_CALL(dsidx.reserve(sidx.size() * 8));
  YR_CALL(dsval.reserve(sval.size() * 8));
  YR_TRY_HIP(hipMemcpy(dsidx.p, sidx.data(), sidx.size() * 8, hipMemcpyHostToDevice));
  YR_TRY_HIP(hipMemcpy(dsval.p, sval.data(), sval.size() * 8, hipMemcpyHostToDevice));

  const bool verbose = std::getenv("YR_VERBOSE") != nullptr;
  SolveOpts so;
  so.tol = o.tol;
  so.max_iter = o.max_iter;
  so.matvec = o.matvec;
  SolveStats st;
  SchurOp<T> S;
  int j1 = 0, j2 = 0;
  double t_solve = 0, t_orth = 0;
  for (int l = 0; l < npts; ++l) {
    // eq. (distrib) for l = 0..L; the conjugate pair of Sec. V-C alone
    const bool real_pt = !pair && l == 0;
    const double th = pair ? 2.0 * kPi * o.fmax * o.dt_ref
                           : (L > 0 ? 2.0 * kPi * ((double)l / L) * o.fmax * o.dt_ref : 0.0);
    const zd z(o.M * std::cos(th), real_pt ? 0.0 : o.M * std::sin(th));
    YR_CALL(S.prepare(op, o.dt_ref, z, s));
    int kcur = 0, prev_first = 0, prev_n = 0;
    for (int m = 0; m < nblk; ++m) {
      double t0 = now();
      int nb;
      const cplx<T>* gptr = nullptr;
      if (m == 0) {
        nb = b;
        k_fill_zero<T><<<grid_for(nE * b), kBlock, 0, s>>>(bhat.as<cplx<T>>(), nE * b);
        k_scatter_real<T><<<grid_for((int64_t)sidx.size()), kBlock, 0, s>>>(
            bhat.as<cplx<T>>(), dsidx.as<int64_t>(), dsval.as<double>(), (int)sidx.size());
        YR_TRY_HIP(hipGetLastError());
      } else {
        nb = prev_n;
        const zd* v = Pb + (int64_t)prev_first * N;
        YR_CALL(rhs_magnetic<T>(S, v, N, 1.0 / kEta0, nb, g.as<cplx<T>>(), s));
        YR_CALL(rhs_electric<T>(S, v, N, g.as<cplx<T>>(), nb, bhat.as<cplx<T>>(), s));
        gptr = g.as<cplx<T>>();
      }
      YR_CALL(cocg_solve<T>(S, bhat.as<cplx<T>>(), x1.as<cplx<T>>(), nb, so, st, s));
      YR_CALL(recover_pack<T>(S, x1.as<cplx<T>>(), gptr, nb, kEta0, Pb + (int64_t)kcur * N, N, s));
      YR_TRY_HIP(hipStreamSynchronize(s));
      double t1 = now();
      t_solve += t1 - t0;
      int kept = 0;
      // one Gram-Schmidt pass when the split bases get their own FP64
      // CholQR2 at the end (the point basis then only feeds the deflation
      // test and the next right-hand side: its loss of orthogonality, eps
      // times the squared ratio of the block's norm before and after the
      // projection, stays far below the deflation tolerance of >= 1e-7)
      YR_CALL(orth_block<zd>(Pb, N, N, kcur, nb, o.defl_tol, &kept, nullptr, gram_split ? 1 : 2, s));
      if (kept > 0) {
        const int both = real_pt ? 0 : 1;
        const int nr = kept * (both ? 2 : 1);
        const zd* newc = Pb + (int64_t)kcur * N;
        if (!defer_split) {
          k_split<<<grid_for(nE), kBlock, 0, s>>>(newc, N, 0, nE, kept, both, V1 + (int64_t)j1 * nE, nE);
          k_split<<<grid_for(nH), kBlock, 0, s>>>(newc, N, nE, nH, kept, both, V2 + (int64_t)j2 * nH, nH);
          YR_TRY_HIP(hipGetLastError());
        }
        if (gram_split) {  // raw columns now, one CholQR2 of each split basis at the end
          j1 += nr;
          j2 += nr;
        } else {
          int k1 = 0, k2 = 0;
          YR_CALL(orth_block<double>(V1, nE, nE, j1, nr, o.defl_tol, &k1, nullptr, 2, s));
          YR_CALL(orth_block<double>(V2, nH, nH, j2, nr, o.defl_tol, &k2, nullptr, 2, s));
          j1 += k1;
          j2 += k2;
        }
      }
      t_orth += now() - t1;
      if (verbose)
        fprintf(stderr, "[mor_reduce] point %d block %d: %d cols, %lld iters so far, solve %.3fs orth %.3fs, V1 %d V2 %d\n",
                l, m, kept, (long long)st.iters, t1 - t0, now() - t1, j1, j2);
      prev_first = kcur;
      prev_n = kept;
      kcur += kept;
      if (kept == 0) break;
    }
  }
  if (defer_split) {
    // one complex point: the split of all kept columns [0, j1 / 2) in one
    // call (the same interleaved order as block by block), after the solver's
    // vectors and the right-hand-side buffers are freed; then P is freed
    cocg_release_workspace();
    bhat.release();
    x1.release();
    g.release();
    const double t3 = now();
    YR_CALL(rom->V1.reserve((size_t)nE * q * 8));
    YR_CALL(rom->V2.reserve((size_t)nH * q * 8));
    V1 = rom->V1.as<double>();
    V2 = rom->V2.as<double>();
    if (j1 > 0) {
      k_split<<<grid_for(nE), kBlock, 0, s>>>(Pb, N, 0, nE, j1 / 2, 1, V1, nE);
      k_split<<<grid_for(nH), kBlock, 0, s>>>(Pb, N, nE, nH, j2 / 2, 1, V2, nH);
      YR_TRY_HIP(hipGetLastError());
    }
    YR_TRY_HIP(hipStreamSynchronize(s));
    P.release();
    t_orth += now() - t3;
  }
  if (gram_split) {
    const double t3 = now();
    int k1 = 0, k2 = 0;
    YR_CALL(cholqr2_columns(rom->V1, nE, j1, o.defl_tol, &k1, s));
    YR_CALL(cholqr2_columns(rom->V2, nH, j2, o.defl_tol, &k2, s));
    V1 = rom->V1.as<double>();  // the passes swap buffers
    V2 = rom->V2.as<double>();
    j1 = k1;
    j2 = k2;
    t_orth += now() - t3;
  }
  rom->q1 = j1;
  rom->q2 = j2;
  rom->deflated = q - std::min(j1, j2);
  rom->solve_iters = st.iters;
  rom->matvecs = st.matvecs;
  rom->relres_max = st.relres_max;
  rom->seconds_solve = t_solve;
  rom->seconds_orth = t_orth;

  // ---- projection, eq. (R_and_Freduced), FP64
  double t2 = now();
  Geo geo = geo_of(op);
  Axes<double> ax = op->axes<double>();
  DevBuf w, Cd, KV;
  YR_CALL(w.reserve((size_t)std::max(nE, nH) * 8));
  int qm = std::max(j1, j2);
  YR_CALL(Cd.reserve((size_t)std::max(1, qm * qm) * 8));
  struct Item {
    const double* mat;
    const uint8_t* mask;
    int electric;
    std::vector<double>* out;
  } items[4] = {{op->eps_e.as<double>(), op->emask.as<uint8_t>(), 1, &rom->De},
                {op->sig_e.as<double>(), op->emask.as<uint8_t>(), 1, &rom->Dse},
                {op->mu_h.as<double>(), op->hmask.as<uint8_t>(), 0, &rom->Dm},
                {op->sigm_h.as<double>(), op->hmask.as<uint8_t>(), 0, &rom->Dsm}};
  for (auto& it : items) {
    int qq = it.electric ? j1 : j2;
    int64_t n = it.electric ? nE : nH;
    const double* V = it.electric ? V1 : V2;
    if ((it.out == &rom->Dse && op->lossless_e) || (it.out == &rom->Dsm && op->uniform_h)) {
      it.out->assign((size_t)qq * qq, 0.0);  // no loss anywhere: the projection is exactly 0
      continue;
    }
    k_weights<<<grid_for(n), kBlock, 0, s>>>(w.as<double>(), it.mat, it.mask, it.electric, ax, geo);
    YR_TRY_HIP(hipGetLastError());
    if (qq > 0)
      YR_CALL(gemm_tn_weighted(V, n, qq, V, n, qq, w.as<double>(), n, Cd.as<double>(), qq, s));
    YR_TRY_HIP(hipStreamSynchronize(s));
    YR_CALL(download_sym(Cd.as<double>(), qq, *it.out, true));
  }
  // K~ = V1^T (K V2)
  rom->K.assign((size_t)j1 * j2, 0.0);
  if (j1 > 0 && j2 > 0) {
    YR_CALL(KV.reserve((size_t)nE * j2 * 8));
    k_apply_K<<<std::min<int64_t>(grid_for(op->len), 4096), kBlock, 0, s>>>(
        V2, nH, j2, KV.as<double>(), nE, op->emask.as<uint8_t>(), ax, geo);
    YR_TRY_HIP(hipGetLastError());
    YR_CALL(gemm_tn_weighted(V1, nE, j1, KV.as<double>(), nE, j2, nullptr, nE, Cd.as<double>(), j1, s));
    YR_TRY_HIP(hipStreamSynchronize(s));
    YR_TRY_HIP(hipMemcpy(rom->K.data(), Cd.p, (size_t)j1 * j2 * 8, hipMemcpyDeviceToHost));
  }
  YR_CALL(port_projection(op, V1, nE, j1, src, nsrc, true, rom->B1));
  YR_CALL(port_projection(op, V1, nE, j1, prb, nprb, false, rom->L1));
  rom->B2.assign((size_t)j2 * nsrc, 0.0);
  rom->L2.assign((size_t)j2 * nprb, 0.0);
  rom->Kp = rom->K;
  rom->seconds_project = now() - t2;
  return YR_OK;
}

static size_t mat_size(const yr_rom* r, int which, std::vector<double>** v) {
  yr_rom* m = const_cast<yr_rom*>(r);
  switch (which) {
    case YR_ROM_DE: *v = &m->De; return (size_t)r->q1 * r->q1;
    case YR_ROM_DSE: *v = &m->Dse; return (size_t)r->q1 * r->q1;
    case YR_ROM_DM: *v = &m->Dm; return (size_t)r->q2 * r->q2;
    case YR_ROM_DSM: *v = &m->Dsm; return (size_t)r->q2 * r->q2;
    case YR_ROM_K: *v = &m->K; return (size_t)r->q1 * r->q2;
    case YR_ROM_KP: *v = &m->Kp; return (size_t)r->q1 * r->q2;
    case YR_ROM_B1: *v = &m->B1; return (size_t)r->q1 * r->nsrc;
    case YR_ROM_B2: *v = &m->B2; return (size_t)r->q2 * r->nsrc;
    case YR_ROM_L1: *v = &m->L1; return (size_t)r->q1 * r->nprb;
    case YR_ROM_L2: *v = &m->L2; return (size_t)r->q2 * r->nprb;
    case YR_ROM_SIGMA: *v = &m->sigma; return (size_t)std::min(r->q1, r->q2);
    default: *v = nullptr; return 0;
  }
}

}  // namespace yr

using namespace yr;

extern "C" {

int mor_reduce(yr_operator* op, const yr_ports* src, const yr_ports* probes, int32_t q,
               const yr_mor_opts* opts, yr_rom** out) {
  YR_REQUIRE(op && src && opts && out, YR_EINVAL, "null argument");
  *out = nullptr;
  const yr_mor_opts& o = *opts;
  YR_REQUIRE(src->n >= 1, YR_EINVAL, "at least one source port is needed");
  YR_REQUIRE(o.pair_only == 0 || o.pair_only == 1, YR_EINVAL, "pair_only must be 0 or 1");
  YR_REQUIRE(o.L >= 0 && o.M > 0 && o.dt_ref > 0 && o.tol > 0 && o.max_iter > 0 &&
                 o.defl_tol > 0 && ((o.L == 0 && !o.pair_only) || o.fmax > 0),
             YR_EINVAL, "bad reduction options");
  YR_REQUIRE(o.solve_dtype == YR_F32 || o.solve_dtype == YR_F64, YR_EINVAL, "bad solve dtype");
  YR_REQUIRE(o.matvec >= 0 && o.matvec <= 2, YR_EINVAL,
             "matvec must be 0 (auto), 1 (two sweeps) or 2 (one pass)");
  if (o.pair_only) {
    YR_REQUIRE(q > 0 && q % (2 * src->n) == 0, YR_EINVAL,
               "with a conjugate pair, q must be a positive multiple of 2 x the source ports");
  } else {
    YR_REQUIRE(q > 0 && q % (2 * o.L + 1) == 0, YR_EINVAL,
               "q must be a positive multiple of the number of points 2L+1");
    YR_REQUIRE((q / (2 * o.L + 1)) % src->n == 0, YR_EINVAL,
               "q/(2L+1) must be a multiple of the number of source ports");
  }
  std::vector<PortEntry> se, pe;
  YR_CALL(resolve_ports(op, src, se, kBlock));
  YR_CALL(resolve_ports(op, probes, pe, kBlock));
  std::unique_ptr<yr_rom> rom(new (std::nothrow) yr_rom());
  YR_REQUIRE(rom, YR_ENOMEM, "host allocation failed");
  int nprb = probes ? probes->n : 0;
  int rc = o.solve_dtype == YR_F64
               ? reduce_impl<double>(op, se, src->n, pe, nprb, q, o, rom.get())
               : reduce_impl<float>(op, se, src->n, pe, nprb, q, o, rom.get());
  if (rc != YR_OK) return rc;
  *out = rom.release();
  return YR_OK;
}

int yr_rom_info(const yr_rom* r, yr_rom_info_t* info) {
  YR_REQUIRE(r && info, YR_EINVAL, "null argument");
  info->q1 = r->q1;
  info->q2 = r->q2;
  info->nsrc = r->nsrc;
  info->nprb = r->nprb;
  info->deflated = r->deflated;
  info->solve_iters = r->solve_iters;
  info->matvecs = r->matvecs;
  info->relres_max = r->relres_max;
  info->seconds_solve = r->seconds_solve;
  info->seconds_orth = r->seconds_orth;
  info->seconds_project = r->seconds_project;
  info->n_clamped = r->n_clamped;
  info->step_dt = r->step_dt;
  info->guard_margin = r->guard_margin;
  return YR_OK;
}

int yr_rom_get(const yr_rom* r, int32_t which, double* host_out) {
  YR_REQUIRE(r && host_out, YR_EINVAL, "null argument");
  std::vector<double>* v;
  size_t n = mat_size(r, which, &v);
  YR_REQUIRE(v, YR_EINVAL, "unknown matrix id");
  YR_REQUIRE(v->size() == n || n == 0, YR_ESTATE, "matrix not available");
  if (n) std::memcpy(host_out, v->data(), n * 8);
  return YR_OK;
}

int yr_rom_set(yr_rom* r, int32_t which, const double* host_in) {
  YR_REQUIRE(r && host_in, YR_EINVAL, "null argument");
  YR_REQUIRE(which != YR_ROM_KP && which != YR_ROM_SIGMA, YR_EINVAL, "matrix is read-only");
  std::vector<double>* v;
  size_t n = mat_size(r, which, &v);
  YR_REQUIRE(v, YR_EINVAL, "unknown matrix id");
  v->assign(host_in, host_in + n);
  if (which == YR_ROM_K) r->Kp = r->K;
  r->step_dt = -1;
  r->step_dtype = -1;
  return YR_OK;
}

int yr_rom_create(int32_t q1, int32_t q2, int32_t nsrc, int32_t nprb, yr_rom** out) {
  YR_REQUIRE(out && q1 > 0 && q2 > 0 && nsrc >= 0 && nprb >= 0, YR_EINVAL, "bad sizes");
  std::unique_ptr<yr_rom> r(new (std::nothrow) yr_rom());
  YR_REQUIRE(r, YR_ENOMEM, "host allocation failed");
  r->q1 = q1;
  r->q2 = q2;
  r->nsrc = nsrc;
  r->nprb = nprb;
  r->De.assign((size_t)q1 * q1, 0.0);
  r->Dse.assign((size_t)q1 * q1, 0.0);
  r->Dm.assign((size_t)q2 * q2, 0.0);
  r->Dsm.assign((size_t)q2 * q2, 0.0);
  r->K.assign((size_t)q1 * q2, 0.0);
  r->Kp = r->K;
  r->B1.assign((size_t)q1 * nsrc, 0.0);
  r->B2.assign((size_t)q2 * nsrc, 0.0);
  r->L1.assign((size_t)q1 * nprb, 0.0);
  r->L2.assign((size_t)q2 * nprb, 0.0);
  *out = r.release();
  return YR_OK;
}

int yr_rom_basis(const yr_rom* r, void* V1, void* V2) {
  YR_REQUIRE(r, YR_EINVAL, "null argument");
  YR_REQUIRE(r->nE > 0, YR_ESTATE, "model has no projection basis");
  if (V1) YR_TRY_HIP(hipMemcpy(V1, r->V1.p, (size_t)r->nE * r->q1 * 8, hipMemcpyDeviceToDevice));
  if (V2) YR_TRY_HIP(hipMemcpy(V2, r->V2.p, (size_t)r->nH * r->q2 * 8, hipMemcpyDeviceToDevice));
  return YR_OK;
}

void yr_rom_destroy(yr_rom* r) { delete r; }

int yr_rom_project_cells(yr_operator* op, const yr_rom* rom, const double* cell_values,
                         int32_t which, double* out) {
  YR_REQUIRE(op && rom && cell_values && out, YR_EINVAL, "null argument");
  YR_REQUIRE(rom->nE == op->ne_slots * op->len, YR_ESTATE, "model was not reduced from this operator");
  YR_REQUIRE(which == 0 || which == 1, YR_EINVAL, "which must be 0 (eps_r) or 1 (sigma_e)");
  const int64_t ncell = (int64_t)op->nx * op->ny * op->nz;
  const int64_t nE = rom->nE;
  DevBuf dc, w, C;
  YR_CALL(dc.reserve(ncell * 8));
  YR_CALL(w.reserve(nE * 8));
  YR_CALL(C.reserve((size_t)rom->q1 * rom->q1 * 8 + 8));
  YR_TRY_HIP(hipMemcpy(dc.p, cell_values, ncell * 8, hipMemcpyHostToDevice));
  const double eps0 = 1.0 / (kMu0 * kC0 * kC0);
  k_direction_e<<<grid_for(nE), kBlock>>>(w.as<double>(), dc.as<double>(), op->emask.as<uint8_t>(),
                                          op->axes<double>(), geo_of(op), op->nx, op->ny,
                                          which == 0 ? eps0 : 1.0);
  YR_TRY_HIP(hipGetLastError());
  YR_CALL(gemm_tn_weighted(rom->V1.as<double>(), nE, rom->q1, rom->V1.as<double>(), nE, rom->q1,
                           w.as<double>(), nE, C.as<double>(), rom->q1, nullptr));
  YR_TRY_HIP(hipDeviceSynchronize());
  std::vector<double> h;
  YR_CALL(download_sym(C.as<double>(), rom->q1, h, true));
  std::memcpy(out, h.data(), h.size() * 8);
  return YR_OK;
}

int yr_schur_apply(yr_operator* op, double dt, double z_re, double z_im, yr_dtype dtype,
                   const void* x, void* y, int32_t ncol) {
  YR_REQUIRE(op && x && y && ncol > 0 && dt > 0, YR_EINVAL, "bad argument");
  if (dtype == YR_F64) {
    SchurOp<double> S;
    YR_CALL(S.prepare(op, dt, zd(z_re, z_im), nullptr));
    YR_CALL(schur_apply<double>(S, (const cplx<double>*)x, (cplx<double>*)y, ncol, nullptr));
  } else {
    SchurOp<float> S;
    YR_CALL(S.prepare(op, dt, zd(z_re, z_im), nullptr));
    YR_CALL(schur_apply<float>(S, (const cplx<float>*)x, (cplx<float>*)y, ncol, nullptr));
  }
  YR_TRY_HIP(hipDeviceSynchronize());
  return YR_OK;
}

}  // extern "C"
