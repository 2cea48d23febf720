// Full-order Yee leapfrog, eq. (MNAform) in field form (Sec. II-A):
//   E^{n+1} = ca E^n + cb (curl H^{n+1/2} + B u^{n+1})
//   H^{n+3/2} = da H^{n+1/2} - db curl E^{n+1}
// with ca, cb (da, db) the per-sample coefficients of the diagonal blocks of
// R + F and R - F.  One thread per padded sample; each thread updates all
// components it owns.  The source entries are added by the thread that owns
// the sample (entries grouped by block, no atomics); probes are gathered by
// block 0 of the magnetic kernel, one wavefront per port, after the electric
// kernel completed.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "fdtd_kernels.hpp"
#include "profile.hpp"

namespace yr {

// ------------------------------------------------------------------ host

// Copies a host staging image into buf on stream s.  The image is pageable
// host memory: the copy must have consumed it before it goes away.
static int upload_image(DevBuf& buf, const std::vector<char>& h, hipStream_t stream) {
  YR_CALL(buf.reserve(h.size() + 16));
  if (!h.empty()) {
    YR_TRY_HIP(hipMemcpyAsync(buf.p, h.data(), h.size(), hipMemcpyHostToDevice, stream));
    YR_TRY_HIP(hipStreamSynchronize(stream));
  }
  return YR_OK;
}

template <typename T>
int stage_src(DevBuf& buf, const std::vector<PortEntry>& v, int nports, int nblocks,
              SrcList<T>& sl, hipStream_t stream) {
  // entries in order of their owning block (stable: a block keeps the given
  // order of its entries), [slot int64][w T][port int32][bptr int32]
  std::vector<size_t> ord(v.size());
  for (size_t q = 0; q < ord.size(); ++q) ord[q] = q;
  std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return v[a].block < v[b].block; });
  const size_t n = v.size(), nb = n ? (size_t)nblocks : 0;
  const size_t o_w = 8 * n, o_p = o_w + sizeof(T) * n, o_b = o_p + 4 * n;
  std::vector<char> h(o_b + 4 * (nb + 1), 0);
  int64_t* hs = reinterpret_cast<int64_t*>(h.data());
  T* hw = reinterpret_cast<T*>(h.data() + o_w);
  int32_t* hp = reinterpret_cast<int32_t*>(h.data() + o_p);
  int32_t* hb = reinterpret_cast<int32_t*>(h.data() + o_b);
  for (size_t q = 0; q < n; ++q) {
    const PortEntry& e = v[ord[q]];
    YR_REQUIRE(e.block >= 0 && e.block < nblocks, YR_EINVAL, "source entry outside the grid");
    hs[q] = e.slot;
    hw[q] = (T)e.w;
    hp[q] = e.port;
    hb[e.block + 1] += 1;
  }
  for (size_t b = 0; b < nb; ++b) hb[b + 1] += hb[b];
  YR_CALL(upload_image(buf, h, stream));
  char* d = buf.as<char>();
  sl.slot = reinterpret_cast<const int64_t*>(d);
  sl.w = reinterpret_cast<const T*>(d + o_w);
  sl.port = reinterpret_cast<const int32_t*>(d + o_p);
  sl.bptr = reinterpret_cast<const int32_t*>(d + o_b);
  sl.n = (int)n;
  sl.nports = nports;
  sl.nblocks = (int)nb;
  return YR_OK;
}

template <typename T>
int stage_prb(DevBuf& buf, const std::vector<PortEntry>& v, int nports, PrbList<T>& pl,
              hipStream_t stream) {
  // entries in order of their port, [slot int64][w T][pptr int32]
  std::vector<size_t> ord(v.size());
  for (size_t q = 0; q < ord.size(); ++q) ord[q] = q;
  std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return v[a].port < v[b].port; });
  const size_t n = v.size(), np = n ? (size_t)nports : 0;
  const size_t o_w = 8 * n, o_p = o_w + sizeof(T) * n;
  std::vector<char> h(o_p + 4 * (np + 1), 0);
  int64_t* hs = reinterpret_cast<int64_t*>(h.data());
  T* hw = reinterpret_cast<T*>(h.data() + o_w);
  int32_t* hp = reinterpret_cast<int32_t*>(h.data() + o_p);
  for (size_t q = 0; q < n; ++q) {
    const PortEntry& e = v[ord[q]];
    YR_REQUIRE(e.port >= 0 && e.port < nports, YR_EINVAL, "probe entry of an unknown port");
    hs[q] = e.slot;
    hw[q] = (T)e.w;
    hp[e.port + 1] += 1;
  }
  for (size_t p = 0; p < np; ++p) hp[p + 1] += hp[p];
  YR_CALL(upload_image(buf, h, stream));
  char* d = buf.as<char>();
  pl.slot = reinterpret_cast<const int64_t*>(d);
  pl.w = reinterpret_cast<const T*>(d + o_w);
  pl.pptr = reinterpret_cast<const int32_t*>(d + o_p);
  pl.n = (int)n;
  pl.nports = nports;
  return YR_OK;
}

// half-step grids: a multiple of 8 workgroups (for the XCD-contiguous order)
static unsigned grid8(const yr_operator* op) { return (grid_for(op->len) + 7u) / 8u * 8u; }

unsigned e_blocks(const yr_operator* op) { return grid8(op); }

// XCD-contiguous block order where two planes of a half-step's streams (six
// fields and six per-sample coefficients) fit in one XCD's 4 MB L2 (measured
// slower above that size even with the coefficients by material number); in
// 2-D the previous row is the only earlier neighbour
template <typename T>
static int xcd_order(const yr_operator* op) {
  if (op->dim == 2) return 1;
  return 2 * (int64_t)op->X * op->Y * 12 * (int64_t)sizeof(T) <= ((int64_t)4 << 20) ? 1 : 0;
}

// 32-bit position arithmetic where every thread index of the grid fits
static bool small_box(const yr_operator* op) {
  return (int64_t)grid8(op) * kBlock <= (int64_t)UINT32_MAX;
}

template <typename T, typename I, int IDX>
static void launch_e_t(const yr_operator* op, T* f, const SrcList<T>& sl, const T* u_n,
                       hipStream_t s) {
  unsigned grid = grid8(op);
  Axes<T> ax = op->axes<T>();
  ECoef<T> ec{op->ca.as<T>(), op->cb.as<T>(), op->e_idx.p, op->e_tab.as<T>()};
  if (op->dim == 3)
    k_e3<T, I, IDX><<<grid, kBlock, 0, s>>>(f, ec, ax, op->X, op->Y, op->Z, op->len, sl, u_n,
                                            xcd_order<T>(op));
  else
    k_e2<T, I, IDX><<<grid, kBlock, 0, s>>>(f, ec, ax, op->X, op->Y, op->len, sl, u_n,
                                            xcd_order<T>(op));
}

template <typename T>
void launch_e(const yr_operator* op, T* f, const SrcList<T>& sl, const T* u_n, hipStream_t s) {
  ProfScope ps("fdtd_e", s);
  const bool sm = small_box(op);
  if (op->e_idx_bytes == 2) {
    if (sm) launch_e_t<T, uint32_t, 2>(op, f, sl, u_n, s);
    else launch_e_t<T, int64_t, 2>(op, f, sl, u_n, s);
  } else if (op->e_idx_bytes == 4) {
    if (sm) launch_e_t<T, uint32_t, 4>(op, f, sl, u_n, s);
    else launch_e_t<T, int64_t, 4>(op, f, sl, u_n, s);
  } else {
    if (sm) launch_e_t<T, uint32_t, 0>(op, f, sl, u_n, s);
    else launch_e_t<T, int64_t, 0>(op, f, sl, u_n, s);
  }
}

template <typename T, typename I>
static void launch_h_t(const yr_operator* op, T* f, const PrbList<T>& pl, T* y_n, hipStream_t s) {
  unsigned grid = grid8(op);
  Axes<T> ax = op->axes<T>();
  const T* da = op->da.as<T>();
  const T* db = op->db.as<T>();
  T db0 = (T)op->db_uniform;
  if (op->dim == 3) {
    if (op->uniform_h)
      k_h3<T, true, I><<<grid, kBlock, 0, s>>>(f, da, db, db0, ax, op->X, op->Y, op->Z, op->len,
                                               pl, y_n, xcd_order<T>(op));
    else
      k_h3<T, false, I><<<grid, kBlock, 0, s>>>(f, da, db, db0, ax, op->X, op->Y, op->Z,
                                                op->len, pl, y_n, xcd_order<T>(op));
  } else {
    if (op->uniform_h)
      k_h2<T, true, I><<<grid, kBlock, 0, s>>>(f, da, db, db0, ax, op->X, op->Y, op->len, pl,
                                               y_n, xcd_order<T>(op));
    else
      k_h2<T, false, I><<<grid, kBlock, 0, s>>>(f, da, db, db0, ax, op->X, op->Y, op->len, pl,
                                                y_n, xcd_order<T>(op));
  }
}

template <typename T>
void launch_h(const yr_operator* op, T* f, const PrbList<T>& pl, T* y_n, hipStream_t s) {
  ProfScope ps("fdtd_h", s);
  if (small_box(op)) launch_h_t<T, uint32_t>(op, f, pl, y_n, s);
  else launch_h_t<T, int64_t>(op, f, pl, y_n, s);
}

template <typename T>
static int run_fdtd(yr_operator* op, int64_t nsteps, T* f, const T* u, T* y, int nsrc, int nprb,
                    hipStream_t stream) {
  SrcList<T> sl{};
  PrbList<T> pl{};
  YR_CALL(stage_src<T>(op->src_dev, op->src_host, nsrc, (int)e_blocks(op), sl, stream));
  YR_CALL(stage_prb<T>(op->prb_dev, op->prb_host, nprb, pl, stream));
  for (int64_t n = 0; n < nsteps; ++n) {
    launch_e<T>(op, f, sl, sl.n ? u + n * nsrc : nullptr, stream);
    launch_h<T>(op, f, pl, pl.n ? y + n * nprb : nullptr, stream);
  }
  YR_TRY_HIP(hipGetLastError());
  return YR_OK;
}

template int stage_src<float>(DevBuf&, const std::vector<PortEntry>&, int, int, SrcList<float>&, hipStream_t);
template int stage_src<double>(DevBuf&, const std::vector<PortEntry>&, int, int, SrcList<double>&, hipStream_t);
template int stage_prb<float>(DevBuf&, const std::vector<PortEntry>&, int, PrbList<float>&, hipStream_t);
template int stage_prb<double>(DevBuf&, const std::vector<PortEntry>&, int, PrbList<double>&, hipStream_t);
template void launch_e<float>(const yr_operator*, float*, const SrcList<float>&, const float*, hipStream_t);
template void launch_e<double>(const yr_operator*, double*, const SrcList<double>&, const double*, hipStream_t);
template void launch_h<float>(const yr_operator*, float*, const PrbList<float>&, float*, hipStream_t);
template void launch_h<double>(const yr_operator*, double*, const PrbList<double>&, double*, hipStream_t);

template <typename T>
int run_fdtd_fused(yr_operator* op, int64_t nsteps, T* f, const T* u, T* y, int nsrc, int nprb,
                   hipStream_t stream);

// The one-pass step moves fewer bytes but pays a halo (a 64 x 16 tile reads
// 66 x 18 magnetic and 65 x 17 electric samples per plane, and one extra
// plane per z chunk) and two barriers per plane.  Measured per step (FP32):
// 128^3 26.7 vs 30.4 us for the two half-step kernels, 256^3 314 vs 318 us;
// FP64 256^3 613 vs 652 us.  The automatic choice takes it for 3-D boxes
// that fill at least a 64 x 16 tile and 16 planes.
static bool use_fused(const yr_operator* op, size_t es) {
  (void)es;
  if (op->dim != 3 || op->leapfrog_mode == 1) return false;
  if (op->leapfrog_mode == 2) return true;
  return op->nx >= 64 && op->ny >= 16 && op->nz >= 16;
}

}  // namespace yr

using namespace yr;

extern "C" int yr_operator_set_leapfrog(yr_operator* op, int32_t mode) {
  YR_REQUIRE(op, YR_EINVAL, "null operator");
  YR_REQUIRE(mode >= 0 && mode <= 2, YR_EINVAL, "mode must be 0 (automatic), 1 or 2");
  YR_CALL(op_wait_idle(op));
  op->leapfrog_mode = mode;
  return YR_OK;
}

extern "C" int fdtd_step(yr_operator* op, yr_dtype dtype, double dt, int64_t nsteps,
                         void* fields, const yr_ports* src, const void* u,
                         const yr_ports* probes, void* y, void* stream_) {
  YR_REQUIRE(op, YR_EINVAL, "null operator");
  YR_REQUIRE(dtype == YR_F32 || dtype == YR_F64, YR_EINVAL, "dtype must be YR_F32 or YR_F64");
  YR_REQUIRE(nsteps >= 0, YR_EINVAL, "nsteps must be >= 0");
  YR_REQUIRE(dt > 0 && std::isfinite(dt), YR_EINVAL, "dt must be positive");
  YR_REQUIRE(dt <= op->dt_max * (1 + 1e-12), YR_EUNSTABLE,
             "dt exceeds the CFL limit: the leapfrog would be unstable");
  YR_REQUIRE(fields || nsteps == 0, YR_EINVAL, "null field buffer");
  int nsrc = src ? src->n : 0, nprb = probes ? probes->n : 0;
  YR_REQUIRE(nsrc == 0 || u, YR_EINVAL, "sources given without a waveform buffer");
  YR_REQUIRE(nprb == 0 || y, YR_EINVAL, "probes given without an output buffer");
  if (nsteps == 0) {
    std::vector<PortEntry> tmp;  // validate the ports only
    YR_CALL(resolve_ports(op, src, tmp, kBlock));
    return resolve_ports(op, probes, tmp, kBlock);
  }
  YR_CALL(op_wait_idle(op));
  YR_CALL(resolve_ports(op, src, op->src_host, kBlock));
  YR_CALL(resolve_ports(op, probes, op->prb_host, kBlock));
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  YR_CALL(ensure_coefficients(op, dt, dtype, stream));
  int rc;
  if (dtype == YR_F64)
    rc = use_fused(op, 8) ? run_fdtd_fused<double>(op, nsteps, static_cast<double*>(fields),
                                                   static_cast<const double*>(u),
                                                   static_cast<double*>(y), nsrc, nprb, stream)
                          : run_fdtd<double>(op, nsteps, static_cast<double*>(fields),
                                             static_cast<const double*>(u),
                                             static_cast<double*>(y), nsrc, nprb, stream);
  else
    rc = use_fused(op, 4) ? run_fdtd_fused<float>(op, nsteps, static_cast<float*>(fields),
                                                  static_cast<const float*>(u),
                                                  static_cast<float*>(y), nsrc, nprb, stream)
                          : run_fdtd<float>(op, nsteps, static_cast<float*>(fields),
                                            static_cast<const float*>(u), static_cast<float*>(y),
                                            nsrc, nprb, stream);
  YR_CALL(rc);
  return op_mark_busy(op, stream);
}
