// Full-order Yee leapfrog, eq. (MNAform) in field form (Sec. II-A):
//   E^{n+1} = ca E^n + cb (curl H^{n+1/2} + B u^{n+1})
//   H^{n+3/2} = da H^{n+1/2} - db curl E^{n+1}
// with ca, cb (da, db) the per-sample coefficients of the diagonal blocks of
// R + F and R - F.  One thread per padded sample; each thread updates all
// components it owns.  The source entries are added by the thread that owns
// the sample (block-matched list, no atomics); probes are gathered by block 0
// of the magnetic kernel, which runs after the electric kernel completed.
#include <cmath>
#include <cstring>
#include <vector>

#include "common.hpp"
#include "fdtd_kernels.hpp"
#include "profile.hpp"

namespace yr {

// ------------------------------------------------------------------ host

// Packs a port list into `buf` as [slot int64][w T][block int32][port int32]
// arrays and fills the kernel-side descriptor.
template <typename T>
int stage_list(DevBuf& buf, const std::vector<PortEntry>& v, int nports, const int64_t*& slot,
               const T*& w, const int32_t*& block, const int32_t*& port, hipStream_t stream) {
  auto bytes_of = [](size_t n) { return n * (8 + sizeof(T) + 4 + 4); };
  const size_t n = v.size();
  YR_CALL(buf.reserve(bytes_of(n) + 16));
  std::vector<char> h(bytes_of(n) + 16, 0);
  char* base = h.data();
  int64_t* hs = reinterpret_cast<int64_t*>(base);
  T* hw = reinterpret_cast<T*>(base + 8 * n);
  int32_t* hb = reinterpret_cast<int32_t*>(base + (8 + sizeof(T)) * n);
  int32_t* hp = reinterpret_cast<int32_t*>(base + (8 + sizeof(T) + 4) * n);
  for (size_t q = 0; q < n; ++q) {
    hs[q] = v[q].slot;
    hw[q] = (T)v[q].w;
    hb[q] = v[q].block;
    hp[q] = v[q].port;
  }
  char* d = buf.as<char>();
  slot = reinterpret_cast<const int64_t*>(d);
  w = reinterpret_cast<const T*>(d + 8 * n);
  block = reinterpret_cast<const int32_t*>(d + (8 + sizeof(T)) * n);
  port = reinterpret_cast<const int32_t*>(d + (8 + sizeof(T) + 4) * n);
  if (n) {
    YR_TRY_HIP(hipMemcpyAsync(d, base, bytes_of(n), hipMemcpyHostToDevice, stream));
    // pageable source: the copy must have consumed it before h goes away
    YR_TRY_HIP(hipStreamSynchronize(stream));
  }
  (void)nports;
  return YR_OK;
}

template <typename T>
int stage_src(DevBuf& buf, const std::vector<PortEntry>& v, int nports, SrcList<T>& sl,
              hipStream_t s) {
  YR_CALL(stage_list<T>(buf, v, nports, sl.slot, sl.w, sl.block, sl.port, s));
  sl.n = (int)v.size();
  sl.nports = nports;
  return YR_OK;
}

template <typename T>
int stage_prb(DevBuf& buf, const std::vector<PortEntry>& v, int nports, PrbList<T>& pl,
              hipStream_t s) {
  const int32_t* unused = nullptr;
  YR_CALL(stage_list<T>(buf, v, nports, pl.slot, pl.w, unused, pl.port, s));
  pl.n = (int)v.size();
  pl.nports = nports;
  return YR_OK;
}

// half-step grids: a multiple of 8 workgroups (for the XCD-contiguous order)
static unsigned grid8(const yr_operator* op) { return (grid_for(op->len) + 7u) / 8u * 8u; }

// XCD-contiguous block order where two planes of a half-step's streams (six
// fields and six coefficients) fit in one XCD's 4 MB L2; in 2-D the previous
// row is the only earlier neighbour
template <typename T>
static int xcd_order(const yr_operator* op) {
  if (op->dim == 2) return 1;
  return 2 * (int64_t)op->X * op->Y * 12 * (int64_t)sizeof(T) <= ((int64_t)4 << 20) ? 1 : 0;
}

// 32-bit position arithmetic where every thread index of the grid fits
static bool small_box(const yr_operator* op) {
  return (int64_t)grid8(op) * kBlock <= (int64_t)UINT32_MAX;
}

template <typename T, typename I>
static void launch_e_t(const yr_operator* op, T* f, const SrcList<T>& sl, const T* u_n,
                       hipStream_t s) {
  unsigned grid = grid8(op);
  Axes<T> ax = op->axes<T>();
  if (op->dim == 3)
    k_e3<T, I><<<grid, kBlock, 0, s>>>(f, op->ca.as<T>(), op->cb.as<T>(), ax, op->X, op->Y,
                                       op->Z, op->len, sl, u_n, xcd_order<T>(op));
  else
    k_e2<T, I><<<grid, kBlock, 0, s>>>(f, op->ca.as<T>(), op->cb.as<T>(), ax, op->X, op->Y,
                                       op->len, sl, u_n, xcd_order<T>(op));
}

template <typename T>
void launch_e(const yr_operator* op, T* f, const SrcList<T>& sl, const T* u_n, hipStream_t s) {
  ProfScope ps("fdtd_e", s);
  if (small_box(op)) launch_e_t<T, uint32_t>(op, f, sl, u_n, s);
  else launch_e_t<T, int64_t>(op, f, sl, u_n, s);
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
  YR_CALL(stage_src<T>(op->src_dev, op->src_host, nsrc, sl, stream));
  YR_CALL(stage_prb<T>(op->prb_dev, op->prb_host, nprb, pl, stream));
  for (int64_t n = 0; n < nsteps; ++n) {
    launch_e<T>(op, f, sl, sl.n ? u + n * nsrc : nullptr, stream);
    launch_h<T>(op, f, pl, pl.n ? y + n * nprb : nullptr, stream);
  }
  YR_TRY_HIP(hipGetLastError());
  return YR_OK;
}

template int stage_src<float>(DevBuf&, const std::vector<PortEntry>&, int, SrcList<float>&, hipStream_t);
template int stage_src<double>(DevBuf&, const std::vector<PortEntry>&, int, SrcList<double>&, hipStream_t);
template int stage_prb<float>(DevBuf&, const std::vector<PortEntry>&, int, PrbList<float>&, hipStream_t);
template int stage_prb<double>(DevBuf&, const std::vector<PortEntry>&, int, PrbList<double>&, hipStream_t);
template void launch_e<float>(const yr_operator*, float*, const SrcList<float>&, const float*, hipStream_t);
template void launch_e<double>(const yr_operator*, double*, const SrcList<double>&, const double*, hipStream_t);
template void launch_h<float>(const yr_operator*, float*, const PrbList<float>&, float*, hipStream_t);
template void launch_h<double>(const yr_operator*, double*, const PrbList<double>&, double*, hipStream_t);

}  // namespace yr

using namespace yr;

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
  YR_CALL(resolve_ports(op, src, op->src_host, kBlock));
  YR_CALL(resolve_ports(op, probes, op->prb_host, kBlock));
  YR_REQUIRE(op->prb_host.size() <= 4096, YR_EINVAL, "at most 4096 probe entries");
  if (nsteps == 0) return YR_OK;
  hipStream_t stream = static_cast<hipStream_t>(stream_);
  YR_CALL(ensure_coefficients(op, dt, dtype, stream));
  if (dtype == YR_F64)
    return run_fdtd<double>(op, nsteps, static_cast<double*>(fields),
                            static_cast<const double*>(u), static_cast<double*>(y), nsrc, nprb,
                            stream);
  return run_fdtd<float>(op, nsteps, static_cast<float*>(fields), static_cast<const float*>(u),
                         static_cast<float*>(y), nsrc, nprb, stream);
}
