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
#include "profile.hpp"

namespace yr {

template <typename T>
struct SrcList {
  const int64_t* slot;  // field-buffer offsets
  const int32_t* block;
  const int32_t* port;
  const T* w;
  int n;
  int nports;
};

template <typename T>
struct PrbList {
  const int64_t* slot;
  const int32_t* port;
  const T* w;
  int n;
  int nports;
};

template <typename T>
__device__ inline void add_sources(T* __restrict__ f, const T* __restrict__ cb, int64_t len,
                                   int nslots, int64_t t, const SrcList<T>& src,
                                   const T* __restrict__ u_n) {
  for (int s = 0; s < src.n; ++s) {
    if (src.block[s] != (int)blockIdx.x) continue;  // uniform across the block
    int64_t slot = src.slot[s];
    int64_t c = slot / len;
    if (slot - c * len == t) f[slot] += cb[slot] * src.w[s] * u_n[src.port[s]];
  }
}

template <typename T>
__device__ inline void gather_probes(const T* __restrict__ f, const PrbList<T>& prb,
                                     T* __restrict__ y_n) {
  if (blockIdx.x != 0) return;
  for (int p = threadIdx.x; p < prb.nports; p += blockDim.x) {
    T acc = 0;
    for (int q = 0; q < prb.n; ++q)
      if (prb.port[q] == p) acc += prb.w[q] * f[prb.slot[q]];
    y_n[p] = acc;
  }
}

// ------------------------------------------------------------------ 3-D

template <typename T>
__global__ void __launch_bounds__(kBlock) k_e3(T* __restrict__ f, const T* __restrict__ ca,
                                               const T* __restrict__ cb, Axes<T> ax, int X, int Y,
                                               int Z, int64_t len, SrcList<T> src,
                                               const T* __restrict__ u_n) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < len) {
    int i = (int)(t % X);
    int64_t r = t / X;
    int j = (int)(r % Y);
    int k = (int)(r / Y);
    const int64_t sY = X, sZ = (int64_t)X * Y;
    T* Ex = f;
    T* Ey = f + len;
    T* Ez = f + 2 * len;
    const T* Hx = f + 3 * len;
    const T* Hy = f + 4 * len;
    const T* Hz = f + 5 * len;
    if (j >= 1 && k >= 1) {  // eps dEx/dt = dHz/dy - dHy/dz
      T c = (Hz[t] - Hz[t - sY]) * ax.id[1][j] - (Hy[t] - Hy[t - sZ]) * ax.id[2][k];
      Ex[t] = ca[t] * Ex[t] + cb[t] * c;
    }
    if (i >= 1 && k >= 1) {  // eps dEy/dt = dHx/dz - dHz/dx
      T c = (Hx[t] - Hx[t - sZ]) * ax.id[2][k] - (Hz[t] - Hz[t - 1]) * ax.id[0][i];
      Ey[t] = ca[len + t] * Ey[t] + cb[len + t] * c;
    }
    if (i >= 1 && j >= 1) {  // eps dEz/dt = dHy/dx - dHx/dy
      T c = (Hy[t] - Hy[t - 1]) * ax.id[0][i] - (Hx[t] - Hx[t - sY]) * ax.id[1][j];
      Ez[t] = ca[2 * len + t] * Ez[t] + cb[2 * len + t] * c;
    }
  }
  if (src.n) {
    if (t < len) add_sources(f, cb, len, 3, t, src, u_n);
  }
}

template <typename T, bool UNIFORM_H>
__global__ void __launch_bounds__(kBlock) k_h3(T* __restrict__ f, const T* __restrict__ da,
                                               const T* __restrict__ db, T db0, Axes<T> ax, int X,
                                               int Y, int Z, int64_t len, PrbList<T> prb,
                                               T* __restrict__ y_n) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < len) {
    int i = (int)(t % X);
    int64_t r = t / X;
    int j = (int)(r % Y);
    int k = (int)(r / Y);
    const int64_t sY = X, sZ = (int64_t)X * Y;
    const T* Ex = f;
    const T* Ey = f + len;
    const T* Ez = f + 2 * len;
    T* Hx = f + 3 * len;
    T* Hy = f + 4 * len;
    T* Hz = f + 5 * len;
    if (j < Y - 1 && k < Z - 1) {  // mu dHx/dt = dEy/dz - dEz/dy
      T c = (Ey[t + sZ] - Ey[t]) * ax.ip[2][k] - (Ez[t + sY] - Ez[t]) * ax.ip[1][j];
      if (UNIFORM_H) Hx[t] += db0 * c;
      else Hx[t] = da[t] * Hx[t] + db[t] * c;
    }
    if (i < X - 1 && k < Z - 1) {  // mu dHy/dt = dEz/dx - dEx/dz
      T c = (Ez[t + 1] - Ez[t]) * ax.ip[0][i] - (Ex[t + sZ] - Ex[t]) * ax.ip[2][k];
      if (UNIFORM_H) Hy[t] += db0 * c;
      else Hy[t] = da[len + t] * Hy[t] + db[len + t] * c;
    }
    if (i < X - 1 && j < Y - 1) {  // mu dHz/dt = dEx/dy - dEy/dx
      T c = (Ex[t + sY] - Ex[t]) * ax.ip[1][j] - (Ey[t + 1] - Ey[t]) * ax.ip[0][i];
      if (UNIFORM_H) Hz[t] += db0 * c;
      else Hz[t] = da[2 * len + t] * Hz[t] + db[2 * len + t] * c;
    }
  }
  if (prb.n) gather_probes(f, prb, y_n);
}

// ------------------------------------------------------------------ 2-D (Ez-pol)

template <typename T>
__global__ void __launch_bounds__(kBlock) k_e2(T* __restrict__ f, const T* __restrict__ ca,
                                               const T* __restrict__ cb, Axes<T> ax, int X, int Y,
                                               int64_t len, SrcList<T> src,
                                               const T* __restrict__ u_n) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < len) {
    int i = (int)(t % X);
    int j = (int)(t / X);
    T* Ez = f;
    const T* Hx = f + len;
    const T* Hy = f + 2 * len;
    if (i >= 1 && j >= 1) {  // eps dEz/dt = dHy/dx - dHx/dy
      T c = (Hy[t] - Hy[t - 1]) * ax.id[0][i] - (Hx[t] - Hx[t - X]) * ax.id[1][j];
      Ez[t] = ca[t] * Ez[t] + cb[t] * c;
    }
    if (src.n) add_sources(f, cb, len, 1, t, src, u_n);
  }
}

template <typename T, bool UNIFORM_H>
__global__ void __launch_bounds__(kBlock) k_h2(T* __restrict__ f, const T* __restrict__ da,
                                               const T* __restrict__ db, T db0, Axes<T> ax, int X,
                                               int Y, int64_t len, PrbList<T> prb,
                                               T* __restrict__ y_n) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < len) {
    int i = (int)(t % X);
    int j = (int)(t / X);
    const T* Ez = f;
    T* Hx = f + len;
    T* Hy = f + 2 * len;
    if (j < Y - 1) {  // mu dHx/dt = -dEz/dy
      T c = -(Ez[t + X] - Ez[t]) * ax.ip[1][j];
      if (UNIFORM_H) Hx[t] += db0 * c;
      else Hx[t] = da[t] * Hx[t] + db[t] * c;
    }
    if (i < X - 1) {  // mu dHy/dt = dEz/dx
      T c = (Ez[t + 1] - Ez[t]) * ax.ip[0][i];
      if (UNIFORM_H) Hy[t] += db0 * c;
      else Hy[t] = da[len + t] * Hy[t] + db[len + t] * c;
    }
  }
  if (prb.n) gather_probes(f, prb, y_n);
}

// ------------------------------------------------------------------ host

template <typename T>
static int stage_ports(yr_operator* op, const std::vector<PortEntry>& src,
                       const std::vector<PortEntry>& prb, int nsrc_ports, int nprb_ports,
                       SrcList<T>& sl, PrbList<T>& pl, hipStream_t stream) {
  // one device buffer: [slots int64][w T][block int32][port int32] per list
  auto bytes_of = [](size_t n) { return n * (8 + sizeof(T) + 4 + 4); };
  YR_CALL(op->src_dev.reserve(bytes_of(src.size()) + 16));
  YR_CALL(op->prb_dev.reserve(bytes_of(prb.size()) + 16));
  auto pack = [&](const std::vector<PortEntry>& v, DevBuf& buf, const int64_t*& slot,
                  const T*& w, const int32_t*& block, const int32_t*& port) -> int {
    size_t n = v.size();
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
    if (n) YR_TRY_HIP(hipMemcpyAsync(d, base, bytes_of(n), hipMemcpyHostToDevice, stream));
    // pageable source: make sure the copy has consumed it before h goes away
    if (n) YR_TRY_HIP(hipStreamSynchronize(stream));
    return YR_OK;
  };
  const int32_t* unused_block = nullptr;
  YR_CALL(pack(src, op->src_dev, sl.slot, sl.w, sl.block, sl.port));
  YR_CALL(pack(prb, op->prb_dev, pl.slot, pl.w, unused_block, pl.port));
  sl.n = (int)src.size();
  sl.nports = nsrc_ports;
  pl.n = (int)prb.size();
  pl.nports = nprb_ports;
  return YR_OK;
}

template <typename T>
static int run_fdtd(yr_operator* op, double dt, int64_t nsteps, T* f, const T* u, T* y,
                    int nsrc, int nprb, hipStream_t stream) {
  SrcList<T> sl{};
  PrbList<T> pl{};
  YR_CALL(stage_ports<T>(op, op->src_host, op->prb_host, nsrc, nprb, sl, pl, stream));
  Axes<T> ax = op->axes<T>();
  const T* ca = op->ca.as<T>();
  const T* cb = op->cb.as<T>();
  const T* da = op->da.as<T>();
  const T* db = op->db.as<T>();
  T db0 = (T)op->db_uniform;
  unsigned grid = grid_for(op->len);
  for (int64_t n = 0; n < nsteps; ++n) {
    const T* u_n = sl.n ? u + n * nsrc : nullptr;
    T* y_n = pl.n ? y + n * nprb : nullptr;
    if (op->dim == 3) {
      {
        ProfScope ps("fdtd_e", stream);
        k_e3<T><<<grid, kBlock, 0, stream>>>(f, ca, cb, ax, op->X, op->Y, op->Z, op->len, sl, u_n);
      }
      ProfScope ps("fdtd_h", stream);
      if (op->uniform_h)
        k_h3<T, true><<<grid, kBlock, 0, stream>>>(f, da, db, db0, ax, op->X, op->Y, op->Z,
                                                    op->len, pl, y_n);
      else
        k_h3<T, false><<<grid, kBlock, 0, stream>>>(f, da, db, db0, ax, op->X, op->Y, op->Z,
                                                     op->len, pl, y_n);
    } else {
      {
        ProfScope ps("fdtd_e", stream);
        k_e2<T><<<grid, kBlock, 0, stream>>>(f, ca, cb, ax, op->X, op->Y, op->len, sl, u_n);
      }
      ProfScope ps("fdtd_h", stream);
      if (op->uniform_h)
        k_h2<T, true><<<grid, kBlock, 0, stream>>>(f, da, db, db0, ax, op->X, op->Y, op->len, pl,
                                                    y_n);
      else
        k_h2<T, false><<<grid, kBlock, 0, stream>>>(f, da, db, db0, ax, op->X, op->Y, op->len,
                                                     pl, y_n);
    }
  }
  YR_TRY_HIP(hipGetLastError());
  return YR_OK;
}

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
    return run_fdtd<double>(op, dt, nsteps, static_cast<double*>(fields),
                            static_cast<const double*>(u), static_cast<double*>(y), nsrc, nprb,
                            stream);
  return run_fdtd<float>(op, dt, nsteps, static_cast<float*>(fields),
                         static_cast<const float*>(u), static_cast<float*>(y), nsrc, nprb, stream);
}
