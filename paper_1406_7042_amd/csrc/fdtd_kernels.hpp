// Leapfrog stencil kernels of eq. (MNAform) in field form, shared by the
// forward sweep (fdtd_step) and the reverse-time adjoint sweep.
#pragma once

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

// host helpers (fdtd.hip)
template <typename T>
int stage_src(DevBuf& buf, const std::vector<PortEntry>& v, int nports, SrcList<T>& sl,
              hipStream_t s);
template <typename T>
int stage_prb(DevBuf& buf, const std::vector<PortEntry>& v, int nports, PrbList<T>& pl,
              hipStream_t s);
// one electric (resp. magnetic) half step of the leapfrog on field buffer f
template <typename T>
void launch_e(const yr_operator* op, T* f, const SrcList<T>& sl, const T* u_n, hipStream_t s);
template <typename T>
void launch_h(const yr_operator* op, T* f, const PrbList<T>& pl, T* y_n, hipStream_t s);

}  // namespace yr
