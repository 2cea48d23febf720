// Leapfrog stencil kernels of eq. (MNAform) in field form, shared by the
// forward sweep (fdtd_step) and the reverse-time adjoint sweep.
#pragma once

#include <vector>

#include "common.hpp"
#include "profile.hpp"

namespace yr {

// Source entries sorted by the (logical) block of the electric kernel that
// owns their slot: block b's entries are bptr[b] .. bptr[b+1]-1, so a thread
// checks only the few entries of its own block (plane sources have thousands).
template <typename T>
struct SrcList {
  const int64_t* slot;  // field-buffer offsets
  const int32_t* port;
  const int32_t* bptr;  // [nblocks + 1]
  const T* w;
  int n;
  int nports;
  int nblocks;
};

// Probe entries sorted by port: port p's entries are pptr[p] .. pptr[p+1]-1.
template <typename T>
struct PrbList {
  const int64_t* slot;
  const int32_t* pptr;  // [nports + 1]
  const T* w;
  int n;
  int nports;
};

// Electric leapfrog coefficients ca, cb of a sample: two per-sample streams
// (IDX = 0), or a material number per sample, 16-bit (IDX = 2) or 32-bit
// (IDX = 4), and a table of (ca, cb) pairs that stays in cache.
template <typename T>
struct ECoef {
  const T* ca;
  const T* cb;
  const void* idx;
  const T* tab;
};

template <int IDX>
__device__ inline uint32_t e_material(const void* idx, int64_t g) {
  if (IDX == 2) return static_cast<const uint16_t*>(idx)[g];
  return static_cast<const uint32_t*>(idx)[g];
}

template <typename T, int IDX>
__device__ inline void e_coef(const ECoef<T>& c, int64_t g, T& a, T& b) {
  if (IDX) {
    const uint32_t m = e_material<IDX>(c.idx, g);
    a = c.tab[2 * m];
    b = c.tab[2 * m + 1];
  } else {
    a = c.ca[g];
    b = c.cb[g];
  }
}

// Workgroups are dealt to the 8 XCDs round-robin by id.  With `xcd` set,
// logical block (id % 8) * (nb / 8) + id / 8 (nb a multiple of 8) gives each
// XCD one contiguous run of positions, so the previous row and plane that a
// thread reads were loaded by the same XCD, into its own L2 (the host sets it
// where two planes of the half-step's streams fit in one L2).
__device__ inline unsigned xcd_block(unsigned b, unsigned nb, int xcd) {
  return xcd ? (b & 7u) * (nb >> 3) + (b >> 3) : b;
}

template <typename T, int IDX>
__device__ inline void add_sources(T* __restrict__ f, const ECoef<T>& ec, int64_t len,
                                   int nslots, int64_t t, const SrcList<T>& src,
                                   const T* __restrict__ u_n, unsigned lblock) {
  if ((int)lblock >= src.nblocks) return;
  const int e1 = src.bptr[lblock + 1];
  for (int s = src.bptr[lblock]; s < e1; ++s) {  // uniform across the block
    int64_t slot = src.slot[s];
    int64_t c = slot / len;
    if (slot - c * len == t) {
      T a, b;
      e_coef<T, IDX>(ec, slot, a, b);
      f[slot] += b * src.w[s] * u_n[src.port[s]];
    }
  }
}

// Block 0 gathers the probes: one wavefront per port, its lanes stride the
// port's entries and a butterfly adds the lanes (line and plane probes have
// many entries).
template <typename T>
__device__ inline void gather_probes(const T* __restrict__ f, const PrbList<T>& prb,
                                     T* __restrict__ y_n) {
  if (blockIdx.x != 0) return;
  const int lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  for (int p = threadIdx.x >> 6; p < prb.nports; p += nw) {
    T acc = 0;
    for (int q = prb.pptr[p] + lane; q < prb.pptr[p + 1]; q += 64) acc += prb.w[q] * f[prb.slot[q]];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) y_n[p] = acc;
  }
}

// ------------------------------------------------------------------ 3-D
//
// One thread per padded position t (index type I: 32-bit where the box allows).
// Every value a thread needs is loaded before its first store: the six
// components share one buffer, so a store to one component would otherwise
// order the loads of the next one behind it (three memory round trips per
// thread instead of one).  Neighbour reads at positions whose component is
// not updated are still inside the buffer (E occupies [0, 3 len) and H
// [3 len, 6 len); no offset exceeds sZ <= len) and are simply not used.

template <typename I>
__device__ inline void decode3(I t, int X, int Y, int& i, int& j, int& k) {
  const I r = t / (I)X;
  i = (int)(t - r * (I)X);
  const I q = r / (I)Y;
  j = (int)(r - q * (I)Y);
  k = (int)q;
}

template <typename T, typename I, int IDX>
__global__ void __launch_bounds__(kBlock) k_e3(T* __restrict__ f, ECoef<T> ec, Axes<T> ax, int X,
                                               int Y, int Z, int64_t len, SrcList<T> src,
                                               const T* __restrict__ u_n, int xcd) {
  const unsigned lb = xcd_block(blockIdx.x, gridDim.x, xcd);
  const I t = (I)lb * (I)blockDim.x + (I)threadIdx.x;
  if (t < (I)len) {
    int i, j, k;
    decode3<I>(t, X, Y, i, j, k);
    const int sY = X, sZ = X * Y;
    T* e = f + t;  // Ex at e[0], Ey at e[len], Ez at e[2 len]
    const T* h = f + 3 * len + t;  // Hx, Hy, Hz likewise
    const T ex = e[0], ey = e[len], ez = e[2 * len];
    const T hx = h[0], hx_y = h[-sY], hx_z = h[-sZ];
    const T hy = h[len], hy_x = h[len - 1], hy_z = h[len - sZ];
    const T hz = h[2 * len], hz_x = h[2 * len - 1], hz_y = h[2 * len - sY];
    T a0, a1, a2, b0, b1, b2;
    e_coef<T, IDX>(ec, (int64_t)t, a0, b0);
    e_coef<T, IDX>(ec, (int64_t)len + t, a1, b1);
    e_coef<T, IDX>(ec, 2 * (int64_t)len + t, a2, b2);
    const T idx = ax.id[0][i], idy = ax.id[1][j], idz = ax.id[2][k];
    if (j >= 1 && k >= 1)  // eps dEx/dt = dHz/dy - dHy/dz
      e[0] = a0 * ex + b0 * ((hz - hz_y) * idy - (hy - hy_z) * idz);
    if (i >= 1 && k >= 1)  // eps dEy/dt = dHx/dz - dHz/dx
      e[len] = a1 * ey + b1 * ((hx - hx_z) * idz - (hz - hz_x) * idx);
    if (i >= 1 && j >= 1)  // eps dEz/dt = dHy/dx - dHx/dy
      e[2 * len] = a2 * ez + b2 * ((hy - hy_x) * idx - (hx - hx_y) * idy);
    if (src.n) add_sources<T, IDX>(f, ec, len, 3, (int64_t)t, src, u_n, lb);
  }
}

template <typename T, bool UNIFORM_H, typename I>
__global__ void __launch_bounds__(kBlock) k_h3(T* __restrict__ f, const T* __restrict__ da,
                                               const T* __restrict__ db, T db0, Axes<T> ax, int X,
                                               int Y, int Z, int64_t len, PrbList<T> prb,
                                               T* __restrict__ y_n, int xcd) {
  const unsigned lb = xcd_block(blockIdx.x, gridDim.x, xcd);
  const I t = (I)lb * (I)blockDim.x + (I)threadIdx.x;
  if (t < (I)len) {
    int i, j, k;
    decode3<I>(t, X, Y, i, j, k);
    const int sY = X, sZ = X * Y;
    const T* e = f + t;
    T* h = f + 3 * len + t;
    const T hx = h[0], hy = h[len], hz = h[2 * len];
    const T ex = e[0], ex_y = e[sY], ex_z = e[sZ];
    const T ey = e[len], ey_x = e[len + 1], ey_z = e[len + sZ];
    const T ez = e[2 * len], ez_x = e[2 * len + 1], ez_y = e[2 * len + sY];
    T a0 = 1, a1 = 1, a2 = 1, b0 = db0, b1 = db0, b2 = db0;
    if (!UNIFORM_H) {
      a0 = da[t], a1 = da[len + t], a2 = da[2 * len + t];
      b0 = db[t], b1 = db[len + t], b2 = db[2 * len + t];
    }
    const T ipx = ax.ip[0][i], ipy = ax.ip[1][j], ipz = ax.ip[2][k];
    if (j < Y - 1 && k < Z - 1)  // mu dHx/dt = dEy/dz - dEz/dy
      h[0] = a0 * hx + b0 * ((ey_z - ey) * ipz - (ez_y - ez) * ipy);
    if (i < X - 1 && k < Z - 1)  // mu dHy/dt = dEz/dx - dEx/dz
      h[len] = a1 * hy + b1 * ((ez_x - ez) * ipx - (ex_z - ex) * ipz);
    if (i < X - 1 && j < Y - 1)  // mu dHz/dt = dEx/dy - dEy/dx
      h[2 * len] = a2 * hz + b2 * ((ex_y - ex) * ipy - (ey_x - ey) * ipx);
  }
  if (prb.n) gather_probes(f, prb, y_n);
}

// ------------------------------------------------------------------ 2-D (Ez-pol)

template <typename T, typename I, int IDX>
__global__ void __launch_bounds__(kBlock) k_e2(T* __restrict__ f, ECoef<T> ec, Axes<T> ax, int X,
                                               int Y, int64_t len, SrcList<T> src,
                                               const T* __restrict__ u_n, int xcd) {
  const unsigned lb = xcd_block(blockIdx.x, gridDim.x, xcd);
  const I t = (I)lb * (I)blockDim.x + (I)threadIdx.x;
  if (t < (I)len) {
    const I r = t / (I)X;
    const int i = (int)(t - r * (I)X), j = (int)r;
    T* ezp = f + t;
    const T* h = f + len + t;  // Hx at h[0], Hy at h[len]
    const T ez = ezp[0];
    const T hx = h[0], hx_y = h[-X], hy = h[len], hy_x = h[len - 1];
    T a, b;
    e_coef<T, IDX>(ec, (int64_t)t, a, b);
    const T idx = ax.id[0][i], idy = ax.id[1][j];
    if (i >= 1 && j >= 1)  // eps dEz/dt = dHy/dx - dHx/dy
      ezp[0] = a * ez + b * ((hy - hy_x) * idx - (hx - hx_y) * idy);
    if (src.n) add_sources<T, IDX>(f, ec, len, 1, (int64_t)t, src, u_n, lb);
  }
}

template <typename T, bool UNIFORM_H, typename I>
__global__ void __launch_bounds__(kBlock) k_h2(T* __restrict__ f, const T* __restrict__ da,
                                               const T* __restrict__ db, T db0, Axes<T> ax, int X,
                                               int Y, int64_t len, PrbList<T> prb,
                                               T* __restrict__ y_n, int xcd) {
  const unsigned lb = xcd_block(blockIdx.x, gridDim.x, xcd);
  const I t = (I)lb * (I)blockDim.x + (I)threadIdx.x;
  if (t < (I)len) {
    const I r = t / (I)X;
    const int i = (int)(t - r * (I)X), j = (int)r;
    const T* ezp = f + t;
    T* h = f + len + t;
    const T hx = h[0], hy = h[len];
    const T ez = ezp[0], ez_x = ezp[1], ez_y = ezp[X];
    T a0 = 1, a1 = 1, b0 = db0, b1 = db0;
    if (!UNIFORM_H) {
      a0 = da[t], a1 = da[len + t];
      b0 = db[t], b1 = db[len + t];
    }
    const T ipx = ax.ip[0][i], ipy = ax.ip[1][j];
    if (j < Y - 1)  // mu dHx/dt = -dEz/dy
      h[0] = a0 * hx + b0 * (-(ez_y - ez) * ipy);
    if (i < X - 1)  // mu dHy/dt = dEz/dx
      h[len] = a1 * hy + b1 * ((ez_x - ez) * ipx);
  }
  if (prb.n) gather_probes(f, prb, y_n);
}

// host helpers (fdtd.hip)
// stage_src sorts the entries by owning block (nblocks blocks of the electric
// kernel), stage_prb by port; both copy the lists into buf on stream s
template <typename T>
int stage_src(DevBuf& buf, const std::vector<PortEntry>& v, int nports, int nblocks,
              SrcList<T>& sl, hipStream_t s);
template <typename T>
int stage_prb(DevBuf& buf, const std::vector<PortEntry>& v, int nports, PrbList<T>& pl,
              hipStream_t s);
// number of blocks the electric kernel launches on this operator
unsigned e_blocks(const yr_operator* op);
// one electric (resp. magnetic) half step of the leapfrog on field buffer f
template <typename T>
void launch_e(const yr_operator* op, T* f, const SrcList<T>& sl, const T* u_n, hipStream_t s);
template <typename T>
void launch_h(const yr_operator* op, T* f, const PrbList<T>& pl, T* y_n, hipStream_t s);

}  // namespace yr
