// Curl stencils of eq. (matrix) on the padded Yee layout, and the row
// weights W_e, W_f that turn the field-form curls into K and K^T:
//   -K H   = W_e * curl_d(H)      (Ampere, dual grid)
//   K^T E  = W_f * cp(E),  cp(E) = -curl(E) (Faraday, primal grid)
// Slots: 3-D E = Ex,Ey,Ez and H = Hx,Hy,Hz; 2-D E = Ez and H = Hx,Hy.
// Callers evaluate the stencils only at unknowns (mask == 1), whose index
// ranges guarantee every neighbour read stays inside the padded box.
#pragma once

#include "common.hpp"
#include "cplx.hpp"

namespace yr {

struct Geo {
  int dim, X, Y, Z;
  int64_t len;
  int ne_slots, nh_slots;
  double inv_v0;
};

inline Geo geo_of(const yr_operator* op) {
  Geo g;
  g.dim = op->dim;
  g.X = op->X;
  g.Y = op->Y;
  g.Z = op->Z;
  g.len = op->len;
  g.ne_slots = op->ne_slots;
  g.nh_slots = op->nh_slots;
  g.inv_v0 = 1.0 / op->v0;
  return g;
}

__device__ inline void decode(int64_t t, const Geo& g, int& i, int& j, int& k) {
  i = (int)(t % g.X);
  int64_t r = t / g.X;
  j = (int)(r % g.Y);
  k = (int)(r / g.Y);
}

// dual curl at electric slot s, position t; hv(slot, index) reads H
template <typename V, typename R, typename F>
__device__ inline V curl_d(const Geo& g, const Axes<R>& ax, int s, int64_t t, int i, int j, int k,
                           F hv) {
  const int64_t sY = g.X, sZ = (int64_t)g.X * g.Y;
  if (g.dim == 2)  // Ez: dHy/dx - dHx/dy
    return (hv(1, t) - hv(1, t - 1)) * ax.id[0][i] - (hv(0, t) - hv(0, t - sY)) * ax.id[1][j];
  if (s == 0)  // Ex: dHz/dy - dHy/dz
    return (hv(2, t) - hv(2, t - sY)) * ax.id[1][j] - (hv(1, t) - hv(1, t - sZ)) * ax.id[2][k];
  if (s == 1)  // Ey: dHx/dz - dHz/dx
    return (hv(0, t) - hv(0, t - sZ)) * ax.id[2][k] - (hv(2, t) - hv(2, t - 1)) * ax.id[0][i];
  // Ez: dHy/dx - dHx/dy
  return (hv(1, t) - hv(1, t - 1)) * ax.id[0][i] - (hv(0, t) - hv(0, t - sY)) * ax.id[1][j];
}

// cp(E) = -curl E at magnetic slot s (the right-hand side of mu dH/dt)
template <typename V, typename R, typename F>
__device__ inline V curl_p(const Geo& g, const Axes<R>& ax, int s, int64_t t, int i, int j, int k,
                           F ev) {
  const int64_t sY = g.X, sZ = (int64_t)g.X * g.Y;
  if (g.dim == 2) {
    if (s == 0) return (ev(0, t) - ev(0, t + sY)) * ax.ip[1][j];  // Hx: -dEz/dy
    return (ev(0, t + 1) - ev(0, t)) * ax.ip[0][i];               // Hy: dEz/dx
  }
  if (s == 0)  // Hx: dEy/dz - dEz/dy
    return (ev(1, t + sZ) - ev(1, t)) * ax.ip[2][k] - (ev(2, t + sY) - ev(2, t)) * ax.ip[1][j];
  if (s == 1)  // Hy: dEz/dx - dEx/dz
    return (ev(2, t + 1) - ev(2, t)) * ax.ip[0][i] - (ev(0, t + sZ) - ev(0, t)) * ax.ip[2][k];
  // Hz: dEx/dy - dEy/dx
  return (ev(0, t + sY) - ev(0, t)) * ax.ip[1][j] - (ev(1, t + 1) - ev(1, t)) * ax.ip[0][i];
}

// W_e = dual area x primal length / V0 of electric slot s
template <typename R>
__device__ inline R w_e(const Geo& g, const Axes<R>& ax, int s, int i, int j, int k) {
  R w;
  if (g.dim == 2 || s == 2) w = ax.d[0][i] * ax.d[1][j] * ax.p[2][k];
  else if (s == 0) w = ax.p[0][i] * ax.d[1][j] * ax.d[2][k];
  else w = ax.d[0][i] * ax.p[1][j] * ax.d[2][k];
  return w * (R)g.inv_v0;
}

// W_f = primal area x dual length / V0 of magnetic slot s
template <typename R>
__device__ inline R w_h(const Geo& g, const Axes<R>& ax, int s, int i, int j, int k) {
  R w;
  if (s == 0) w = ax.d[0][i] * ax.p[1][j] * ax.p[2][k];
  else if (s == 1) w = ax.p[0][i] * ax.d[1][j] * ax.p[2][k];
  else w = ax.p[0][i] * ax.p[1][j] * ax.d[2][k];
  return w * (R)g.inv_v0;
}

// ---- block reductions (wave64 shuffles, then LDS across the waves)

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sums `n` per-thread values over the block; result valid in thread 0.
// `lds` must hold n * (blockDim.x / 64) doubles.
template <int N>
__device__ inline void block_sum(double (&v)[N], double* lds, double* out) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    double s = wave_sum(v[q]);
    if (lane == 0) lds[q * nw + wid] = s;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < N; q += blockDim.x) {
    double s = 0;
    for (int w = 0; w < nw; ++w) s += lds[q * nw + w];
    out[q] = s;
  }
}

}  // namespace yr
