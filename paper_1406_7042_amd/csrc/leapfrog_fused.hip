// One-pass leapfrog step for 3-D grids, eq. (MNAform) in field form:
//   E^{n+1} = ca E^n + cb (curl H^{n+1/2} + B u^{n+1})
//   H^{n+3/2} = da H^{n+1/2} - db curl E^{n+1}
// Both half steps of a step run in one sweep that reads E^n, H^{n+1/2} from
// one field buffer and writes E^{n+1}, H^{n+3/2} into a second one (the two
// buffers alternate between steps), so each field value crosses HBM once in
// and once out per step: 48 bytes per cell in FP32 instead of 72 for the two
// half-step kernels.
//
// A workgroup owns a TX x TY column of cells (TX / 64 wavefronts per row) over
// a run of z planes and marches up the planes.  At plane k it stages H^{n+1/2}
// of plane k with a one-cell low-side halo in LDS, forms E^{n+1} of plane k
// on the tile plus a one-cell high-side halo (column i0 + TX and row j0 + TY,
// computed by the first threads as a second position; the halo values are
// what the magnetic update of the tile's edge cells needs), keeps it in LDS
// (two planes) and then forms H^{n+3/2} of plane k - 1, whose curl needs
// E^{n+1} of planes k - 1 (LDS, with the halo) and k (the thread's own
// registers).  H^{n+1/2} stays in LDS for three planes (the plane below, the
// current one and the one being staged), so each plane takes two barriers,
// and the global loads of plane k + 1 are issued before plane k is computed.
// The chunk's last plane k1 is recomputed by the next chunk (E only, not
// stored).
//
// Positions i = nx, j = ny, k = nz of the padded layout hold no unknown of
// any component and are never written: both buffers keep them at zero.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

#include "common.hpp"
#include "fdtd_kernels.hpp"
#include "profile.hpp"

namespace yr {

template <int TX, int TY>
struct LfGeom {
  static_assert(TX % 64 == 0, "whole wavefronts per tile row");
  static constexpr int NT = TX * TY;
  static constexpr int RW = TX + 1, RH = TY + 1, RE = RW * RH;  // E region, high halo
  static constexpr int HW = TX + 2, HH = TY + 2, RHS = HW * HH;  // H region, both halos
  static constexpr int NHALO = TX + TY + 1;                      // halo positions of E
};

// Tile shapes: 128 x 8 or 64 x 16 (FP32, 1024 threads), 128 x 4 or 64 x 8
// (FP64, 512 threads).
struct LfShape {
  int tx, ty;
};

// Source entries of one workgroup, sorted by plane: entry (k, pos, c, port)
// adds w * cb * u[port] to component c of E region position pos at plane k.
template <typename T>
struct LfSrc {
  const int32_t* bptr;  // [nblocks + 1]
  const int32_t* k;
  const int32_t* pos;   // li + lj * RW
  const int32_t* c;
  const int32_t* port;
  const int64_t* slot;  // field-buffer offset (for the coefficient)
  const T* w;
};

struct LfTiling {
  int ntx, nty, nkz, KZ;  // tiles in x, y; z chunks; planes per chunk
  int per_xcd;            // tiles x chunks per XCD (blocks are dealt round-robin)
};

template <typename T, int TX, int TY, int IDX, bool UH>
__global__ void __launch_bounds__(TX * TY)
    k_leap3(const T* __restrict__ fin, T* __restrict__ fout, ECoef<T> ec,
            const T* __restrict__ da, const T* __restrict__ db, T db0, Axes<T> ax, int nx, int ny,
            int nz, int64_t len, LfTiling tl, LfSrc<T> src, const T* __restrict__ u_n,
            PrbList<T> prb, T* __restrict__ y_prev) {
  using G = LfGeom<TX, TY>;
  constexpr int NLS = (3 * G::RHS + G::NT - 1) / G::NT;  // H staging loads per thread
  // H^{n+1/2} of three planes (k - 1, k and the one being staged), E^{n+1}
  // of two (k - 1 and k)
  __shared__ T Hs[3 * 3 * G::RHS];
  __shared__ T Es[2 * 3 * G::RE];
  if (y_prev && prb.n) gather_probes(fin, prb, y_prev);  // E^n of the previous step
  const int b = blockIdx.x;
  const int wl = (b & 7) * tl.per_xcd + (b >> 3);
  if (wl >= tl.ntx * tl.nty * tl.nkz || (b >> 3) >= tl.per_xcd) return;
  const int tx = wl % tl.ntx, ty = (wl / tl.ntx) % tl.nty, ch = wl / (tl.ntx * tl.nty);
  const int i0 = tx * TX, j0 = ty * TY;
  const int k0 = ch * tl.KZ, k1 = min(nz, k0 + tl.KZ);
  const int X = nx + 1, Y = ny + 1;
  const int64_t XY = (int64_t)X * Y;
  // the thread's positions in the E region: slot 0 its own cell (x fastest),
  // slot 1 (first NHALO threads) a halo position: row TY, then column TX
  int li[2], lj[2];
  bool act[2];
  li[0] = threadIdx.x % TX;
  lj[0] = threadIdx.x / TX;
  act[0] = true;
  {
    const int h = threadIdx.x;
    act[1] = h < G::NHALO;
    li[1] = h < TX ? h : TX;
    lj[1] = h < TX ? TY : (act[1] ? h - TX : 0);  // inside the tile for every thread
  }
  uint32_t goff[2];  // offset of the position in a component plane
  bool inb[2];       // holds unknowns (i < nx, j < ny)
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const int i = i0 + li[s], j = j0 + lj[s];
    inb[s] = act[s] && i < nx && j < ny;
    goff[s] = inb[s] ? (uint32_t)(j * X + i) : 0u;
  }
  const bool own = inb[0];  // slot 0 cells are the tile's own
  // H staging slots of this thread: offsets from the start of a plane of
  // the first magnetic component (the components are len apart; a field
  // buffer of up to 2^31 values per component set)
  uint32_t hoff[NLS];
  bool hok[NLS];
#pragma unroll
  for (int u = 0; u < NLS; ++u) {
    const int idx = threadIdx.x + u * G::NT;
    const int c = idx / G::RHS, r = idx - c * G::RHS;
    const int rj = r / G::HW, ri = r - rj * G::HW;
    const int i = i0 - 1 + ri, j = j0 - 1 + rj;
    hok[u] = idx < 3 * G::RHS && i >= 0 && j >= 0 && i < X && j < Y;
    hoff[u] = hok[u] ? (uint32_t)(c * len + j * X + i) : 0u;
  }
  const T* fh = fin + 3 * len;
  // register pipeline: the loads of plane k + 1 fly while plane k is
  // computed (two planes deep measured no faster).  fetch() issues loads
  // only: positions off the grid read a valid element (offset 0 of their
  // plane, plane 0 off the box) and are zeroed or skipped where the values
  // are used, so no instruction needs a loaded value before the next plane (a
  // select right after a load makes the wave wait for it at once)
  struct Pl {
    T h[NLS], eo[2][3];
    uint32_t m[2][3];
    T idz, ipz;  // dual step along z at plane kk, primal step at kk - 1
    bool okz;
  };
  Pl S0;
  // steps along x and y at the thread's positions, read once (a table load
  // inside the plane loop would wait behind the prefetch)
  T aidx[2], aidy[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    aidx[s] = ax.id[0][min(i0 + li[s], nx - 1)];
    aidy[s] = ax.id[1][min(j0 + lj[s], ny - 1)];
  }
  const T aipx = ax.ip[0][min(i0 + li[0], nx - 1)], aipy = ax.ip[1][min(j0 + lj[0], ny - 1)];
  // Called once per plane, also past the chunk's last plane (k1 + 1): the
  // loads must not sit behind a branch, or the waits after the branch merge
  // would count as if they had not been issued and wait for them all.  The
  // plane read is kk clamped to [0, min(k1, nz - 1)] (past the chunk: plane
  // k1 again, cache hits); the address differs only by a uniform offset, so
  // no lane takes another instruction form.
  auto fetch = [&](Pl& S, int kk) __attribute__((always_inline)) {
    S.okz = kk >= 0 && kk < nz;
    const int kr = max(0, min(kk, min(k1, nz - 1)));
    const int64_t kz = (int64_t)kr * XY;
    S.idz = ax.id[2][kr];
    S.ipz = ax.ip[2][kk >= 1 && kk <= nz ? kk - 1 : 0];
#pragma unroll
    for (int u = 0; u < NLS; ++u) S.h[u] = fh[kz + hoff[u]];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int64_t g = c * len + kz + goff[s];
        S.eo[s][c] = fin[g];  // used only where inb[s] on a plane of the box
        if (IDX) S.m[s][c] = e_material<IDX>(ec.idx, g);
      }
  };
  auto stage = [&](const Pl& S, int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < NLS; ++u) {
      const int idx = threadIdx.x + u * G::NT;
      if (idx < 3 * G::RHS) Hs[buf * 3 * G::RHS + idx] = S.okz && hok[u] ? S.h[u] : T(0);
    }
  };
  // H of plane k0 - 1 into LDS buffer (k0 + 2) % 3, then plane k0 in flight
  fetch(S0, k0 - 1);
  stage(S0, (k0 + 2) % 3);
  fetch(S0, k0);
  T ep[3] = {T(0), T(0), T(0)};  // E^{n+1} of plane k - 1 at slot 0
  int sp = src.bptr ? src.bptr[b] : 0;
  const int se = src.bptr ? src.bptr[b + 1] : 0;

  auto plane = [&](int k, Pl& S) __attribute__((always_inline)) {
    const bool eplane = k < nz;  // plane k holds electric unknowns
    const int hb = k % 3, hbp = (k + 2) % 3;  // LDS buffers of H planes k and k - 1
    stage(S, hb);
    // steps along z of planes k (electric) and k - 1 (magnetic), before S
    // takes plane k + 1
    const T idz_k = S.idz, ipz = S.ipz;
    T eo[2][3], ca_[2][3], cb_[2][3];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        eo[s][c] = S.eo[s][c];
        // unconditional loads (every material number read is a valid entry;
        // plane nz lies inside the buffers): the coefficients are used only
        // where inb[s] on a plane of the box
        if (IDX) {
          ca_[s][c] = ec.tab[2 * S.m[s][c]];
          cb_[s][c] = ec.tab[2 * S.m[s][c] + 1];
        } else {
          const int64_t g = c * len + (int64_t)k * XY + goff[s];
          ca_[s][c] = ec.ca[g];
          cb_[s][c] = ec.cb[g];
        }
      }
    fetch(S, k + 1);
    __syncthreads();
    // ---- E^{n+1} of plane k
    const int eb = (k & 1) * 3 * G::RE;
    const T* Hc = Hs + hb * 3 * G::RHS;
    const T* Hp = Hs + hbp * 3 * G::RHS;
    T en0[3] = {T(0), T(0), T(0)};
    const T idz = eplane ? idz_k : T(0);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int hl = (lj[s] + 1) * G::HW + (li[s] + 1);
      // formed on every thread (hl lies inside the staged region for every
      // slot) and masked after: straight-line code, so the waits for the
      // coefficient loads count past the prefetch of plane k + 1
      const bool ok = inb[s] && eplane;
      const int i = i0 + li[s], j = j0 + lj[s];
      const T idx_ = aidx[s], idy = aidy[s];
      const T hx = Hc[hl], hy = Hc[G::RHS + hl], hz = Hc[2 * G::RHS + hl];
      const T hz_y = Hc[2 * G::RHS + hl - G::HW], hy_x = Hc[G::RHS + hl - 1];
      const T hz_x = Hc[2 * G::RHS + hl - 1], hx_y = Hc[hl - G::HW];
      const T hx_z = Hp[hl], hy_z = Hp[G::RHS + hl];
      // eps dEx/dt = dHz/dy - dHy/dz; eps dEy/dt = dHx/dz - dHz/dx;
      // eps dEz/dt = dHy/dx - dHx/dy
      const T f0 = ca_[s][0] * eo[s][0] + cb_[s][0] * ((hz - hz_y) * idy - (hy - hy_z) * idz);
      const T f1 = ca_[s][1] * eo[s][1] + cb_[s][1] * ((hx - hx_z) * idz - (hz - hz_x) * idx_);
      const T f2 = ca_[s][2] * eo[s][2] + cb_[s][2] * ((hy - hy_x) * idx_ - (hx - hx_y) * idy);
      const T e0 = ok && j >= 1 && k >= 1 ? f0 : T(0);
      const T e1 = ok && i >= 1 && k >= 1 ? f1 : T(0);
      const T e2 = ok && i >= 1 && j >= 1 ? f2 : T(0);
      if (s == 0) {
        en0[0] = e0;
        en0[1] = e1;
        en0[2] = e2;
      }
      if (act[s]) {
        const int el = lj[s] * G::RW + li[s];
        Es[eb + el] = e0;
        Es[eb + G::RE + el] = e1;
        Es[eb + 2 * G::RE + el] = e2;
      }
    }
    // ---- sources of plane k (entries sorted by plane)
    int sq = sp;
    while (sq < se && src.k[sq] == k) ++sq;
    if (sq > sp) {  // uniform across the block
      __syncthreads();
      for (int q = sp + (int)threadIdx.x; q < sq; q += G::NT) {
        T a, bb;
        e_coef<T, IDX>(ec, src.slot[q], a, bb);
        atomicAdd(&Es[eb + src.c[q] * G::RE + src.pos[q]], bb * src.w[q] * u_n[src.port[q]]);
      }
      __syncthreads();
      const int el = lj[0] * G::RW + li[0];
#pragma unroll
      for (int c = 0; c < 3; ++c) en0[c] = Es[eb + c * G::RE + el];
      sp = sq;
    }
    if (own && k < k1) {
      const int64_t g = (int64_t)k * XY + goff[0];
      fout[g] = en0[0];
      fout[len + g] = en0[1];
      fout[2 * len + g] = en0[2];
    }
    __syncthreads();
    // ---- H^{n+3/2} of plane k - 1 (needs E^{n+1} of planes k - 1 and k)
    if (k > k0 && own) {
      const int kh = k - 1;
      const int pb = ((k - 1) & 1) * 3 * G::RE;
      const int el = lj[0] * G::RW + li[0];
      const int hl = (lj[0] + 1) * G::HW + (li[0] + 1);
      const int i = i0 + li[0], j = j0 + lj[0];
      const T ipx = aipx, ipy = aipy;
      const T ex = ep[0], ey = ep[1], ez = ep[2];
      const T ey_x = Es[pb + G::RE + el + 1], ez_x = Es[pb + 2 * G::RE + el + 1];
      const T ex_y = Es[pb + el + G::RW], ez_y = Es[pb + 2 * G::RE + el + G::RW];
      const T ex_z = en0[0], ey_z = en0[1];
      const T hx = Hp[hl], hy = Hp[G::RHS + hl], hz = Hp[2 * G::RHS + hl];
      const int64_t g = 3 * len + (int64_t)kh * XY + goff[0];
      T a0 = 1, a1 = 1, a2 = 1, b0 = db0, b1 = db0, b2 = db0;
      if (!UH) {
        a0 = da[g - 3 * len];
        a1 = da[g - 2 * len];
        a2 = da[g - len];
        b0 = db[g - 3 * len];
        b1 = db[g - 2 * len];
        b2 = db[g - len];
      }
      T h0 = 0, h1 = 0, h2 = 0;
      if (j < ny)  // mu dHx/dt = dEy/dz - dEz/dy
        h0 = a0 * hx + b0 * ((ey_z - ey) * ipz - (ez_y - ez) * ipy);
      if (i < nx)  // mu dHy/dt = dEz/dx - dEx/dz
        h1 = a1 * hy + b1 * ((ez_x - ez) * ipx - (ex_z - ex) * ipz);
      if (i < nx && j < ny)  // mu dHz/dt = dEx/dy - dEy/dx
        h2 = a2 * hz + b2 * ((ex_y - ex) * ipy - (ey_x - ey) * ipx);
      fout[g] = h0;
      fout[g + len] = h1;
      fout[g + 2 * len] = h2;
    }
    ep[0] = en0[0];
    ep[1] = en0[1];
    ep[2] = en0[2];
  };
  for (int k = k0; k <= k1; ++k) plane(k, S0);
}

template <typename T>
__global__ void k_gather(const T* __restrict__ f, PrbList<T> prb, T* __restrict__ y) {
  gather_probes(f, prb, y);
}

// ------------------------------------------------------------------ host

static LfTiling lf_tiling(const yr_operator* op, LfShape sh) {
  LfTiling t;
  t.ntx = (op->nx + sh.tx - 1) / sh.tx;
  t.nty = (op->ny + sh.ty - 1) / sh.ty;
  const int64_t tiles = (int64_t)t.ntx * t.nty;
  int kz;
  if (sh.tx * sh.ty == 1024) {
    // one 1024-thread workgroup per compute unit at a time: a run takes
    // ceil(workgroups / 256) rounds of (planes per chunk + 1) plane steps
    // (the chunk's last plane is recomputed by the next chunk); take the
    // chunk length that minimises that product, the longer one on a tie
    // (192^3: 7 planes, 1008 workgroups instead of 8 planes, 864 of them
    // with the fourth round a third full)
    kz = op->nz;
    int64_t best = -1;
    for (int c = 4; c <= op->nz; ++c) {
      const int64_t wg = tiles * ((op->nz + c - 1) / c);
      const int64_t cost = (wg + 255) / 256 * (c + 1);
      if (best < 0 || cost <= best) {
        best = cost;
        kz = c;
      }
    }
  } else {
    // about 4 workgroups per compute unit over the whole box, >= 8 planes each
    kz = (int)std::max<int64_t>(8, (tiles * op->nz + 1023) / 1024);
  }
  if (const char* e = std::getenv("YR_LF_KZ")) {  // tuning sweeps
    const int v = std::atoi(e);
    if (v >= 2) kz = v;
  }
  kz = std::min(kz, op->nz);
  t.KZ = kz;
  t.nkz = (op->nz + kz - 1) / kz;
  t.per_xcd = (int)((tiles * t.nkz + 7) / 8);
  return t;
}

// Tile shape.  FP32: 128 x 8 (LDS 75 KB) where the wider tiles cover the x
// extent with no more padding than 64-wide ones, else 64 x 16.  Each field
// row is then read in runs of 512 instead of 256 bytes, and the HBM-streamed
// boxes are bound by how the tiles walk memory more than by the bytes: the
// same loads and stores marched over a 256^3 box with no stencil at all take
// 272 us per step on 64 x 16 tiles and 228 us on 128 x 8, a flat stream of
// them 196 us.  The one-pass step gains less (256^3: 279 -> 264 us; 200^3:
// 171 -> 149 us), its H halo being a larger share of a 128 x 8 tile.  FP64:
// 64 x 8 (512 threads, LDS 76 KB); 128 x 4 measured slower (256^3: 484 vs
// 496 us).
static LfShape lf_shape(const yr_operator* op, size_t es) {
  const int w128 = (op->nx + 127) / 128 * 128, w64 = (op->nx + 63) / 64 * 64;
  bool wide = es == 4 && 20 * w128 <= 21 * w64;
  if (const char* e = std::getenv("YR_LF_TX")) wide = std::atoi(e) == 128;  // tuning sweeps
  if (es == 8) return wide ? LfShape{128, 4} : LfShape{64, 8};
  return wide ? LfShape{128, 8} : LfShape{64, 16};
}

// Source entries grouped by workgroup (an entry inside a neighbour's halo
// belongs to both), sorted by plane, staged into buf.
template <typename T>
static int stage_lf_sources(const yr_operator* op, LfShape sh, const std::vector<PortEntry>& v,
                            DevBuf& buf, LfSrc<T>& out, hipStream_t stream) {
  const int TX = sh.tx, TY = sh.ty, RW = TX + 1;
  const LfTiling t = lf_tiling(op, sh);
  const int nb = 8 * t.per_xcd;
  struct E {
    int blk, k, pos, c, port;
    int64_t slot;
    double w;
  };
  std::vector<E> es;
  const int X = op->X, Y = op->Y;
  for (const auto& e : v) {
    const int c = (int)(e.slot / op->len);
    const int64_t tpos = e.slot - c * op->len;
    const int i = (int)(tpos % X), j = (int)((tpos / X) % Y), k = (int)(tpos / ((int64_t)X * Y));
    // workgroups whose E region (tile + high halo, planes k0 .. k1) holds it
    for (int ch = 0; ch < t.nkz; ++ch) {
      const int k0 = ch * t.KZ, k1 = std::min(op->nz, k0 + t.KZ);
      if (k < k0 || k > k1) continue;
      for (int tyy = 0; tyy < t.nty; ++tyy) {
        const int lj = j - tyy * TY;
        if (lj < 0 || lj > TY) continue;
        for (int txx = 0; txx < t.ntx; ++txx) {
          const int li = i - txx * TX;
          if (li < 0 || li > TX) continue;
          if (li == TX && lj == TY) continue;  // the corner is no halo position
          const int wl = (ch * t.nty + tyy) * t.ntx + txx;
          const int blk = (wl % t.per_xcd) * 8 + wl / t.per_xcd;
          es.push_back({blk, k, li + lj * RW, c, e.port, e.slot, e.w});
        }
      }
    }
  }
  std::stable_sort(es.begin(), es.end(), [](const E& a, const E& b) {
    return a.blk != b.blk ? a.blk < b.blk : a.k < b.k;
  });
  const size_t n = es.size();
  const size_t o_k = 4 * (size_t)(nb + 1), o_p = o_k + 4 * n, o_c = o_p + 4 * n,
               o_q = o_c + 4 * n, o_s = (o_q + 4 * n + 7) / 8 * 8, o_w = o_s + 8 * n;
  std::vector<char> h(o_w + sizeof(T) * n + 16, 0);
  int32_t* bp = reinterpret_cast<int32_t*>(h.data());
  for (size_t q = 0; q < n; ++q) {
    bp[es[q].blk + 1] += 1;
    reinterpret_cast<int32_t*>(h.data() + o_k)[q] = es[q].k;
    reinterpret_cast<int32_t*>(h.data() + o_p)[q] = es[q].pos;
    reinterpret_cast<int32_t*>(h.data() + o_c)[q] = es[q].c;
    reinterpret_cast<int32_t*>(h.data() + o_q)[q] = es[q].port;
    reinterpret_cast<int64_t*>(h.data() + o_s)[q] = es[q].slot;
    reinterpret_cast<T*>(h.data() + o_w)[q] = (T)es[q].w;
  }
  for (int q = 0; q < nb; ++q) bp[q + 1] += bp[q];
  YR_CALL(buf.reserve(h.size()));
  YR_TRY_HIP(hipMemcpyAsync(buf.p, h.data(), h.size(), hipMemcpyHostToDevice, stream));
  YR_TRY_HIP(hipStreamSynchronize(stream));  // pageable source
  const char* d = buf.as<char>();
  out.bptr = n ? reinterpret_cast<const int32_t*>(d) : nullptr;
  out.k = reinterpret_cast<const int32_t*>(d + o_k);
  out.pos = reinterpret_cast<const int32_t*>(d + o_p);
  out.c = reinterpret_cast<const int32_t*>(d + o_c);
  out.port = reinterpret_cast<const int32_t*>(d + o_q);
  out.slot = reinterpret_cast<const int64_t*>(d + o_s);
  out.w = reinterpret_cast<const T*>(d + o_w);
  return YR_OK;
}

template <typename T, int TX, int TY, int IDX, bool UH>
static void launch_leap3_t(const yr_operator* op, const T* fin, T* fout, const LfTiling& t,
                           const LfSrc<T>& src, const T* u_n, const PrbList<T>& pl, T* y_prev,
                           hipStream_t s) {
  ECoef<T> ec{op->ca.as<T>(), op->cb.as<T>(), op->e_idx.p, op->e_tab.as<T>()};
  k_leap3<T, TX, TY, IDX, UH><<<8 * t.per_xcd, LfGeom<TX, TY>::NT, 0, s>>>(
      fin, fout, ec, op->da.as<T>(), op->db.as<T>(), (T)op->db_uniform, op->axes<T>(), op->nx,
      op->ny, op->nz, op->len, t, src, u_n, pl, y_prev);
}

template <typename T>
static void launch_leap3(const yr_operator* op, LfShape sh, const T* fin, T* fout, const LfTiling& t,
                         const LfSrc<T>& src, const T* u_n, const PrbList<T>& pl, T* y_prev,
                         hipStream_t s) {
  ProfScope ps("fdtd_fused", s);
  const int ix = op->e_idx_bytes;
  const bool uh = op->uniform_h;
#define YR_LF(TX_, TY_, IX_)                                                                     \
  do {                                                                                           \
    if (uh) launch_leap3_t<T, TX_, TY_, IX_, true>(op, fin, fout, t, src, u_n, pl, y_prev, s);   \
    else launch_leap3_t<T, TX_, TY_, IX_, false>(op, fin, fout, t, src, u_n, pl, y_prev, s);     \
  } while (0)
#define YR_LF_SHAPE(TX_, TY_)            \
  do {                                   \
    if (ix == 2) YR_LF(TX_, TY_, 2);     \
    else if (ix == 4) YR_LF(TX_, TY_, 4); \
    else YR_LF(TX_, TY_, 0);             \
  } while (0)
  if constexpr (sizeof(T) == 8) {
    if (sh.tx == 128) YR_LF_SHAPE(128, 4);
    else YR_LF_SHAPE(64, 8);
  } else {
    if (sh.tx == 64) YR_LF_SHAPE(64, 16);
    else YR_LF_SHAPE(128, 8);
  }
#undef YR_LF_SHAPE
#undef YR_LF
}

// nsteps one-pass steps on f (3-D), with the operator's second field buffer;
// the final fields end in f
template <typename T>
int run_fdtd_fused(yr_operator* op, int64_t nsteps, T* f, const T* u, T* y, int nsrc, int nprb,
                   hipStream_t stream) {
  const LfShape sh = lf_shape(op, sizeof(T));
  const LfTiling t = lf_tiling(op, sh);
  const int64_t flen = (int64_t)(op->ne_slots + op->nh_slots) * op->len;
  // the second buffer's positions without unknowns are never written: zero
  // them whenever the buffer is new or held the other precision
  if (op->lf_buf.bytes < (size_t)flen * sizeof(T) || op->lf_dtype != (int)sizeof(T)) {
    YR_CALL(op->lf_buf.reserve((size_t)flen * sizeof(T)));
    YR_TRY_HIP(hipMemsetAsync(op->lf_buf.p, 0, (size_t)flen * sizeof(T), stream));
    op->lf_dtype = (int)sizeof(T);
  }
  LfSrc<T> src{};
  YR_CALL(stage_lf_sources<T>(op, sh, op->src_host, op->src_dev, src, stream));
  PrbList<T> pl{};
  YR_CALL(stage_prb<T>(op->prb_dev, op->prb_host, nprb, pl, stream));
  T* buf[2] = {f, op->lf_buf.as<T>()};
  for (int64_t n = 0; n < nsteps; ++n) {
    const T* fin = buf[n & 1];
    T* fout = buf[(n + 1) & 1];
    T* yp = (pl.n && n > 0) ? y + (n - 1) * nprb : nullptr;
    launch_leap3<T>(op, sh, fin, fout, t, src, nsrc ? u + n * nsrc : nullptr, pl, yp, stream);
  }
  T* last = buf[nsteps & 1];
  if (pl.n) k_gather<T><<<1, kBlock, 0, stream>>>(last, pl, y + (nsteps - 1) * nprb);
  if (last != f)
    YR_TRY_HIP(hipMemcpyAsync(f, last, (size_t)flen * sizeof(T), hipMemcpyDeviceToDevice, stream));
  YR_TRY_HIP(hipGetLastError());
  return YR_OK;
}

template int run_fdtd_fused<float>(yr_operator*, int64_t, float*, const float*, float*, int, int,
                                   hipStream_t);
template int run_fdtd_fused<double>(yr_operator*, int64_t, double*, const double*, double*, int,
                                    int, hipStream_t);

}  // namespace yr
