// Shared host/device helpers of libyeerom: status handling, the operator
// object and the padded Yee-grid index arithmetic.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <utility>
#include <vector>

#include "yeerom.h"

namespace yr {

void set_error(const std::string& msg);

#define YR_TRY_HIP(expr)                                                          \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess) {                                                       \
      ::yr::set_error(std::string(#expr " failed: ") + hipGetErrorString(e_));   \
      return YR_EDEVICE;                                                          \
    }                                                                             \
  } while (0)

#define YR_REQUIRE(cond, code, msg) \
  do {                              \
    if (!(cond)) {                  \
      ::yr::set_error(msg);         \
      return (code);                \
    }                               \
  } while (0)

#define YR_CALL(expr)     \
  do {                    \
    int s_ = (expr);      \
    if (s_ != YR_OK) return s_; \
  } while (0)

// Device buffer owned by the library.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  // grows (never shrinks); contents are not preserved
  int reserve(size_t nbytes) {
    if (nbytes <= bytes) return YR_OK;
    release();
    if (nbytes == 0) return YR_OK;
    hipError_t e = hipMalloc(&p, nbytes);
    if (e != hipSuccess) {
      p = nullptr;
      set_error(std::string("hipMalloc failed: ") + hipGetErrorString(e));
      return YR_ENOMEM;
    }
    bytes = nbytes;
    return YR_OK;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
  void swap(DevBuf& o) {
    std::swap(p, o.p);
    std::swap(bytes, o.bytes);
  }
};

// Per-axis spacing tables on the device, one copy per precision.
// For axis a with n cells (node indices 0..n):
//   p[a][c]  primal spacing of cell c (c < n), 0 beyond
//   d[a][m]  dual spacing at node m (mean of the two adjacent cells)
//   ip, id   their reciprocals (0 where the spacing is 0)
template <typename T>
struct Axes {
  const T* p[3];
  const T* d[3];
  const T* ip[3];
  const T* id[3];
};

struct PortEntry {  // one electric sample of a port, resolved to the padded layout
  int64_t slot;     // offset in the field buffer (component * len + t)
  int32_t port;
  int32_t block;    // block of the E kernel that owns the slot
  double w;         // weight
};

}  // namespace yr

struct yr_operator {
  int dim = 3;
  int nx = 0, ny = 0, nz = 0;
  int X = 0, Y = 0, Z = 0;  // padded sizes (n+1; Z = 1 in 2-D)
  int64_t len = 0;          // entries per component
  int ne_slots = 3, nh_slots = 3;
  int64_t n_e = 0, n_h = 0;
  double dt_max = 0;
  double v0 = 1;  // reference cell volume
  std::vector<double> hp[3], hd[3];  // host primal / dual spacings (lengths X, Y, Z)
  bool uniform_h = true;  // mu_r == 1 and sigma_m == 0 everywhere
  bool lossless_e = true; // sigma_e == 0 everywhere
  // device data
  yr::DevBuf axes64, axes32;   // 12 tables each, see Axes
  yr::DevBuf eps_e, sig_e;     // FP64 [ne_slots*len], 0 at non-unknowns
  yr::DevBuf mu_h, sigm_h;     // FP64 [nh_slots*len], 0 at non-unknowns
  yr::DevBuf emask;            // uint8 [ne_slots*len], 1 at electric unknowns
  yr::DevBuf hmask;            // uint8 [nh_slots*len], 1 at magnetic unknowns
  std::vector<uint8_t> emask_host;  // host copy of emask (port validation)
  // leapfrog coefficient cache (one dt / dtype at a time)
  double coef_dt = -1;
  int coef_dtype = -1;
  yr::DevBuf ca, cb;  // dtype [ne_slots*len] (only when the electric index is off)
  // Electric coefficients by material number.  When the (D_eps, D_sigma_e)
  // pairs of the electric samples take at most 65535 (2^20) values, e_idx
  // numbers each sample in 16 (32) bits, 0 = not an unknown, and the leapfrog
  // reads ca, cb from a table of e_nmat pairs instead of two per-sample
  // streams (6 or 12 instead of 24 bytes per cell in FP32).  Built on first use.
  bool e_index_built = false;
  int e_idx_bytes = 0;                   // 0 (per-sample streams), 2 or 4
  int e_nmat = 0;
  std::vector<double> e_mat_d, e_mat_s;  // host: D_eps, D_sigma_e of each number
  yr::DevBuf e_idx;                      // uint16 / uint32 [ne_slots*len]
  yr::DevBuf e_tab;                      // dtype [2 e_nmat]: ca, cb per number
  yr::DevBuf da, db;  // dtype [nh_slots*len] (only when !uniform_h)
  double db_uniform = 0;
  // one-pass leapfrog (3-D): second field buffer, its element size, and the
  // path choice (0 automatic, 1 two half-step kernels, 2 one-pass)
  yr::DevBuf lf_buf;
  int lf_dtype = -1;
  int leapfrog_mode = 0;
  // port staging
  yr::DevBuf src_dev, prb_dev;
  std::vector<yr::PortEntry> src_host, prb_host;
  // recorded after the last launch that read the cached coefficients or the
  // staged port lists; a later call waits on it before rewriting them (the
  // earlier call may still run, on another stream)
  hipEvent_t busy = nullptr;
  bool busy_recorded = false;
  ~yr_operator() {
    if (busy) (void)hipEventDestroy(busy);
  }

  template <typename T>
  yr::Axes<T> axes() const {
    const yr::DevBuf& b = (sizeof(T) == 8) ? axes64 : axes32;
    const T* base = b.as<const T>();
    const int64_t n[3] = {X, Y, Z};
    yr::Axes<T> a;
    int64_t off = 0;
    for (int t = 0; t < 4; ++t)
      for (int ax = 0; ax < 3; ++ax) {
        const T* p = base + off;
        if (t == 0) a.p[ax] = p;
        if (t == 1) a.d[ax] = p;
        if (t == 2) a.ip[ax] = p;
        if (t == 3) a.id[ax] = p;
        off += n[ax];
      }
    return a;
  }
};

namespace yr {

// electric unknown ranges: component c (0..2 = Ex,Ey,Ez) at (i,j,k)
__host__ __device__ inline bool e_valid(int dim, int c, int i, int j, int k, int nx, int ny,
                                        int nz) {
  if (dim == 2) return c == 2 && i >= 1 && i <= nx - 1 && j >= 1 && j <= ny - 1 && k == 0;
  switch (c) {
    case 0: return i >= 0 && i < nx && j >= 1 && j <= ny - 1 && k >= 1 && k <= nz - 1;
    case 1: return i >= 1 && i <= nx - 1 && j >= 0 && j < ny && k >= 1 && k <= nz - 1;
    default: return i >= 1 && i <= nx - 1 && j >= 1 && j <= ny - 1 && k >= 0 && k < nz;
  }
}

// magnetic unknown ranges: component c (3..5 = Hx,Hy,Hz)
__host__ __device__ inline bool h_valid(int dim, int c, int i, int j, int k, int nx, int ny,
                                        int nz) {
  if (dim == 2) {
    if (c == 3) return i >= 1 && i <= nx - 1 && j >= 0 && j < ny && k == 0;
    return c == 4 && i >= 0 && i < nx && j >= 1 && j <= ny - 1 && k == 0;
  }
  switch (c) {
    case 3: return i >= 1 && i <= nx - 1 && j >= 0 && j < ny && k >= 0 && k < nz;
    case 4: return i >= 0 && i < nx && j >= 1 && j <= ny - 1 && k >= 0 && k < nz;
    default: return i >= 0 && i < nx && j >= 0 && j < ny && k >= 1 && k <= nz - 1;
  }
}

// slot of electric component c in the E half of a field buffer
inline int e_slot(int dim, int c) { return dim == 2 ? 0 : c; }

int resolve_ports(const yr_operator* op, const yr_ports* ports, std::vector<PortEntry>& out,
                  int block_threads);

int ensure_coefficients(yr_operator* op, double dt, yr_dtype dtype, hipStream_t stream);

// wait until no queued launch reads the operator's coefficients or staged
// port lists (op_wait_idle), and mark the launches just queued on s (op_mark_busy)
int op_wait_idle(yr_operator* op);
int op_mark_busy(yr_operator* op, hipStream_t s);

// W_e (dual area x primal length / V0) of an electric slot of the field buffer
double host_we(const yr_operator* op, int64_t slot);

constexpr int kBlock = 256;

inline unsigned grid_for(int64_t n, int threads = kBlock) {
  return static_cast<unsigned>((n + threads - 1) / threads);
}

}  // namespace yr
