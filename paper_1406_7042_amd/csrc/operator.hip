// Discretisation (Sec. II-A): per-cell materials -> the diagonal matrices of
// eq. (matrix) on the padded Yee samples, grid spacing tables, ports.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"

namespace yr {

namespace {
thread_local std::string g_last_error;
constexpr double kMu0 = 1.25663706212e-6;  // H/m, CODATA 2018
constexpr double kC0 = 299792458.0;        // m/s
const double kEps0 = 1.0 / (kMu0 * kC0 * kC0);
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

double host_we(const yr_operator* op, int64_t slot) {
  int s = (int)(slot / op->len);
  int64_t t = slot - s * op->len;
  int i = (int)(t % op->X);
  int64_t r = t / op->X;
  int j = (int)(r % op->Y);
  int k = (int)(r / op->Y);
  const auto& p = op->hp;
  const auto& d = op->hd;
  double w;
  if (op->dim == 2 || s == 2) w = d[0][i] * d[1][j] * p[2][k];
  else if (s == 0) w = p[0][i] * d[1][j] * d[2][k];
  else w = d[0][i] * p[1][j] * d[2][k];
  return w / op->v0;
}

// ---------------------------------------------------------------- kernels

__global__ void k_mark_pec(uint8_t* __restrict__ mask, const int64_t* __restrict__ slots,
                           int64_t n) {
  int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) mask[slots[t]] = 2;  // 2 = PEC (removed unknown)
}

struct CellTables {
  const double* eps_r;  // may be null -> 1
  const double* sig_e;  // may be null -> 0
  const double* mu_r;
  const double* sig_m;
};

__device__ inline double cell_or(const double* a, int nx, int ny, int i, int j, int k,
                                 double dflt) {
  return a ? a[((int64_t)k * ny + j) * nx + i] : dflt;
}

// electric samples: dual-area weighted mean of the touching cells
__global__ void k_average_e(double* __restrict__ eps_e, double* __restrict__ sig_e,
                            uint8_t* __restrict__ emask, CellTables ct, Axes<double> ax, int dim,
                            int nx, int ny, int nz, int X, int Y, int64_t len, int nslots,
                            double eps0) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= nslots * len) return;
  int s = (int)(g / len);
  int64_t t = g - s * len;
  int i = (int)(t % X);
  int64_t r = t / X;
  int j = (int)(r % Y);
  int k = (int)(r / Y);
  int c = dim == 2 ? 2 : s;
  bool valid = e_valid(dim, c, i, j, k, nx, ny, nz) && emask[g] != 2;
  emask[g] = valid ? 1 : 0;
  if (!valid) {
    eps_e[g] = 0;
    sig_e[g] = 0;
    return;
  }
  int ci[4], cj[4], ck[4];
  double w[4];
  const double* px = ax.p[0];
  const double* py = ax.p[1];
  const double* pz = ax.p[2];
  if (dim == 2 || c == 2) {  // cells (i-1..i, j-1..j, k)
    for (int q = 0; q < 4; ++q) {
      ci[q] = i - 1 + (q & 1);
      cj[q] = j - 1 + (q >> 1);
      ck[q] = k;
      w[q] = px[ci[q]] * py[cj[q]];
    }
  } else if (c == 0) {  // cells (i, j-1..j, k-1..k)
    for (int q = 0; q < 4; ++q) {
      ci[q] = i;
      cj[q] = j - 1 + (q & 1);
      ck[q] = k - 1 + (q >> 1);
      w[q] = py[cj[q]] * pz[ck[q]];
    }
  } else {  // c == 1: cells (i-1..i, j, k-1..k)
    for (int q = 0; q < 4; ++q) {
      ci[q] = i - 1 + (q & 1);
      cj[q] = j;
      ck[q] = k - 1 + (q >> 1);
      w[q] = px[ci[q]] * pz[ck[q]];
    }
  }
  double ws = 0, e = 0, sg = 0;
  for (int q = 0; q < 4; ++q) {
    ws += w[q];
    e += w[q] * cell_or(ct.eps_r, nx, ny, ci[q], cj[q], ck[q], 1.0);
    sg += w[q] * cell_or(ct.sig_e, nx, ny, ci[q], cj[q], ck[q], 0.0);
  }
  eps_e[g] = eps0 * e / ws;
  sig_e[g] = sg / ws;
}

// magnetic samples: dual-length weighted mean of the two touching cells
__global__ void k_average_h(double* __restrict__ mu_h, double* __restrict__ sigm_h,
                            uint8_t* __restrict__ hmask, CellTables ct, Axes<double> ax, int dim,
                            int nx, int ny, int nz, int X, int Y, int64_t len, int nslots,
                            double mu0) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= nslots * len) return;
  int s = (int)(g / len);
  int64_t t = g - s * len;
  int i = (int)(t % X);
  int64_t r = t / X;
  int j = (int)(r % Y);
  int k = (int)(r / Y);
  int c = 3 + s;
  bool valid = h_valid(dim, c, i, j, k, nx, ny, nz);
  hmask[g] = valid ? 1 : 0;
  if (!valid) {
    mu_h[g] = 0;
    sigm_h[g] = 0;
    return;
  }
  int ai = i, aj = j, ak = k;  // the other cell is one step back along the normal
  double w0, w1;
  if (c == 3) {
    ai = i - 1;
    w0 = ax.p[0][ai];
    w1 = ax.p[0][i];
  } else if (c == 4) {
    aj = j - 1;
    w0 = ax.p[1][aj];
    w1 = ax.p[1][j];
  } else {
    ak = k - 1;
    w0 = ax.p[2][ak];
    w1 = ax.p[2][k];
  }
  double m = w0 * cell_or(ct.mu_r, nx, ny, ai, aj, ak, 1.0) + w1 * cell_or(ct.mu_r, nx, ny, i, j, k, 1.0);
  double sm = w0 * cell_or(ct.sig_m, nx, ny, ai, aj, ak, 0.0) + w1 * cell_or(ct.sig_m, nx, ny, i, j, k, 0.0);
  mu_h[g] = mu0 * m / (w0 + w1);
  sigm_h[g] = sm / (w0 + w1);
}

// leapfrog coefficients of eq. (MNAform) in field form:
//   a = (D/dt - S/2) / (D/dt + S/2),  b = 1 / (D/dt + S/2),  0 at non-unknowns
template <typename T>
__global__ void k_coefficients(T* __restrict__ a, T* __restrict__ b, const double* __restrict__ d,
                               const double* __restrict__ s, int64_t n, double dt) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= n) return;
  double dd = d[g];
  if (dd > 0) {
    double p = dd / dt + 0.5 * s[g];
    double m = dd / dt - 0.5 * s[g];
    a[g] = (T)(m / p);
    b[g] = (T)(1.0 / p);
  } else {
    a[g] = 0;
    b[g] = 0;
  }
}

// ---------------------------------------------------------------- host helpers

template <typename T>
static int upload_axes(yr_operator* op, DevBuf& buf) {
  const int64_t n[3] = {op->X, op->Y, op->Z};
  std::vector<T> h;
  for (int t = 0; t < 4; ++t)
    for (int ax = 0; ax < 3; ++ax)
      for (int64_t m = 0; m < n[ax]; ++m) {
        double v = (t == 0 || t == 2) ? op->hp[ax][m] : op->hd[ax][m];
        if (t >= 2) v = v > 0 ? 1.0 / v : 0.0;
        h.push_back((T)v);
      }
  YR_CALL(buf.reserve(h.size() * sizeof(T)));
  YR_TRY_HIP(hipMemcpy(buf.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return YR_OK;
}

// Numbers the distinct (D_eps, D_sigma_e) pairs of the electric samples
// (open addressing on their bit patterns, the table doubled as it fills);
// 16-bit numbers up to 65535 pairs, 32-bit up to 2^20, per-sample streams
// beyond (the table would no longer stay in cache).
static int build_e_index(yr_operator* op) {
  op->e_index_built = true;
  op->e_idx_bytes = 0;
  const int64_t ne = op->ne_slots * op->len;
  std::vector<double> d(ne), sg(ne);
  std::vector<uint8_t> m(ne);
  YR_TRY_HIP(hipMemcpy(d.data(), op->eps_e.p, ne * 8, hipMemcpyDeviceToHost));
  YR_TRY_HIP(hipMemcpy(sg.data(), op->sig_e.p, ne * 8, hipMemcpyDeviceToHost));
  YR_TRY_HIP(hipMemcpy(m.data(), op->emask.p, ne, hipMemcpyDeviceToHost));
  constexpr size_t kMaxMat = (size_t)1 << 20;
  size_t cap = (size_t)1 << 16;  // slots, a power of two, kept >= 2 x entries
  std::vector<int32_t> slot(cap, -1);
  std::vector<uint64_t> kd, ks;
  std::vector<uint32_t> idx(ne, 0);
  auto hash = [](uint64_t a, uint64_t b) {
    return a * 0x9E3779B97F4A7C15ull ^ (b + 0x632BE59BD9B4E019ull) * 0xC2B2AE3D27D4EB4Full;
  };
  auto insert_slot = [&](uint64_t a, uint64_t b, int32_t e) {
    size_t q = (size_t)(hash(a, b) >> 20) & (cap - 1);
    while (slot[q] >= 0) q = (q + 1) & (cap - 1);
    slot[q] = e;
  };
  op->e_mat_d.assign(1, 0.0);  // number 0: not an unknown (ca = cb = 0)
  op->e_mat_s.assign(1, 0.0);
  for (int64_t g = 0; g < ne; ++g) {
    if (m[g] != 1) continue;
    uint64_t a, b;
    std::memcpy(&a, &d[g], 8);
    std::memcpy(&b, &sg[g], 8);
    size_t q = (size_t)(hash(a, b) >> 20) & (cap - 1);
    while (true) {
      const int32_t e = slot[q];
      if (e < 0) {
        if (kd.size() + 1 >= kMaxMat) return YR_OK;  // too many: per-sample streams
        const int32_t ne_ = (int32_t)kd.size();
        kd.push_back(a);
        ks.push_back(b);
        op->e_mat_d.push_back(d[g]);
        op->e_mat_s.push_back(sg[g]);
        idx[g] = (uint32_t)(ne_ + 1);
        slot[q] = ne_;
        if (2 * kd.size() > cap) {  // grow and reinsert
          cap *= 2;
          slot.assign(cap, -1);
          for (int32_t r = 0; r < (int32_t)kd.size(); ++r) insert_slot(kd[r], ks[r], r);
        }
        break;
      }
      if (kd[e] == a && ks[e] == b) {
        idx[g] = (uint32_t)(e + 1);
        break;
      }
      q = (q + 1) & (cap - 1);
    }
  }
  op->e_nmat = (int)op->e_mat_d.size();
  const int bytes = op->e_nmat <= 65536 ? 2 : 4;
  YR_CALL(op->e_idx.reserve((size_t)ne * bytes));
  YR_CALL(op->e_tab.reserve((size_t)2 * op->e_nmat * 8));
  if (bytes == 2) {
    std::vector<uint16_t> i16(idx.begin(), idx.end());
    YR_TRY_HIP(hipMemcpy(op->e_idx.p, i16.data(), (size_t)ne * 2, hipMemcpyHostToDevice));
  } else {
    YR_TRY_HIP(hipMemcpy(op->e_idx.p, idx.data(), (size_t)ne * 4, hipMemcpyHostToDevice));
  }
  op->e_idx_bytes = bytes;
  return YR_OK;
}

int ensure_coefficients(yr_operator* op, double dt, yr_dtype dtype, hipStream_t stream) {
  if (op->coef_dt == dt && op->coef_dtype == (int)dtype) return YR_OK;
  size_t es = dtype == YR_F64 ? 8 : 4;
  int64_t ne = op->ne_slots * op->len, nh = op->nh_slots * op->len;
  if (!op->e_index_built) YR_CALL(build_e_index(op));
  if (op->e_idx_bytes) {
    // the same formula as k_coefficients, per material number, on the host
    const int n = op->e_nmat;
    std::vector<double> t64(2 * (size_t)n, 0.0);
    for (int q = 1; q < n; ++q) {
      const double p = op->e_mat_d[q] / dt + 0.5 * op->e_mat_s[q];
      const double mm = op->e_mat_d[q] / dt - 0.5 * op->e_mat_s[q];
      t64[2 * q] = mm / p;
      t64[2 * q + 1] = 1.0 / p;
    }
    if (dtype == YR_F64) {
      YR_TRY_HIP(hipMemcpyAsync(op->e_tab.p, t64.data(), t64.size() * 8, hipMemcpyHostToDevice,
                                stream));
      YR_TRY_HIP(hipStreamSynchronize(stream));  // pageable source
    } else {
      std::vector<float> t32(t64.begin(), t64.end());
      YR_TRY_HIP(hipMemcpyAsync(op->e_tab.p, t32.data(), t32.size() * 4, hipMemcpyHostToDevice,
                                stream));
      YR_TRY_HIP(hipStreamSynchronize(stream));
    }
  } else {
    YR_CALL(op->ca.reserve(ne * es));
    YR_CALL(op->cb.reserve(ne * es));
    if (dtype == YR_F64)
      k_coefficients<double><<<grid_for(ne), kBlock, 0, stream>>>(
          op->ca.as<double>(), op->cb.as<double>(), op->eps_e.as<double>(),
          op->sig_e.as<double>(), ne, dt);
    else
      k_coefficients<float><<<grid_for(ne), kBlock, 0, stream>>>(
          op->ca.as<float>(), op->cb.as<float>(), op->eps_e.as<double>(), op->sig_e.as<double>(),
          ne, dt);
    YR_TRY_HIP(hipGetLastError());
  }
  if (!op->uniform_h) {
    YR_CALL(op->da.reserve(nh * es));
    YR_CALL(op->db.reserve(nh * es));
    if (dtype == YR_F64)
      k_coefficients<double><<<grid_for(nh), kBlock, 0, stream>>>(
          op->da.as<double>(), op->db.as<double>(), op->mu_h.as<double>(),
          op->sigm_h.as<double>(), nh, dt);
    else
      k_coefficients<float><<<grid_for(nh), kBlock, 0, stream>>>(
          op->da.as<float>(), op->db.as<float>(), op->mu_h.as<double>(), op->sigm_h.as<double>(),
          nh, dt);
    YR_TRY_HIP(hipGetLastError());
  }
  op->db_uniform = dt / kMu0;
  op->coef_dt = dt;
  op->coef_dtype = (int)dtype;
  return YR_OK;
}

int op_wait_idle(yr_operator* op) {
  if (op->busy_recorded) {
    YR_TRY_HIP(hipEventSynchronize(op->busy));
    op->busy_recorded = false;
  }
  return YR_OK;
}

int op_mark_busy(yr_operator* op, hipStream_t s) {
  if (!op->busy) YR_TRY_HIP(hipEventCreateWithFlags(&op->busy, hipEventDisableTiming));
  YR_TRY_HIP(hipEventRecord(op->busy, s));
  op->busy_recorded = true;
  return YR_OK;
}

int resolve_ports(const yr_operator* op, const yr_ports* ports, std::vector<PortEntry>& out,
                  int block_threads) {
  out.clear();
  if (!ports || ports->n == 0) return YR_OK;
  YR_REQUIRE(ports->n > 0 && ports->offset && ports->sample && ports->weight, YR_EINVAL,
             "port list: null arrays");
  const std::vector<uint8_t>& em = op->emask_host;
  for (int p = 0; p < ports->n; ++p) {
    int b = ports->offset[p], e = ports->offset[p + 1];
    YR_REQUIRE(b >= 0 && e >= b, YR_EINVAL, "port list: bad offsets");
    for (int q = b; q < e; ++q) {
      int c = ports->sample[4 * q], i = ports->sample[4 * q + 1], j = ports->sample[4 * q + 2],
          k = ports->sample[4 * q + 3];
      YR_REQUIRE(c >= 0 && c <= 2 && e_valid(op->dim, c, i, j, k, op->nx, op->ny, op->nz),
                 YR_EINVAL, "port entry is not an electric unknown of the grid");
      int64_t t = ((int64_t)k * op->Y + j) * op->X + i;
      int64_t slot = (int64_t)e_slot(op->dim, c) * op->len + t;
      YR_REQUIRE(em[slot] == 1, YR_EINVAL, "port entry lies on a PEC object");
      PortEntry pe;
      pe.slot = slot;
      pe.port = p;
      pe.block = (int32_t)(t / block_threads);
      pe.w = ports->weight[q];
      out.push_back(pe);
    }
  }
  return YR_OK;
}

}  // namespace yr

using namespace yr;

extern "C" {

const char* yr_last_error(void) { return yr::g_last_error.c_str(); }

int yr_operator_create(const yr_grid* g, const yr_materials* mat, yr_operator** out) {
  YR_REQUIRE(g && out, YR_EINVAL, "null argument");
  *out = nullptr;
  YR_REQUIRE(g->dim == 2 || g->dim == 3, YR_EINVAL, "dim must be 2 or 3");
  YR_REQUIRE(g->nx >= 2 && g->ny >= 2 && g->nz >= 1, YR_EINVAL, "grid needs >= 2 cells per axis");
  YR_REQUIRE(g->dim == 3 || g->nz == 1, YR_EINVAL, "2-D grids have nz = 1");
  YR_REQUIRE(g->dim == 2 || g->nz >= 2, YR_EINVAL, "3-D grids need nz >= 2");
  YR_REQUIRE(g->dx && g->dy && (g->dim == 2 || g->dz), YR_EINVAL, "null spacing array");
  std::unique_ptr<yr_operator> op(new (std::nothrow) yr_operator());
  YR_REQUIRE(op, YR_ENOMEM, "host allocation failed");
  op->dim = g->dim;
  op->nx = g->nx;
  op->ny = g->ny;
  op->nz = g->nz;
  op->X = g->nx + 1;
  op->Y = g->ny + 1;
  op->Z = g->dim == 3 ? g->nz + 1 : 1;
  op->len = (int64_t)op->X * op->Y * op->Z;
  YR_REQUIRE((int64_t)op->X * op->Y < ((int64_t)1 << 31), YR_EINVAL,
             "an x-y plane of the padded box exceeds 2^31 positions");
  op->ne_slots = g->dim == 3 ? 3 : 1;
  op->nh_slots = g->dim == 3 ? 3 : 2;
  const double* sp[3] = {g->dx, g->dy, g->dim == 3 ? g->dz : nullptr};
  const int n[3] = {g->nx, g->ny, g->nz};
  const int N[3] = {op->X, op->Y, op->Z};
  double hmin[3] = {1e300, 1e300, 1e300};
  for (int a = 0; a < 3; ++a) {
    op->hp[a].assign(N[a], 0.0);
    op->hd[a].assign(N[a], 0.0);
    if (a == 2 && g->dim == 2) {  // per unit length along z
      op->hp[2][0] = 1.0;
      op->hd[2][0] = 1.0;
      continue;
    }
    for (int c = 0; c < n[a]; ++c) {
      YR_REQUIRE(std::isfinite(sp[a][c]) && sp[a][c] > 0, YR_EINVAL, "spacings must be > 0");
      op->hp[a][c] = sp[a][c];
      hmin[a] = std::min(hmin[a], sp[a][c]);
    }
    for (int m = 0; m <= n[a]; ++m) {
      double l = m > 0 ? sp[a][m - 1] : 0.0, r = m < n[a] ? sp[a][m] : 0.0;
      op->hd[a][m] = 0.5 * (l + r);
    }
  }
  double s = 1.0 / (hmin[0] * hmin[0]) + 1.0 / (hmin[1] * hmin[1]);
  if (g->dim == 3) s += 1.0 / (hmin[2] * hmin[2]);
  op->dt_max = 1.0 / (kC0 * std::sqrt(s));  // eq. (CFL)
  op->v0 = g->dx[0] * g->dy[0] * (g->dim == 3 ? g->dz[0] : 1.0);

  YR_CALL(upload_axes<double>(op.get(), op->axes64));
  YR_CALL(upload_axes<float>(op.get(), op->axes32));

  int64_t ne = op->ne_slots * op->len, nh = op->nh_slots * op->len;
  YR_CALL(op->eps_e.reserve(ne * 8));
  YR_CALL(op->sig_e.reserve(ne * 8));
  YR_CALL(op->emask.reserve(ne));
  YR_CALL(op->mu_h.reserve(nh * 8));
  YR_CALL(op->sigm_h.reserve(nh * 8));
  YR_CALL(op->hmask.reserve(nh));
  YR_TRY_HIP(hipMemset(op->emask.p, 0, ne));

  // PEC objects
  std::vector<int64_t> pec_slots;
  if (mat && mat->n_pec > 0) {
    YR_REQUIRE(mat->pec, YR_EINVAL, "n_pec > 0 with null pec list");
    for (int64_t q = 0; q < mat->n_pec; ++q) {
      int c = mat->pec[4 * q], i = mat->pec[4 * q + 1], j = mat->pec[4 * q + 2],
          k = mat->pec[4 * q + 3];
      YR_REQUIRE(c >= 0 && c <= 2 && i >= 0 && i < op->X && j >= 0 && j < op->Y && k >= 0 &&
                     k < op->Z && (g->dim == 3 || c == 2),
                 YR_EINVAL, "PEC entry outside the grid");
      int64_t t = ((int64_t)k * op->Y + j) * op->X + i;
      pec_slots.push_back((int64_t)e_slot(g->dim, c) * op->len + t);
    }
    DevBuf d;
    YR_CALL(d.reserve(pec_slots.size() * 8));
    YR_TRY_HIP(hipMemcpy(d.p, pec_slots.data(), pec_slots.size() * 8, hipMemcpyHostToDevice));
    k_mark_pec<<<grid_for(pec_slots.size()), kBlock>>>(op->emask.as<uint8_t>(), d.as<int64_t>(),
                                                       (int64_t)pec_slots.size());
    YR_TRY_HIP(hipGetLastError());
    YR_TRY_HIP(hipDeviceSynchronize());
  }

  // per-cell tables
  int64_t ncell = (int64_t)g->nx * g->ny * g->nz;
  DevBuf cells[4];
  const double* src[4] = {mat ? mat->eps_r : nullptr, mat ? mat->sigma_e : nullptr,
                          mat ? mat->mu_r : nullptr, mat ? mat->sigma_m : nullptr};
  const double* dev[4] = {nullptr, nullptr, nullptr, nullptr};
  for (int a = 0; a < 4; ++a) {
    if (!src[a]) continue;
    for (int64_t c = 0; c < ncell; ++c)
      YR_REQUIRE(std::isfinite(src[a][c]) && (a % 2 == 0 ? src[a][c] > 0 : src[a][c] >= 0),
                 YR_EINVAL, "materials: eps_r, mu_r > 0 and conductivities >= 0 required");
    YR_CALL(cells[a].reserve(ncell * 8));
    YR_TRY_HIP(hipMemcpy(cells[a].p, src[a], ncell * 8, hipMemcpyHostToDevice));
    dev[a] = cells[a].as<double>();
  }
  op->lossless_e = true;
  if (src[1])
    for (int64_t c = 0; c < ncell && op->lossless_e; ++c) op->lossless_e = src[1][c] == 0.0;
  op->uniform_h = true;
  if (src[2])
    for (int64_t c = 0; c < ncell && op->uniform_h; ++c) op->uniform_h = src[2][c] == 1.0;
  if (src[3])
    for (int64_t c = 0; c < ncell && op->uniform_h; ++c) op->uniform_h = src[3][c] == 0.0;
  CellTables ct{dev[0], dev[1], dev[2], dev[3]};
  Axes<double> ax = op->axes<double>();
  k_average_e<<<grid_for(ne), kBlock>>>(op->eps_e.as<double>(), op->sig_e.as<double>(),
                                        op->emask.as<uint8_t>(), ct, ax, g->dim, g->nx, g->ny,
                                        g->nz, op->X, op->Y, op->len, op->ne_slots, kEps0);
  YR_TRY_HIP(hipGetLastError());
  k_average_h<<<grid_for(nh), kBlock>>>(op->mu_h.as<double>(), op->sigm_h.as<double>(),
                                        op->hmask.as<uint8_t>(), ct, ax, g->dim, g->nx, g->ny,
                                        g->nz, op->X, op->Y, op->len, op->nh_slots, kMu0);
  YR_TRY_HIP(hipGetLastError());
  YR_TRY_HIP(hipDeviceSynchronize());

  // unknown counts and the host mask copy
  op->emask_host.resize(ne);
  YR_TRY_HIP(hipMemcpy(op->emask_host.data(), op->emask.p, ne, hipMemcpyDeviceToHost));
  std::vector<uint8_t> hm(nh);
  YR_TRY_HIP(hipMemcpy(hm.data(), op->hmask.p, nh, hipMemcpyDeviceToHost));
  op->n_e = std::count(op->emask_host.begin(), op->emask_host.end(), (uint8_t)1);
  op->n_h = std::count(hm.begin(), hm.end(), (uint8_t)1);
  *out = op.release();
  return YR_OK;
}

void yr_operator_destroy(yr_operator* op) { delete op; }

int yr_operator_info(const yr_operator* op, int64_t* len, int64_t* n_e, int64_t* n_h,
                     double* dt_max) {
  YR_REQUIRE(op, YR_EINVAL, "null operator");
  if (len) *len = op->len;
  if (n_e) *n_e = op->n_e;
  if (n_h) *n_h = op->n_h;
  if (dt_max) *dt_max = op->dt_max;
  return YR_OK;
}

}  // extern "C"
