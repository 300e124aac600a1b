// Host runtime of the 3-D solver: parameter checks, FP64 plan construction
// (medium diagonals, PML, k-space symbols, FFT plans and twiddles, trilinear
// sensor taps), work buffers per batch size, the forward / adjoint time loops
// with optional hipGraph replay, and the qpat3d_* entry points of qpat.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/qpat.h"
#include "k3d_internal.hpp"

namespace qpat {
qpat_status set_error(qpat_status s, const std::string& msg);
}

using namespace qpat3;
using qpat::set_error;

namespace {

#define H3CHK(expr)                                                                       \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return set_error(e_ == hipErrorOutOfMemory ? QPAT_E_OOM : QPAT_E_HIP,                \
                       std::string(#expr) + ": " + hipGetErrorString(e_));                \
  } while (0)
#define S3CHK(expr)               \
  do {                            \
    qpat_status s_ = (expr);      \
    if (s_ != QPAT_OK) return s_; \
  } while (0)
#define L3CHK(expr)                   \
  do {                                \
    hipError_t e_ = (expr);           \
    if (e_ != hipSuccess) return e_;  \
  } while (0)

bool is_prime(int p) {
  if (p < 2) return false;
  for (int d = 2; d * d <= p; ++d)
    if (p % d == 0) return false;
  return true;
}

// Stage radices of an axis of length n: 8s, then a 4 or 2, then 3s, 5s, 7s,
// then any larger prime factors (direct DFT stages).
bool axis_plan(int n, AxisPlan* P) {
  if (n < 4 || n > kMaxN) return false;
  std::vector<int> r;
  int m = n, a = 0;
  while (m % 2 == 0) {
    m /= 2;
    ++a;
  }
  for (int i = 0; i < a / 3; ++i) r.push_back(8);
  if (a % 3 == 1) r.push_back(2);
  if (a % 3 == 2) r.push_back(4);
  for (int p : {3, 5, 7})
    while (m % p == 0) {
      m /= p;
      r.push_back(p);
    }
  for (int p = 11; m > 1; ++p)
    while (m % p == 0) {
      if (!is_prime(p)) return false;
      m /= p;
      r.push_back(p);
    }
  if (int(r.size()) > kMaxStages) return false;
  P->n = n;
  P->nst = int(r.size());
  for (int i = 0; i < kMaxStages; ++i) P->r[i] = i < P->nst ? r[i] : 1;
  return true;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

double alpha0_np(double a_db, double y) {
  return a_db * 100.0 / (20.0 * std::log10(std::exp(1.0))) * std::pow(1e-6 / (2.0 * M_PI), y);
}

double stability_limit3(double cmax, double c_ref, double dx, double dy, double dz) {
  if (c_ref >= cmax) return INFINITY;
  const double kmax = std::sqrt(std::pow(M_PI / dx, 2) + std::pow(M_PI / dy, 2) + std::pow(M_PI / dz, 2));
  return 2.0 * std::asin(c_ref / cmax) / (c_ref * kmax);
}

bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

bool tiles_ok(const qpat_params3d& p, int rt, int ct, int rthr = 256, int pthr = 256) {
  if (rt < 2 || rt > 64 || (rt & 1) || ct < 1 || ct > p.nx / 2 + 1) return false;
  if (!pow2_in(rthr, 64, kRowMax) || !pow2_in(pthr, 64, kPlaneMax)) return false;
  return row3_lds(p.nx, rt) <= kMaxLds && plane3_lds(p.ny, p.nz, ct) <= kMaxLds;
}

qpat_status validate3(const qpat_params3d* p) {
  if (!p) return set_error(QPAT_E_INVALID, "params is NULL");
  AxisPlan a;
  if (!axis_plan(p->nx, &a) || !axis_plan(p->ny, &a) || !axis_plan(p->nz, &a))
    return set_error(QPAT_E_UNSUPPORTED, "nx, ny, nz must be in [4, 128]");
  if (p->ny * p->nz > 4096) return set_error(QPAT_E_UNSUPPORTED, "ny * nz must be at most 4096");
  if (!finite_pos(p->dx) || !finite_pos(p->dy) || !finite_pos(p->dz) || !finite_pos(p->dt))
    return set_error(QPAT_E_INVALID, "dx, dy, dz, dt must be finite and > 0");
  if (p->nt < 1) return set_error(QPAT_E_INVALID, "nt must be >= 1");
  if (p->ns < 0) return set_error(QPAT_E_INVALID, "ns must be >= 0");
  if (int64_t(p->nt) * p->ns >= (int64_t(1) << 28))
    return set_error(QPAT_E_UNSUPPORTED, "nt * ns must be below 2^28");
  if (!finite_pos(p->c_ref)) return set_error(QPAT_E_INVALID, "c_ref must be finite and > 0");
  if (p->pml_size < 0 || 2 * p->pml_size >= std::min(p->nx, std::min(p->ny, p->nz)))
    return set_error(QPAT_E_INVALID, "pml_size must be in [0, min(nx, ny, nz)/2)");
  if (!(std::isfinite(p->pml_alpha) && p->pml_alpha >= 0.0))
    return set_error(QPAT_E_INVALID, "pml_alpha must be finite and >= 0");
  if (!(std::isfinite(p->alpha0_db) && p->alpha0_db >= 0.0))
    return set_error(QPAT_E_INVALID, "alpha0_db must be finite and >= 0");
  if (p->alpha0_db > 0.0) {
    if (!(std::isfinite(p->y) && p->y > 0.0 && p->y <= 3.0))
      return set_error(QPAT_E_INVALID, "y must be in (0, 3]");
    if (std::fabs(p->y - std::round(p->y)) < 1e-12 && (int(std::round(p->y)) % 2) == 1)
      return set_error(QPAT_E_INVALID, "odd integer y makes tan(pi y / 2) singular");
  }
  if (p->ns > 0 && !p->sensor_xyz) return set_error(QPAT_E_INVALID, "sensor_xyz is NULL");
  for (int s = 0; s < p->ns; ++s) {
    const double u = p->sensor_xyz[3 * s] / p->dx + p->nx / 2.0;
    const double v = p->sensor_xyz[3 * s + 1] / p->dy + p->ny / 2.0;
    const double w = p->sensor_xyz[3 * s + 2] / p->dz + p->nz / 2.0;
    if (!(u >= 0.0 && u <= p->nx - 1 && v >= 0.0 && v <= p->ny - 1 && w >= 0.0 && w <= p->nz - 1))
      return set_error(QPAT_E_INVALID, "sensor " + std::to_string(s) + " lies outside the node grid");
  }
  return QPAT_OK;
}

// Trilinear taps: four line entries per sensor (slots (z0,y0), (z0,y1),
// (z1,y0), (z1,y1)), sorted by line.
void build_taps3(const qpat_params3d& p, std::vector<Tap3>& taps, std::vector<int>& off) {
  const int nl = p.ny * p.nz;
  std::vector<std::vector<Tap3>> byline(nl);
  for (int s = 0; s < p.ns; ++s) {
    const double u = p.sensor_xyz[3 * s] / p.dx + p.nx / 2.0;
    const double v = p.sensor_xyz[3 * s + 1] / p.dy + p.ny / 2.0;
    const double w = p.sensor_xyz[3 * s + 2] / p.dz + p.nz / 2.0;
    const int i0 = int(std::floor(u)), j0 = int(std::floor(v)), k0 = int(std::floor(w));
    const double fx = u - i0, fy = v - j0, fz = w - k0;
    const int i1 = std::min(i0 + 1, p.nx - 1), j1 = std::min(j0 + 1, p.ny - 1), k1 = std::min(k0 + 1, p.nz - 1);
    const int ks[2] = {k0, k1}, js[2] = {j0, j1};
    const double wz[2] = {1.0 - fz, fz}, wy[2] = {1.0 - fy, fy};
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        const int line = ks[a] * p.ny + js[b];
        const double ww = wz[a] * wy[b];
        byline[line].push_back(Tap3{s, 2 * a + b, line, i0, i1, float(ww * (1.0 - fx)), float(ww * fx), 0});
      }
  }
  taps.clear();
  off.assign(nl + 1, 0);
  for (int l = 0; l < nl; ++l) {
    off[l] = int(taps.size());
    for (const Tap3& t : byline[l]) taps.push_back(t);
  }
  off[nl] = int(taps.size());
}

// The scatter list of M^T: every (node, sensor, weight) of the taps grouped by
// node, nodes sorted by (line, ix), with per-line offsets into the nodes.
void build_scatter3(const qpat_params3d& p, const std::vector<Tap3>& taps, std::vector<int>& noff,
                    std::vector<ScatterNode>& nodes, std::vector<ScatterEntry>& entries) {
  const int nl = p.ny * p.nz;
  std::map<std::pair<int, int>, std::vector<ScatterEntry>> by;
  for (const Tap3& t : taps) {
    by[{t.line, t.ixl}].push_back(ScatterEntry{t.s, t.wl});
    by[{t.line, t.ixr}].push_back(ScatterEntry{t.s, t.wr});
  }
  nodes.clear();
  entries.clear();
  noff.assign(nl + 1, 0);
  for (const auto& kv : by) {
    const int e0 = int(entries.size());
    for (const ScatterEntry& e : kv.second) entries.push_back(e);
    nodes.push_back(ScatterNode{kv.first.first, kv.first.second, e0, int(entries.size())});
  }
  // nodes are in (line, ix) order; offsets per line
  size_t k = 0;
  for (int l = 0; l <= nl; ++l) {
    while (k < nodes.size() && nodes[k].line < l) ++k;
    noff[l] = int(k);
  }
}

struct Carver {
  size_t off = 0;
  template <typename T>
  size_t take(size_t count) {
    off = (off + 255) & ~size_t(255);
    const size_t o = off;
    off += count * sizeof(T);
    return o;
  }
};

// Launch state for one batch size: the items' work buffers are equally
// spaced, so every launch carries the medium and the first item's buffers.
struct Exec3 {
  Launch3 L{};
  IO3* d_io = nullptr;
  IO3* h_io = nullptr;
  hipEvent_t ev = nullptr;
  bool ev_used = false;
  int row_ntile = 0, row_chunk = 0, pl_ntile = 0, pl_chunk = 0;
  std::map<int, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
  ~Exec3() {
    for (auto& g : graphs) {
      if (g.second.second) (void)hipGraphExecDestroy(g.second.second);
      if (g.second.first) (void)hipGraphDestroy(g.second.first);
    }
    if (d_io) (void)hipFree(d_io);
    if (h_io) (void)hipHostFree(h_io);
    if (ev) (void)hipEventDestroy(ev);
  }
};

}  // namespace

struct qpat_plan3d_s {
  qpat_params3d prm{};
  std::vector<double> sensors;
  Medium3 med{};
  void* d_med = nullptr;
  void* d_work = nullptr;
  int cap = 0;
  size_t item_bytes = 0;
  Work3 w0{};
  std::vector<float*> datas;
  std::map<int, std::unique_ptr<Exec3>> execs;
  bool graph = false;
  bool auto_shape = true;   // rows and thread counts chosen per batch size until set_tiles
};

namespace {

qpat_status plan3_build(qpat_plan3d P, const double* c0, const double* rho0) {
  const qpat_params3d& p = P->prm;
  const int nx = p.nx, ny = p.ny, nz = p.nz, nxh1 = nx / 2 + 1, nl = ny * nz;
  const size_t N = size_t(nx) * nl;
  const double dx = p.dx, dy = p.dy, dz = p.dz, dt = p.dt;
  double cmax = 0.0;
  for (size_t i = 0; i < N; ++i) {
    if (!finite_pos(c0[i])) return set_error(QPAT_E_INVALID, "c0 must be finite and > 0 everywhere");
    if (!finite_pos(rho0[i])) return set_error(QPAT_E_INVALID, "rho0 must be finite and > 0 everywhere");
    cmax = std::max(cmax, c0[i]);
  }
  const double lim = stability_limit3(cmax, p.c_ref, dx, dy, dz);
  if (dt > lim)
    return set_error(QPAT_E_UNSTABLE, "dt exceeds the k-space stability bound " + std::to_string(lim) +
                                          " for c_ref < max(c0)");
  const bool lossy = p.alpha0_db > 0.0;
  const double a0 = lossy ? alpha0_np(p.alpha0_db, p.y) : 0.0;
  const double tn = lossy ? std::tan(M_PI * p.y / 2.0) : 0.0;

  std::vector<float> c2(N), c2eta(N), c2tau(N), r0(N), bx(N), by(N), bz(N);
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const size_t q = (size_t(k) * ny + j) * nx + i;
        const double c = c0[q];
        c2[q] = float(c * c);
        // eq Twelve: tau = -2 a0 c^(y-1), eta = 2 a0 c^y tan(pi y / 2)
        c2eta[q] = lossy ? float(c * c * 2.0 * a0 * std::pow(c, p.y) * tn) : 0.f;
        c2tau[q] = lossy ? float(c * c * -2.0 * a0 * std::pow(c, p.y - 1.0)) : 0.f;
        r0[q] = float(rho0[q]);
        const double rx = 0.5 * (rho0[q] + rho0[(size_t(k) * ny + j) * nx + (i + 1) % nx]);
        const double ry = 0.5 * (rho0[q] + rho0[(size_t(k) * ny + (j + 1) % ny) * nx + i]);
        const double rz = 0.5 * (rho0[q] + rho0[(size_t((k + 1) % nz) * ny + j) * nx + i]);
        bx[q] = float(dt / rx);
        by[q] = float(dt / ry);
        bz[q] = float(dt / rz);
      }
  // PML (eq dis-pml) inside the grid, 4th-power profile, velocities at half nodes
  auto sigma = [&](double pos, int n, double d) {
    const int L = p.pml_size;
    if (L <= 0) return 0.0;
    const double xi = std::max(0.0, std::max(L - pos, pos - (n - 1 - L)));
    return p.pml_alpha * (p.c_ref / d) * std::pow(xi / L, 4);
  };
  auto pml = [&](int n, double d, std::vector<float>& av, std::vector<float>& ar) {
    av.resize(n);
    ar.resize(n);
    for (int i = 0; i < n; ++i) {
      ar[i] = float(std::exp(-sigma(i, n, d) * dt / 2.0));
      av[i] = float(std::exp(-sigma(i + 0.5, n, d) * dt / 2.0));
    }
  };
  std::vector<float> avx, arx, avy, ary, avz, arz;
  pml(nx, dx, avx, arx);
  pml(ny, dy, avy, ary);
  pml(nz, dz, avz, arz);
  // wavenumbers in numpy's order; the Nyquist bin of an even axis is -pi/d,
  // where the staggered symbol i k e^{+-i k d/2} is real
  auto kval = [](int idx, int n, double d) {
    const int f = idx < (n + 1) / 2 ? idx : idx - n;
    return 2.0 * M_PI * f / (n * d);
  };
  auto dsym = [](double k, double d, int sgn, bool nyq) {
    const double th = sgn * k * d / 2.0;
    if (nyq) return make_float2(float(-k * std::sin(th)), 0.f);
    return make_float2(float(-k * std::sin(th)), float(k * std::cos(th)));
  };
  auto sym1 = [&](int n, int count, double d, std::vector<float2>& pl, std::vector<float2>& mi) {
    pl.resize(count);
    mi.resize(count);
    for (int i = 0; i < count; ++i) {
      const double k = kval(i, n, d);
      const bool nyq = (n % 2 == 0) && i == n / 2;
      pl[i] = dsym(k, d, +1, nyq);
      mi[i] = dsym(k, d, -1, nyq);
    }
  };
  std::vector<float2> dxp, dxm, dyp, dym, dzp, dzm;
  sym1(nx, nxh1, dx, dxp, dxm);
  sym1(ny, ny, dy, dyp, dym);
  sym1(nz, nz, dz, dzp, dzm);
  const size_t nk = size_t(nl) * nxh1;
  std::vector<float> kap(nk), ldis(nk), labs(nk);
  const double inv = 1.0 / double(N);
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nxh1; ++i) {
        const double kx = kval(i, nx, dx), ky = kval(j, ny, dy), kz = kval(k, nz, dz);
        const double K = std::sqrt(kx * kx + ky * ky + kz * kz);
        const double arg = p.c_ref * K * dt / 2.0;
        const double kp = arg == 0.0 ? 1.0 : std::sin(arg) / arg;
        const size_t t = size_t(i) * nl + size_t(k) * ny + j;   // [column][line]
        kap[t] = float(kp * inv);
        ldis[t] = (K == 0.0 || !lossy) ? 0.f : float(std::pow(K, p.y - 1.0) * inv);
        labs[t] = (K == 0.0 || !lossy) ? 0.f : float(std::pow(K, p.y - 2.0) * inv);
      }
  auto twid = [](int n) {
    std::vector<float2> t(n);
    for (int m = 0; m < n; ++m) {
      const double a = -2.0 * M_PI * double(m) / double(n);
      t[m] = make_float2(float(std::cos(a)), float(std::sin(a)));
    }
    return t;
  };
  const std::vector<float2> twx = twid(nx), twy = twid(ny), twz = twid(nz);
  std::vector<Tap3> taps;
  std::vector<int> toff;
  build_taps3(p, taps, toff);
  std::vector<int> noff;
  std::vector<ScatterNode> nodes;
  std::vector<ScatterEntry> entries;
  build_scatter3(p, taps, noff, nodes, entries);
  if (taps.empty()) taps.push_back(Tap3{});
  if (nodes.empty()) nodes.push_back(ScatterNode{});
  if (entries.empty()) entries.push_back(ScatterEntry{});

  {
    const hipError_t e = k3d_allow_lds(kMaxLds);
    if (e != hipSuccess) return set_error(QPAT_E_HIP, std::string("LDS attribute: ") + hipGetErrorString(e));
  }
  Carver cv;
  const size_t o_c2 = cv.take<float>(N), o_ce = cv.take<float>(N), o_ct = cv.take<float>(N);
  const size_t o_r0 = cv.take<float>(N), o_bx = cv.take<float>(N), o_by = cv.take<float>(N),
               o_bz = cv.take<float>(N);
  const size_t o_avx = cv.take<float>(nx), o_arx = cv.take<float>(nx), o_avy = cv.take<float>(ny),
               o_ary = cv.take<float>(ny), o_avz = cv.take<float>(nz), o_arz = cv.take<float>(nz);
  const size_t o_dxp = cv.take<float2>(nxh1), o_dxm = cv.take<float2>(nxh1), o_dyp = cv.take<float2>(ny),
               o_dym = cv.take<float2>(ny), o_dzp = cv.take<float2>(nz), o_dzm = cv.take<float2>(nz);
  const size_t o_kap = cv.take<float>(nk), o_ldis = cv.take<float>(nk), o_labs = cv.take<float>(nk);
  const size_t o_twx = cv.take<float2>(nx), o_twy = cv.take<float2>(ny), o_twz = cv.take<float2>(nz);
  const size_t o_toff = cv.take<int>(toff.size()), o_taps = cv.take<Tap3>(taps.size());
  const size_t o_noff = cv.take<int>(noff.size()), o_nodes = cv.take<ScatterNode>(nodes.size()),
               o_ent = cv.take<ScatterEntry>(entries.size());
  std::vector<char> host(cv.off, 0);
  auto put = [&](size_t o, const void* src, size_t bytes) { std::memcpy(host.data() + o, src, bytes); };
  put(o_c2, c2.data(), N * 4);
  put(o_ce, c2eta.data(), N * 4);
  put(o_ct, c2tau.data(), N * 4);
  put(o_r0, r0.data(), N * 4);
  put(o_bx, bx.data(), N * 4);
  put(o_by, by.data(), N * 4);
  put(o_bz, bz.data(), N * 4);
  put(o_avx, avx.data(), nx * 4);
  put(o_arx, arx.data(), nx * 4);
  put(o_avy, avy.data(), ny * 4);
  put(o_ary, ary.data(), ny * 4);
  put(o_avz, avz.data(), nz * 4);
  put(o_arz, arz.data(), nz * 4);
  put(o_dxp, dxp.data(), nxh1 * 8);
  put(o_dxm, dxm.data(), nxh1 * 8);
  put(o_dyp, dyp.data(), ny * 8);
  put(o_dym, dym.data(), ny * 8);
  put(o_dzp, dzp.data(), nz * 8);
  put(o_dzm, dzm.data(), nz * 8);
  put(o_kap, kap.data(), nk * 4);
  put(o_ldis, ldis.data(), nk * 4);
  put(o_labs, labs.data(), nk * 4);
  put(o_twx, twx.data(), nx * 8);
  put(o_twy, twy.data(), ny * 8);
  put(o_twz, twz.data(), nz * 8);
  put(o_toff, toff.data(), toff.size() * 4);
  put(o_taps, taps.data(), taps.size() * sizeof(Tap3));
  put(o_noff, noff.data(), noff.size() * 4);
  put(o_nodes, nodes.data(), nodes.size() * sizeof(ScatterNode));
  put(o_ent, entries.data(), entries.size() * sizeof(ScatterEntry));
  char* d = nullptr;
  H3CHK(hipMalloc(&d, cv.off));
  P->d_med = d;
  H3CHK(hipMemcpy(d, host.data(), cv.off, hipMemcpyHostToDevice));

  Medium3& M = P->med;
  M.nx = nx;
  M.ny = ny;
  M.nz = nz;
  M.nxh1 = nxh1;
  M.nlines = nl;
  M.nt = p.nt;
  M.ns = p.ns;
  M.lossy = lossy ? 1 : 0;
  M.dt = float(dt);
  axis_plan(nx, &M.px);
  axis_plan(ny, &M.py);
  axis_plan(nz, &M.pz);
  M.c2 = (const float*)(d + o_c2);
  M.c2eta = (const float*)(d + o_ce);
  M.c2tau = (const float*)(d + o_ct);
  M.rho0 = (const float*)(d + o_r0);
  M.bx = (const float*)(d + o_bx);
  M.by = (const float*)(d + o_by);
  M.bz = (const float*)(d + o_bz);
  M.avx = (const float*)(d + o_avx);
  M.arx = (const float*)(d + o_arx);
  M.avy = (const float*)(d + o_avy);
  M.ary = (const float*)(d + o_ary);
  M.avz = (const float*)(d + o_avz);
  M.arz = (const float*)(d + o_arz);
  M.dxp = (const float2*)(d + o_dxp);
  M.dxm = (const float2*)(d + o_dxm);
  M.dyp = (const float2*)(d + o_dyp);
  M.dym = (const float2*)(d + o_dym);
  M.dzp = (const float2*)(d + o_dzp);
  M.dzm = (const float2*)(d + o_dzm);
  M.kap = (const float*)(d + o_kap);
  M.ldis = (const float*)(d + o_ldis);
  M.labs = (const float*)(d + o_labs);
  M.twx = (const float2*)(d + o_twx);
  M.twy = (const float2*)(d + o_twy);
  M.twz = (const float2*)(d + o_twz);
  M.tap_off = (const int*)(d + o_toff);
  M.taps = (const Tap3*)(d + o_taps);
  M.node_off = (const int*)(d + o_noff);
  M.nodes = (const ScatterNode*)(d + o_nodes);
  M.entries = (const ScatterEntry*)(d + o_ent);
  // default shape: 16 lines per row block (fewer when nx is long), one
  // spectrum column per plane block
  int rt = 16;
  while (rt > 2 && !tiles_ok(p, rt, 1)) rt -= 2;
  if (!tiles_ok(p, rt, 1)) return set_error(QPAT_E_UNSUPPORTED, "grid too large for the LDS of one block");
  M.rt = rt;
  M.ct = 1;
  M.ctiles = nxh1;
  M.rthr = 256;
  M.pthr = 512;
  return QPAT_OK;
}

// Work buffers of `count` vectors: 7 fields, 4 half spectra, sensor partials
// and a data buffer for jtjv.
qpat_status reserve3(qpat_plan3d P, int count) {
  if (count <= P->cap) return QPAT_OK;
  if (P->d_work) {
    H3CHK(hipDeviceSynchronize());
    H3CHK(hipFree(P->d_work));
    P->d_work = nullptr;
  }
  P->execs.clear();
  P->cap = 0;
  const Medium3& M = P->med;
  const size_t N = size_t(M.nx) * M.nlines;
  // spectra sized for any column tile: ctiles * ct < nxh1 + ct <= 2 nxh1
  const size_t specN = size_t(2 * M.nxh1) * M.nlines;
  const size_t nd = size_t(M.nt) * M.ns;
  Carver cv;
  const size_t o_f = cv.take<float>(7 * N), o_s = cv.take<float2>(4 * specN), o_p = cv.take<float>(4 * nd + 1),
               o_d = cv.take<float>(nd + 1);
  const size_t per = (cv.off + 255) & ~size_t(255);
  char* d = nullptr;
  H3CHK(hipMalloc(&d, per * count));
  P->d_work = d;
  P->item_bytes = per;
  P->w0.f = (float*)(d + o_f);
  P->w0.s = (float2*)(d + o_s);
  P->w0.part = (float*)(d + o_p);
  P->datas.clear();
  for (int i = 0; i < count; ++i) P->datas.push_back((float*)(d + per * i + o_d));
  P->cap = count;
  return QPAT_OK;
}

// Launch shape for b vectors on automatic shape: 8-line row blocks while
// 16-line ones would give fewer than two blocks per CU, and 1024-thread plane
// blocks while the plane launches give at most one block per CU (more lines
// and threads per block only lengthen each block's chain of dependent FFT
// stages then); 16 lines (the plan's rows) and 512 threads otherwise.
void auto_shape3(const Medium3& base, int b, Medium3& m) {
  m.rt = size_t(b) * ((base.nlines + base.rt - 1) / base.rt) < size_t(2) * kCus ? std::min(8, base.rt) : base.rt;
  m.rthr = 256;
  m.pthr = size_t(3) * b * base.ctiles <= size_t(kCus) ? 1024 : 512;
}

qpat_status exec3(qpat_plan3d P, int b, Exec3** out) {
  S3CHK(reserve3(P, b));
  auto it = P->execs.find(b);
  if (it == P->execs.end()) {
    std::unique_ptr<Exec3> E(new Exec3());
    E->L.m = P->med;
    if (P->auto_shape) auto_shape3(P->med, b, E->L.m);
    E->L.w0 = P->w0;
    E->L.wstride = (long long)P->item_bytes;
    E->L.nitems = b;
    H3CHK(hipMalloc(&E->d_io, sizeof(IO3) * b));
    H3CHK(hipHostMalloc(&E->h_io, sizeof(IO3) * b, hipHostMallocDefault));
    H3CHK(hipEventCreateWithFlags(&E->ev, hipEventDisableTiming));
    E->L.io = E->d_io;
    const Medium3& M = E->L.m;
    E->row_ntile = (M.nlines + M.rt - 1) / M.rt;
    E->pl_ntile = M.ctiles;
    E->row_chunk = (b * E->row_ntile + kXcds - 1) / kXcds;
    E->pl_chunk = (b * E->pl_ntile + kXcds - 1) / kXcds;
    it = P->execs.emplace(b, std::move(E)).first;
  }
  *out = it->second.get();
  return QPAT_OK;
}

qpat_status set_io3(Exec3& E, const std::vector<IO3>& io, hipStream_t st) {
  if (E.ev_used) H3CHK(hipEventSynchronize(E.ev));
  std::memcpy(E.h_io, io.data(), sizeof(IO3) * io.size());
  H3CHK(hipMemcpyAsync(E.d_io, E.h_io, sizeof(IO3) * io.size(), hipMemcpyHostToDevice, st));
  H3CHK(hipEventRecord(E.ev, st));
  E.ev_used = true;
  return QPAT_OK;
}

hipError_t row3(Exec3& E, int mode, int n, hipStream_t st) {
  return launch_row3(mode, E.L, E.row_ntile, E.row_chunk, n, st);
}
hipError_t plane3(Exec3& E, int mode, int n, hipStream_t st, int code = 0) {
  const int ntile = E.pl_ntile * plane3_split(mode);
  const int chunk = (E.L.nitems * ntile + kXcds - 1) / kXcds;
  return launch_plane3(mode, code, E.L, ntile, chunk, n, st);
}

hipError_t seq_forward3(Exec3& E, hipStream_t st) {
  const bool lossy = E.L.m.lossy != 0;
  for (int n = -1; n <= E.L.m.nt - 2; ++n) {
    if (n > -1) {
      L3CHK(plane3(E, P3_GRADP1, n, st));
      L3CHK(row3(E, R3_F1, n, st));
      L3CHK(plane3(E, P3_GRADM2, n, st));
    }
    if (lossy) {
      L3CHK(row3(E, R3_F2, n, st));
      L3CHK(plane3(E, P3_FRAC, n, st));
      L3CHK(row3(E, R3_F3, n, st));
    } else {
      L3CHK(row3(E, R3_F2L, n, st));
    }
  }
  return launch_combine3(E.L, st);
}

hipError_t seq_adjoint3(Exec3& E, hipStream_t st) {
  const bool lossy = E.L.m.lossy != 0;
  for (int n = E.L.m.nt - 2; n >= -1; --n) {
    if (lossy) {
      L3CHK(row3(E, R3_A1, n, st));
      L3CHK(plane3(E, P3_FRAC, n, st));
      L3CHK(row3(E, R3_A2, n, st));
    } else {
      L3CHK(row3(E, R3_A1L, n, st));
    }
    if (n == -1) break;
    L3CHK(plane3(E, P3_GRADP2, n, st));
    L3CHK(row3(E, R3_A3, n, st));
    L3CHK(plane3(E, P3_GRADM2, n, st));   // the terms of the divergence, summed by the next row pass
  }
  return hipSuccess;
}

enum { OP3_FWD = 1, OP3_ADJ = 2 };

qpat_status run3(qpat_plan3d P, Exec3& E, int op, hipStream_t st) {
  auto body = [&](hipStream_t s) { return op == OP3_FWD ? seq_forward3(E, s) : seq_adjoint3(E, s); };
  if (!P->graph || st == nullptr) {
    const hipError_t e = body(st);
    if (e != hipSuccess) return set_error(QPAT_E_HIP, std::string("3-D launch: ") + hipGetErrorString(e));
    return QPAT_OK;
  }
  auto it = E.graphs.find(op);
  if (it == E.graphs.end()) {
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    H3CHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const hipError_t e = body(st);
    const hipError_t e2 = hipStreamEndCapture(st, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return set_error(QPAT_E_HIP, std::string("3-D graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    H3CHK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
    it = E.graphs.emplace(op, std::make_pair(g, ge)).first;
  }
  H3CHK(hipGraphLaunch(it->second.second, st));
  return QPAT_OK;
}

qpat_status check3(qpat_plan3d P, const void* a, const void* b, int batch) {
  if (!P) return set_error(QPAT_E_INVALID, "plan is NULL");
  if (!a || !b) return set_error(QPAT_E_INVALID, "input / output pointer is NULL");
  if (batch < 1 || batch > 4096) return set_error(QPAT_E_INVALID, "batch must be in [1, 4096]");
  return QPAT_OK;
}

size_t nfield(qpat_plan3d P) { return size_t(P->med.nx) * P->med.nlines; }
size_t ndata(qpat_plan3d P) { return size_t(P->med.nt) * P->med.ns; }

qpat_status fwd3(qpat_plan3d P, const float* p0, float* data, int batch, hipStream_t st, bool internal) {
  Exec3* E = nullptr;
  S3CHK(exec3(P, batch, &E));
  std::vector<IO3> io(batch);
  for (int i = 0; i < batch; ++i) io[i] = IO3{p0 + nfield(P) * i, internal ? P->datas[i] : data + ndata(P) * i};
  S3CHK(set_io3(*E, io, st));
  return run3(P, *E, OP3_FWD, st);
}

qpat_status adj3(qpat_plan3d P, const float* res, float* grad, int batch, hipStream_t st, bool internal) {
  Exec3* E = nullptr;
  S3CHK(exec3(P, batch, &E));
  std::vector<IO3> io(batch);
  for (int i = 0; i < batch; ++i) io[i] = IO3{internal ? P->datas[i] : res + ndata(P) * i, grad + nfield(P) * i};
  S3CHK(set_io3(*E, io, st));
  return run3(P, *E, OP3_ADJ, st);
}

}  // namespace

extern "C" {

qpat_status qpat3d_validate(const qpat_params3d* prm) { return validate3(prm); }

qpat_status qpat3d_plan_create(const qpat_params3d* prm, const double* c0, const double* rho0,
                               qpat_plan3d* out) {
  if (!out) return set_error(QPAT_E_INVALID, "out is NULL");
  *out = nullptr;
  S3CHK(validate3(prm));
  if (!c0 || !rho0) return set_error(QPAT_E_INVALID, "c0 / rho0 is NULL");
  qpat_plan3d P = new qpat_plan3d_s();
  P->prm = *prm;
  P->sensors.assign(prm->sensor_xyz, prm->sensor_xyz + 3 * size_t(prm->ns));
  P->prm.sensor_xyz = P->sensors.data();
  const qpat_status s = plan3_build(P, c0, rho0);
  if (s != QPAT_OK) {
    qpat3d_plan_destroy(P);
    return s;
  }
  *out = P;
  return QPAT_OK;
}

void qpat3d_plan_destroy(qpat_plan3d P) {
  if (!P) return;
  (void)hipDeviceSynchronize();
  P->execs.clear();
  if (P->d_work) (void)hipFree(P->d_work);
  if (P->d_med) (void)hipFree(P->d_med);
  delete P;
}

qpat_status qpat3d_forward(qpat_plan3d P, const float* p0, float* data, int32_t batch, qpat_stream stream) {
  S3CHK(check3(P, p0, data, batch));
  return fwd3(P, p0, data, batch, (hipStream_t)stream, false);
}

qpat_status qpat3d_adjoint(qpat_plan3d P, const float* res, float* grad, int32_t batch, qpat_stream stream) {
  S3CHK(check3(P, res, grad, batch));
  return adj3(P, res, grad, batch, (hipStream_t)stream, false);
}

qpat_status qpat3d_jtjv(qpat_plan3d P, const float* v, float* out, int32_t batch, qpat_stream stream) {
  S3CHK(check3(P, v, out, batch));
  S3CHK(fwd3(P, v, nullptr, batch, (hipStream_t)stream, true));
  return adj3(P, nullptr, out, batch, (hipStream_t)stream, true);
}

qpat_status qpat3d_apply(qpat_plan3d P, int32_t op, const float* in, float* out, int32_t batch,
                         qpat_stream stream) {
  S3CHK(check3(P, in, out, batch));
  if (op < 0 || op > OP_LABS) return set_error(QPAT_E_INVALID, "op must be in [0, 7]");
  hipStream_t st = (hipStream_t)stream;
  Exec3* E = nullptr;
  S3CHK(exec3(P, batch, &E));
  std::vector<IO3> io(batch);
  for (int i = 0; i < batch; ++i) io[i] = IO3{in + nfield(P) * i, out + nfield(P) * i};
  S3CHK(set_io3(*E, io, st));
  hipError_t e = row3(*E, R3_FWD1, 0, st);
  if (e == hipSuccess) e = plane3(*E, P3_APPLY, 0, st, op);
  if (e == hipSuccess) e = row3(*E, R3_INV1, 0, st);
  if (e != hipSuccess) return set_error(QPAT_E_HIP, std::string("3-D apply: ") + hipGetErrorString(e));
  return QPAT_OK;
}

qpat_status qpat3d_set_tiles(qpat_plan3d P, int32_t rows, int32_t cols, int32_t row_threads,
                             int32_t plane_threads) {
  if (!P) return set_error(QPAT_E_INVALID, "plan is NULL");
  if (!tiles_ok(P->prm, rows, cols, row_threads, plane_threads))
    return set_error(QPAT_E_INVALID, "tiles: rows even in [2, 64], cols in [1, nx/2 + 1], both within the LDS; "
                                     "row threads 64..512 and plane threads 64..1024, powers of two");
  Medium3& M = P->med;
  if (P->auto_shape || rows != M.rt || cols != M.ct || row_threads != M.rthr || plane_threads != M.pthr) {
    H3CHK(hipDeviceSynchronize());
    M.rt = rows;
    M.ct = cols;
    M.ctiles = (M.nxh1 + cols - 1) / cols;
    M.rthr = row_threads;
    M.pthr = plane_threads;
    P->auto_shape = false;
    P->execs.clear();
  }
  return QPAT_OK;
}

qpat_status qpat3d_get_tiles(qpat_plan3d P, int32_t* rows, int32_t* cols, int32_t* row_threads,
                             int32_t* plane_threads) {
  if (!P || !rows || !cols) return set_error(QPAT_E_INVALID, "NULL argument");
  Medium3 m = P->med;
  if (P->auto_shape) auto_shape3(P->med, 1, m);
  *rows = m.rt;
  *cols = m.ct;
  if (row_threads) *row_threads = m.rthr;
  if (plane_threads) *plane_threads = m.pthr;
  return QPAT_OK;
}

qpat_status qpat3d_set_graph(qpat_plan3d P, int32_t enable) {
  if (!P) return set_error(QPAT_E_INVALID, "plan is NULL");
  P->graph = enable != 0;
  return QPAT_OK;
}

}  // extern "C"
