// Host runtime of libqpat: parameter validation, FP64 plan construction,
// work buffers, launch sequencing of the forward / adjoint time loops,
// checkpoints, uneven-grid batches, launch-shape tuning, hipGraph replay and
// the extern "C" entry points declared in include/qpat.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "../../include/qpat.h"
#include "qpat_internal.hpp"

using namespace qpat;

// ============================================================== errors
namespace {
thread_local std::string g_err;

qpat_status fail(qpat_status s, const std::string& msg) {
  g_err = msg;
  return s;
}
}  // namespace

namespace qpat {
// the error channel of qpat_last_error, for the other translation units
qpat_status set_error(qpat_status s, const std::string& msg) { return fail(s, msg); }

// A roctx range named after an entry point around its host side (argument
// checks and launches), seen by a profiler's marker trace next to the kernels.
TraceRange::TraceRange(const char* name) { roctxRangePushA(name); }
TraceRange::~TraceRange() { roctxRangePop(); }
}  // namespace qpat

namespace {

#define HIPCHK(expr)                                                                    \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(e_ == hipErrorOutOfMemory ? QPAT_E_OOM : QPAT_E_HIP,                  \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                  \
  } while (0)

#define STCHK(expr)                 \
  do {                              \
    qpat_status s_ = (expr);        \
    if (s_ != QPAT_OK) return s_;   \
  } while (0)

constexpr int kMaxN = 1024;
constexpr int kMinN = 8;

// n = 2^a or 3 * 2^a: radix plan with radices up to `maxr` (8 or 4), 4 bits
// per stage, first stage lowest (the kernels' compile-time plans, plan_radix,
// are the same); the radix-3 stage comes last so that the sub-transform
// length before every stage is a power of two.
bool radix_plan(int n, uint32_t* rad, int* nst, int maxr = 8) {
  if (n < kMinN || n > kMaxN || (n & 1)) return false;
  std::vector<int> r;
  int m = n;
  const bool three = (m % 3 == 0);
  if (three) m /= 3;
  if (m & (m - 1)) return false;
  int a = 0;
  while ((1 << a) < m) ++a;
  if (maxr == 8) {
    // radix 8, the remainder as 4 .. 4 (a = 3q + 1) or a radix-4 second stage
    // (a = 3q + 2), so that the plan starts and ends with the same radix
    const int q = a / 3, rem = a % 3;
    if (rem == 0) {
      for (int i = 0; i < q; ++i) r.push_back(8);
    } else if (rem == 1) {
      if (q == 0) {
        r.push_back(2);
      } else {
        r.push_back(4);
        for (int i = 0; i < q - 1; ++i) r.push_back(8);
        r.push_back(4);
      }
    } else {
      if (q == 0) {
        r.push_back(4);
      } else {
        r.push_back(8);
        r.push_back(4);
        for (int i = 0; i < q - 1; ++i) r.push_back(8);
      }
    }
  } else {
    const int q = a / 2, rem = a % 2;
    if (rem == 1) r.push_back(2);
    for (int i = 0; i < q; ++i) r.push_back(4);
  }
  if (three) r.push_back(3);
  *rad = 0;
  for (size_t i = 0; i < r.size(); ++i) *rad |= uint32_t(r[i]) << (4 * i);
  *nst = int(r.size());
  return true;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

double alpha0_np(double a_db, double y) {
  return a_db * 100.0 / (20.0 * std::log10(std::exp(1.0))) * std::pow(1e-6 / (2.0 * M_PI), y);
}

double stability_limit(double cmax, double cref, double dx, double dy) {
  if (cref >= cmax) return INFINITY;
  const double kmax = std::hypot(M_PI / dx, M_PI / dy);
  return 2.0 * std::asin(cref / cmax) / (cref * kmax);
}

int pow2_floor(int v) {
  int p = 1;
  while (p * 2 <= v) p *= 2;
  return p;
}
int pow2_divisor(int v) { return v & (-v); }

int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

bool threads_ok(int t) { return t == 64 || t == 128 || t == 256 || t == 512; }

// Column launches at these lengths take an instance whose FFT stages run in
// place (a compile-time power-of-two plan).
bool col_in_place(int ny) { return kernels_have_length(ny, true) && (ny & (ny - 1)) == 0; }

// A row tile of rt rows (rt even, dividing ny) fits the LDS limit and leaves
// at most kMaxPer pointwise elements per thread.
bool row_tile_ok(int nx, int ny, int rt, int thr) {
  // power-of-two columns of 128+ take the fused column pass, which needs the
  // tile height to divide the first-stage stride (at least ny / 8)
  const bool fused_cols = ny >= 128 && (ny & (ny - 1)) == 0;
  return rt >= 2 && (rt & (rt - 1)) == 0 && ny % rt == 0 && row_lds_bytes(nx, rt) <= kMaxLds &&
         threads_ok(thr) && rt * nx <= kMaxPer * thr && (!fused_cols || rt <= ny / 8);
}
// A column tile of ct spectrum columns fits the LDS limit and leaves at most
// kColPer elements of each field per thread (a column pass holds its input
// fields' first-stage values, multipliers and twiddles in registers together;
// the tighter bound keeps those under 128 VGPRs).
bool col_tile_ok(int nxh, int ny, int ct, int thr) {
  return ct >= 1 && (ct & (ct - 1)) == 0 && nxh % ct == 0 && col_lds_bytes(ny, ct) <= kMaxLds &&
         threads_ok(thr) && ct * ny <= kColPer * thr;
}

// Rows of the spectrum's storage tiles for row tiles of rt rows: at least
// kStorageRows where the grid allows it (a power of two, a multiple of rt,
// dividing ny and the first-stage stride of the fused column pass).  At one
// column per tile, row blocks of two rows then write and read 16-byte halves
// of 32-byte tiles, and column blocks read 32-byte runs instead of 16-byte
// ones.  Measured
// (1024^2 x 8, tiles 2,1,256,512): column passes 251 -> 208 us per iterate
// pair, row passes 307 -> 317 us; 8 or 16 rows cost the row passes more than
// the column passes gain.
constexpr int kStorageRows = 4;
int storage_rows(int ny, int rt) {
  const bool fused_cols = ny >= 128 && (ny & (ny - 1)) == 0;
  int s = rt;
  while (2 * s <= kStorageRows && ny % (2 * s) == 0 && (!fused_cols || 2 * s <= ny / 8)) s *= 2;
  return s;
}

// Defaults: small tiles (many blocks) with enough threads to keep every
// thread busy in the radix-8 stages.
void default_tiles(int nx, int ny, int* rt, int* ct, int* rthr, int* cthr) {
  int r = 2;
  while (r < 16 && r * nx < 2048 && row_tile_ok(nx, ny, 2 * r, 256)) r *= 2;
  int rthr_ = 64;
  while (rthr_ < 256 && (r * nx / 8 > rthr_ || !row_tile_ok(nx, ny, r, rthr_))) rthr_ *= 2;
  int c = 1;
  while (c < 16 && c * ny < 1024 && col_tile_ok(nx / 2, ny, 2 * c, 256)) c *= 2;
  int cthr_ = 64;
  while (cthr_ < 256 && (2 * c * ny / 8 > cthr_ || !col_tile_ok(nx / 2, ny, c, cthr_))) cthr_ *= 2;
  *rt = r;
  *ct = c;
  *rthr = rthr_;
  *cthr = cthr_;
}

}  // namespace

// ============================================================== executor
// A set of items (vectors / problems) advanced together: device item array,
// per-call I/O table, block maps of the row and column passes.
struct Exec {
  std::vector<Item> items;
  Item* d_items = nullptr;
  IO* d_io = nullptr;
  int2* d_rowmap = nullptr;
  int2* d_colmap = nullptr;
  int nrow = 0, ncol = 0;
  size_t row_lds = 0, col_lds = 0;
  int rthr = kBlock, cthr = kBlock;  // threads per block (max over items)
  int max_nt = 0, max_data = 0;
  // launch arguments; uniform = all items are vectors of one plan with equally
  // spaced work buffers (no block map / descriptor loads in the kernels)
  Launch L{};
  bool uniform = false;
  int row_ntile = 0, col_ntile = 0, row_chunk = 0, col_chunk = 0;
  int tab_nx = 0, tab_ny = 0;  // table launches: the row / column length all items share (0: they differ)
  bool row_tg = false, col_tg = false;  // uniform launches: FFT twiddles read from global memory
  bool lossy = false;
  // pinned staging ring for the I/O table
  static constexpr int kRing = 16;
  IO* h_io = nullptr;
  hipEvent_t ev[kRing] = {};
  bool ev_used[kRing] = {};
  int ring_pos = 0;
  // captured graphs, keyed by operation
  std::map<int, std::pair<hipGraph_t, hipGraphExec_t>> graphs;

  ~Exec() { release(); }
  void release() {
    for (auto& g : graphs) {
      if (g.second.second) (void)hipGraphExecDestroy(g.second.second);
      if (g.second.first) (void)hipGraphDestroy(g.second.first);
    }
    graphs.clear();
    if (d_items) (void)hipFree(d_items);
    if (d_io) (void)hipFree(d_io);
    if (d_rowmap) (void)hipFree(d_rowmap);
    if (d_colmap) (void)hipFree(d_colmap);
    if (h_io) (void)hipHostFree(h_io);
    for (int i = 0; i < kRing; ++i)
      if (ev[i]) (void)hipEventDestroy(ev[i]);
    d_items = nullptr;
    d_io = nullptr;
    d_rowmap = d_colmap = nullptr;
    h_io = nullptr;
    for (int i = 0; i < kRing; ++i) {
      ev[i] = nullptr;
      ev_used[i] = false;
    }
  }
};

namespace {

// XCD-aware block map: natural entry i goes to XCD i / chunk, so that
// consecutive tiles of one item share an XCD (and its L2).
std::vector<int2> xcd_map(const std::vector<int2>& nat) {
  const int L = int(nat.size());
  const int chunk = (L + kXcds - 1) / kXcds;
  std::vector<int2> out(size_t(chunk) * kXcds, make_int2(-1, -1));
  for (int i = 0; i < L; ++i) {
    const int x = i / chunk, s = i % chunk;
    out[size_t(s) * kXcds + x] = nat[i];
  }
  return out;
}

qpat_status exec_build(Exec& E, const std::vector<Item>& items) {
  E.release();
  E.items = items;
  const int ni = int(items.size());
  std::vector<int2> rows, cols;
  E.max_nt = 0;
  E.max_data = 0;
  E.row_lds = E.col_lds = 0;
  E.rthr = E.cthr = 0;
  E.lossy = items[0].m.lossy != 0;
  for (int i = 0; i < ni; ++i) {
    const Medium& m = items[i].m;
    for (int t = 0; t < m.ny / m.rt; ++t) rows.push_back(make_int2(i, t));
    for (int t = 0; t < m.nxh / m.ct; ++t) cols.push_back(make_int2(i, t));
    E.max_nt = std::max(E.max_nt, m.nt);
    E.max_data = std::max(E.max_data, m.nt * m.ns);
    E.row_lds = std::max(E.row_lds, row_lds_bytes(m.nx, m.rt));
    E.col_lds = std::max(E.col_lds, col_lds_bytes(m.ny, m.ct));
    E.rthr = std::max(E.rthr, m.rthr);
    E.cthr = std::max(E.cthr, m.cthr);
  }
  E.tab_nx = items[0].m.nx;
  E.tab_ny = items[0].m.ny;
  for (int i = 1; i < ni; ++i) {
    if (items[i].m.nx != E.tab_nx) E.tab_nx = 0;
    if (items[i].m.ny != E.tab_ny) E.tab_ny = 0;
  }
  const std::vector<int2> rm = xcd_map(rows), cm = xcd_map(cols);
  E.nrow = int(rm.size());
  E.ncol = int(cm.size());
  // uniform launch?
  {
    const Medium& m0 = items[0].m;
    bool u = true;
    long long stride = 0;
    if (ni > 1) stride = (const char*)items[1].w.f0 - (const char*)items[0].w.f0;
    for (int i = 0; i < ni && u; ++i) {
      const Medium& m = items[i].m;
      u = m.c2 == m0.c2 && m.nx == m0.nx && m.ny == m0.ny && m.nt == m0.nt && m.rt == m0.rt &&
          m.srt == m0.srt && m.ct == m0.ct && m.rthr == m0.rthr && m.cthr == m0.cthr;
      const Work& w = items[i].w;
      const Work& w0 = items[0].w;
      auto d = [&](const void* a, const void* b) { return (long long)((const char*)a - (const char*)b); };
      const long long off = stride * i;
      u = u && d(w.f0, w0.f0) == off && d(w.f1, w0.f1) == off && d(w.f2, w0.f2) == off &&
          d(w.f3, w0.f3) == off && d(w.q, w0.q) == off && d(w.s0, w0.s0) == off && d(w.s1, w0.s1) == off &&
          d(w.part, w0.part) == off;
    }
    E.uniform = u;
    E.L.m = m0;
    E.L.w0 = items[0].w;
    E.L.wstride = stride;
    E.L.nitems = ni;
    E.row_ntile = m0.ny / m0.rt;
    E.col_ntile = m0.nxh / m0.ct;
    E.row_chunk = (ni * E.row_ntile + kXcds - 1) / kXcds;
    E.col_chunk = (ni * E.col_ntile + kXcds - 1) / kXcds;
    // Twiddles from global memory when a pass has at most about two blocks
    // per CU (latency-bound: the LDS staging of the table is on the critical
    // path); with more blocks the LDS copy is kept.
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 0;
    E.row_tg = u && cus > 0 && kernels_have_length(m0.nx, false) && ni * E.row_ntile <= 2 * cus;
    E.col_tg = u && cus > 0 && kernels_have_length(m0.ny, true) && ni * E.col_ntile <= 2 * cus;
    // row instances with a compile-time length, and column instances with a
    // compile-time power-of-two length, run in place unless they read global
    // twiddles (one LDS line buffer instead of two)
    if (u) E.row_lds = row_lds_bytes(m0.nx, m0.rt, E.row_tg, kernels_have_length(m0.nx, false) && !E.row_tg);
    if (u) E.col_lds = col_lds_bytes(m0.ny, m0.ct, E.col_tg, col_in_place(m0.ny) && !E.col_tg);
  }
  if (!E.uniform && E.tab_nx && kernels_have_length(E.tab_nx, false)) {
    E.row_lds = 0;
    for (int i = 0; i < ni; ++i)
      E.row_lds = std::max(E.row_lds, row_lds_bytes(items[i].m.nx, items[i].m.rt, false, true));
  }
  if (!E.uniform && E.tab_ny && col_in_place(E.tab_ny)) {
    E.col_lds = 0;
    for (int i = 0; i < ni; ++i)
      E.col_lds = std::max(E.col_lds, col_lds_bytes(items[i].m.ny, items[i].m.ct, false, true));
  }
  HIPCHK(hipMalloc(&E.d_items, sizeof(Item) * ni));
  HIPCHK(hipMalloc(&E.d_io, sizeof(IO) * ni));
  HIPCHK(hipMalloc(&E.d_rowmap, sizeof(int2) * rm.size()));
  HIPCHK(hipMalloc(&E.d_colmap, sizeof(int2) * cm.size()));
  HIPCHK(hipMemcpy(E.d_items, items.data(), sizeof(Item) * ni, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(E.d_rowmap, rm.data(), sizeof(int2) * rm.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(E.d_colmap, cm.data(), sizeof(int2) * cm.size(), hipMemcpyHostToDevice));
  HIPCHK(hipMemset(E.d_io, 0, sizeof(IO) * ni));
  HIPCHK(hipHostMalloc(&E.h_io, sizeof(IO) * ni * Exec::kRing, hipHostMallocDefault));
  E.L.map = nullptr;
  E.L.items = E.d_items;
  E.L.io = E.d_io;
  for (int i = 0; i < Exec::kRing; ++i) HIPCHK(hipEventCreateWithFlags(&E.ev[i], hipEventDisableTiming));
  return QPAT_OK;
}

// Upload the per-call I/O table (stream ordered; the staging slot is reused
// only after its previous copy has executed).
qpat_status exec_set_io(Exec& E, const std::vector<IO>& io, hipStream_t st) {
  const int ni = int(E.items.size());
  const int slot = E.ring_pos;
  E.ring_pos = (E.ring_pos + 1) % Exec::kRing;
  if (E.ev_used[slot]) HIPCHK(hipEventSynchronize(E.ev[slot]));
  IO* h = E.h_io + size_t(slot) * ni;
  std::memcpy(h, io.data(), sizeof(IO) * ni);
  HIPCHK(hipMemcpyAsync(E.d_io, h, sizeof(IO) * ni, hipMemcpyHostToDevice, st));
  HIPCHK(hipEventRecord(E.ev[slot], st));
  E.ev_used[slot] = true;
  return QPAT_OK;
}

hipError_t row(Exec& E, int mode, int n, int flags, hipStream_t st) {
  // the lossy density passes past the first iterates take the instances that
  // hold only the fused-boundary-stage path, where one exists
  if ((mode == RM_F2 || mode == RM_A2) && n >= 1 &&
      (E.uniform ? kernels_row_fused(E.L.m.nx, E.row_tg) : kernels_row_fused(E.tab_nx, false)))
    mode |= RM_FZ;
  if (E.uniform)
    return launch_row(mode, E.L, true, 0, E.row_tg, E.row_ntile, E.row_chunk, E.row_chunk * kXcds, E.rthr,
                      E.row_lds, n, flags, st);
  Launch L = E.L;
  L.map = E.d_rowmap;
  return launch_row(mode, L, false, E.tab_nx, false, 0, 0, E.nrow, E.rthr, E.row_lds, n, flags, st);
}
hipError_t col(Exec& E, int cm, int n, hipStream_t st, int mcode = 0) {
  if (E.uniform)
    return launch_col(cm, mcode, E.L, true, 0, E.col_tg, E.col_ntile, E.col_chunk, E.col_chunk * kXcds, E.cthr,
                      E.col_lds, n, st);
  Launch L = E.L;
  L.map = E.d_colmap;
  return launch_col(cm, mcode, L, false, E.tab_ny, false, 0, 0, E.ncol, E.cthr, E.col_lds, n, st);
}

#define LCHK(expr)                           \
  do {                                       \
    hipError_t e_ = (expr);                  \
    if (e_ != hipSuccess) return e_;         \
  } while (0)

// One forward iterate n (eqs num-vel, num-rho, num-p, num-m).  With `sens`
// the pressure pass also stores dp^{n+1}/dc at the slot carried in `flags`.
hipError_t fwd_iterate(Exec& E, int n, int flags, hipStream_t st, bool sens = false) {
  if (n > -1) {
    LCHK(col(E, CM_GRADP1, n, st));
    LCHK(row(E, RM_F1, n, 0, st));
    LCHK(col(E, CM_GRADM2, n, st));
  }
  if (E.lossy) {
    LCHK(row(E, RM_F2, n, 0, st));
    LCHK(col(E, CM_FRAC, n, st));
    LCHK(row(E, sens ? (RM_F3 | RM_X) : RM_F3, n, flags, st));
  } else {
    LCHK(row(E, sens ? (RM_F2L | RM_X) : RM_F2L, n, flags, st));
  }
  return hipSuccess;
}

// The forward time loop up to iterate n_last (inclusive), then the sensor data.
hipError_t seq_forward(Exec& E, int n_last, hipStream_t st) {
  for (int n = -1; n <= n_last; ++n) LCHK(fwd_iterate(E, n, 0, st));
  return launch_combine(E.d_items, E.d_io, int(E.items.size()), E.max_data, st);
}

// One adjoint iterate n (transposes of the forward passes of iterate n, in
// reverse order).  With `gc` the first pass also adds p*^{n+1} dp^{n+1}/dc,
// the sensitivity read from the slot carried in `flags`.
hipError_t adj_iterate(Exec& E, int n, int flags, hipStream_t st, bool gc = false) {
  if (E.lossy) {
    LCHK(row(E, gc ? (RM_A1 | RM_X) : RM_A1, n, flags, st));
    LCHK(col(E, CM_FRAC, n, st));
    LCHK(row(E, RM_A2, n, 0, st));
  } else {
    LCHK(row(E, gc ? (RM_A1L | RM_X) : RM_A1L, n, flags, st));
  }
  if (n == -1) return hipSuccess;
  LCHK(col(E, CM_GRADP2, n, st));
  LCHK(row(E, RM_A3, n, 0, st));
  LCHK(col(E, CM_DIVM, n, st));
  return hipSuccess;
}

// The reverse time loop of the adjoint.
hipError_t seq_adjoint(Exec& E, hipStream_t st) {
  LCHK(launch_tap_order(E.d_items, E.d_io, int(E.items.size()), 2 * E.max_data, st));
  for (int n = E.max_nt - 2; n >= -1; --n) LCHK(adj_iterate(E, n, 0, st));
  return hipSuccess;
}

enum Op { OP_FWD = 1, OP_ADJ = 2 };

// Run `op` on the executor, via a captured graph when enabled.
qpat_status exec_run(Exec& E, int op, bool use_graph, hipStream_t st) {
  auto body = [&](hipStream_t s) -> hipError_t {
    return op == OP_FWD ? seq_forward(E, E.max_nt - 2, s) : seq_adjoint(E, s);
  };
  if (!use_graph || st == nullptr) {
    hipError_t e = body(st);
    if (e != hipSuccess) return fail(QPAT_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return QPAT_OK;
  }
  auto it = E.graphs.find(op);
  if (it == E.graphs.end()) {
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    hipError_t e = body(st);
    hipError_t e2 = hipStreamEndCapture(st, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(QPAT_E_HIP, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    HIPCHK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
    it = E.graphs.emplace(op, std::make_pair(g, ge)).first;
  }
  HIPCHK(hipGraphLaunch(it->second.second, st));
  return QPAT_OK;
}

}  // namespace

// ============================================================== plan
struct qpat_plan_s {
  qpat_params prm{};
  std::vector<double> sensors;
  Medium med{};
  void* d_med = nullptr;      // one allocation for all medium tables
  size_t med_bytes = 0;
  // per-vector work buffers
  int cap = 0;
  void* d_work = nullptr;
  size_t work_item_bytes = 0;
  std::vector<Work> works;
  std::vector<float*> datas;  // per-vector data buffers for jtjv
  // executors per batch size (rebuilt when tiles change)
  std::map<int, std::unique_ptr<Exec>> execs;
  // sound-speed gradient: per batch size, a forward executor on work vectors
  // [0, B) and an adjoint executor on [B, 2B), so that replaying the forward
  // leaves the adjoint state alone
  std::map<int, std::pair<std::unique_ptr<Exec>, std::unique_ptr<Exec>>> grad_execs;
  void clear_execs() {
    execs.clear();
    grad_execs.clear();
  }
  bool graph = false;
  int rt = 2, ct = 1, rthr = kBlock, cthr = kBlock;
  // opt-in output check: flag set by a kernel after each solve
  bool check = false;
  int* d_flag = nullptr;
};

struct qpat_batch_s {
  std::vector<qpat_plan> plans;
  std::vector<void*> blocks;       // per-problem work allocations (owned)
  std::vector<Work> works;
  std::vector<float*> datas;
  // Schedule: the problems are split into groups, each advanced by one
  // executor (one launch per pass for the group, with the launch shape of its
  // plans).  Schedule 0 has one group; schedule 1 one group per grid size,
  // the groups running side by side on streams forked from the caller's.
  struct Group {
    std::vector<int> members;
    Exec exec;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
  };
  std::vector<std::unique_ptr<Group>> groups;
  int schedule = 0;
  hipEvent_t fork = nullptr;
  bool graph = false;
  std::map<int, std::pair<hipGraph_t, hipGraphExec_t>> graphs;  // whole fork/join sequences, by operation
  void release_groups() {
    for (auto& g : graphs) {
      if (g.second.second) (void)hipGraphExecDestroy(g.second.second);
      if (g.second.first) (void)hipGraphDestroy(g.second.first);
    }
    graphs.clear();
    for (auto& g : groups) {
      g->exec.release();
      if (g->stream) (void)hipStreamDestroy(g->stream);
      if (g->done) (void)hipEventDestroy(g->done);
    }
    groups.clear();
  }
  ~qpat_batch_s() {
    release_groups();
    if (fork) (void)hipEventDestroy(fork);
    for (void* b : blocks)
      if (b) (void)hipFree(b);
  }
};

namespace {

qpat_status validate(const qpat_params* p) {
  if (!p) return fail(QPAT_E_INVALID, "params is NULL");
  uint32_t r;
  int s;
  if (!radix_plan(p->nx, &r, &s) || !radix_plan(p->ny, &r, &s))
    return fail(QPAT_E_UNSUPPORTED, "nx, ny must be 2^a or 3*2^a in [8, 1024] (got " +
                                        std::to_string(p->nx) + " x " + std::to_string(p->ny) + ")");
  if (!finite_pos(p->dx) || !finite_pos(p->dy) || !finite_pos(p->dt))
    return fail(QPAT_E_INVALID, "dx, dy, dt must be finite and > 0");
  if (p->nt < 1) return fail(QPAT_E_INVALID, "nt must be >= 1");
  if (int64_t(p->nt) * std::max(p->ns, 0) >= (int64_t(1) << 30))
    return fail(QPAT_E_UNSUPPORTED, "nt * ns must be below 2^30 (32-bit sample indices)");
  if (!finite_pos(p->c_ref)) return fail(QPAT_E_INVALID, "c_ref must be finite and > 0");
  if (p->pml_size < 0 || 2 * p->pml_size >= std::min(p->nx, p->ny))
    return fail(QPAT_E_INVALID, "pml_size must be in [0, min(nx, ny)/2)");
  if (!(std::isfinite(p->pml_alpha) && p->pml_alpha >= 0.0))
    return fail(QPAT_E_INVALID, "pml_alpha must be finite and >= 0");
  if (!(std::isfinite(p->alpha0_db) && p->alpha0_db >= 0.0))
    return fail(QPAT_E_INVALID, "alpha0_db must be finite and >= 0");
  if (p->alpha0_db > 0.0) {
    if (!(std::isfinite(p->y) && p->y > 0.0 && p->y <= 3.0))
      return fail(QPAT_E_INVALID, "y must be in (0, 3]");
    if (std::fabs(std::cos(M_PI * p->y / 2.0)) < 1e-9)
      return fail(QPAT_E_UNSUPPORTED, "tan(pi y / 2) is singular for odd integer y");
  }
  if (p->ns < 1) return fail(QPAT_E_INVALID, "ns must be >= 1");
  if (!p->sensor_xy) return fail(QPAT_E_INVALID, "sensor_xy is NULL");
  for (int s2 = 0; s2 < p->ns; ++s2) {
    const double x = p->sensor_xy[2 * s2], y = p->sensor_xy[2 * s2 + 1];
    const double u = x / p->dx + p->nx / 2, v = y / p->dy + p->ny / 2;
    if (!(std::isfinite(u) && std::isfinite(v) && u >= 0.0 && u <= p->nx - 1 && v >= 0.0 &&
          v <= p->ny - 1))
      return fail(QPAT_E_INVALID, "sensor " + std::to_string(s2) + " lies outside the grid");
  }
  const long long data = (long long)p->nt * p->ns;
  if (data > (1LL << 30)) return fail(QPAT_E_INVALID, "nt * ns too large");
  return QPAT_OK;
}

// Bilinear taps (eq num-m), grouped by grid row in CSR form.
void build_taps(const qpat_params& p, std::vector<Tap>& taps, std::vector<int>& off) {
  std::vector<std::vector<Tap>> byrow(p.ny);
  for (int s = 0; s < p.ns; ++s) {
    const double u = p.sensor_xy[2 * s] / p.dx + p.nx / 2, v = p.sensor_xy[2 * s + 1] / p.dy + p.ny / 2;
    const int ix = int(std::floor(u)), iy = int(std::floor(v));
    const double fx = u - ix, fy = v - iy;
    const int ix1 = std::min(ix + 1, p.nx - 1), iy1 = std::min(iy + 1, p.ny - 1);
    Tap a{s, 0, iy, ix, ix1, float((1 - fx) * (1 - fy)), float(fx * (1 - fy)), 0};
    Tap b{s, 1, iy1, ix, ix1, float((1 - fx) * fy), float(fx * fy), 0};
    byrow[iy].push_back(a);
    byrow[iy1].push_back(b);
  }
  taps.clear();
  off.assign(p.ny + 1, 0);
  for (int y = 0; y < p.ny; ++y) {
    off[y] = int(taps.size());
    for (const Tap& t : byrow[y]) taps.push_back(t);
  }
  off[p.ny] = int(taps.size());
}

// The adjoint of the tap gather as a gather per grid node: for every node a
// tap touches, its contributions (tap e, left / right weight) in increasing e,
// the order in which a serial scatter over the taps of its row adds them.
void build_scatter(const qpat_params& p, const std::vector<Tap>& taps, const std::vector<int>& toff,
                   std::vector<int4>& nodes, std::vector<int>& noff, std::vector<int>& scon) {
  nodes.clear();
  scon.clear();
  noff.assign(p.ny + 1, 0);
  for (int y = 0; y < p.ny; ++y) {
    noff[y] = int(nodes.size() / 2);  // offsets count records (two int4 each)
    std::map<int, std::vector<int>> byx;   // x -> contributions in tap order
    for (int e = toff[y]; e < toff[y + 1]; ++e) {
      byx[taps[e].ixl].push_back(e << 1);
      byx[taps[e].ixr].push_back((e << 1) | 1);
    }
    for (const auto& kv : byx) {
      const int c0 = int(scon.size());
      for (int c : kv.second) scon.push_back(c);
      const int c1 = int(scon.size());
      // the record: (y, x, c0, c1), then the first kConRegs contributions
      // inline (the kernel reads them with the record, not after it)
      nodes.push_back(make_int4(y, kv.first, c0, c1));
      int in[kConRegs] = {0, 0, 0, 0};
      for (int k = 0; k < kConRegs && c0 + k < c1; ++k) in[k] = scon[c0 + k];
      nodes.push_back(make_int4(in[0], in[1], in[2], in[3]));
    }
  }
  noff[p.ny] = int(nodes.size() / 2);
}

// Carve aligned sub-buffers out of one allocation.
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

qpat_status plan_build(qpat_plan P, const double* c0, const double* rho0) {
  const qpat_params& p = P->prm;
  const int nx = p.nx, ny = p.ny, nxh = nx / 2, N = nx * ny;
  const double dx = p.dx, dy = p.dy, dt = p.dt;
  // medium checks
  double cmax = 0.0;
  for (int i = 0; i < N; ++i) {
    if (!finite_pos(c0[i])) return fail(QPAT_E_INVALID, "c0 must be finite and > 0 everywhere");
    if (!finite_pos(rho0[i])) return fail(QPAT_E_INVALID, "rho0 must be finite and > 0 everywhere");
    cmax = std::max(cmax, c0[i]);
  }
  const double lim = stability_limit(cmax, p.c_ref, dx, dy);
  if (dt > lim)
    return fail(QPAT_E_UNSTABLE, "dt = " + std::to_string(dt) + " exceeds the k-space stability bound " +
                                     std::to_string(lim) + " for c_ref < max(c0)");
  const bool lossy = p.alpha0_db > 0.0;

  // ---- FP64 derived quantities
  std::vector<float> c2(N), c2eta(N), c2tau(N), r0(N), bx(N), by(N);
  const double a0 = lossy ? alpha0_np(p.alpha0_db, p.y) : 0.0;
  const double tn = lossy ? std::tan(M_PI * p.y / 2.0) : 0.0;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const int k = j * nx + i;
      const double c = c0[k];
      c2[k] = float(c * c);
      // eq Twelve: tau = -2 a0 c^(y-1), eta = 2 a0 c^y tan(pi y/2)
      c2eta[k] = lossy ? float(c * c * 2.0 * a0 * std::pow(c, p.y) * tn) : 0.f;
      c2tau[k] = lossy ? float(c * c * -2.0 * a0 * std::pow(c, p.y - 1.0)) : 0.f;
      r0[k] = float(rho0[k]);
      const double rx = 0.5 * (rho0[k] + rho0[j * nx + (i + 1) % nx]);
      const double ry = 0.5 * (rho0[k] + rho0[((j + 1) % ny) * nx + i]);
      bx[k] = float(dt / rx);
      by[k] = float(dt / ry);
    }
  // PML (eq dis-pml), 4th-power profile inside the grid
  auto sigma = [&](double pos, int n, double d) {
    const int L = p.pml_size;
    if (L <= 0) return 0.0;
    const double xi = std::max(0.0, std::max(L - pos, pos - (n - 1 - L)));
    return p.pml_alpha * (p.c_ref / d) * std::pow(xi / L, 4);
  };
  std::vector<float> avx(nx), arx(nx), avy(ny), ary(ny);
  for (int i = 0; i < nx; ++i) {
    arx[i] = float(std::exp(-sigma(i, nx, dx) * dt / 2.0));
    avx[i] = float(std::exp(-sigma(i + 0.5, nx, dx) * dt / 2.0));
  }
  for (int j = 0; j < ny; ++j) {
    ary[j] = float(std::exp(-sigma(j, ny, dy) * dt / 2.0));
    avy[j] = float(std::exp(-sigma(j + 0.5, ny, dy) * dt / 2.0));
  }
  // wavenumbers; Nyquist at -pi/d where the staggered symbol is real
  auto kval = [](int idx, int n, double d) {
    const int f = idx < n / 2 ? idx : idx - n;
    return 2.0 * M_PI * f / (n * d);
  };
  auto dsym = [](double k, double d, int sgn, bool nyq) {
    // i k e^{sgn i k d/2}
    const double th = sgn * k * d / 2.0;
    if (nyq) return make_float2(float(-k * std::sin(th)), 0.f);
    return make_float2(float(-k * std::sin(th)), float(k * std::cos(th)));
  };
  std::vector<float2> dxp(nxh + 1), dxm(nxh + 1), dyp(ny), dym(ny);
  for (int i = 0; i <= nxh; ++i) {
    const double k = kval(i, nx, dx);
    dxp[i] = dsym(k, dx, +1, i == nxh);
    dxm[i] = dsym(k, dx, -1, i == nxh);
  }
  for (int j = 0; j < ny; ++j) {
    const double k = kval(j, ny, dy);
    dyp[j] = dsym(k, dy, +1, j == ny / 2);
    dym[j] = dsym(k, dy, -1, j == ny / 2);
  }
  const size_t nt2 = size_t(ny) * (nxh + 1);
  std::vector<float> kap(nt2), ldis(nt2), labs(nt2);
  const double inv = 1.0 / (double(nx) * ny);
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i <= nxh; ++i) {
      const double kx = kval(i, nx, dx), ky = kval(j, ny, dy);
      const double K = std::sqrt(kx * kx + ky * ky);
      const double arg = p.c_ref * K * dt / 2.0;
      const double kp = arg == 0.0 ? 1.0 : std::sin(arg) / arg;
      const size_t t = size_t(i) * ny + j;   // [kx][ky]: a spectrum column's entries contiguous
      kap[t] = float(kp * inv);
      ldis[t] = (K == 0.0 || !lossy) ? 0.f : float(std::pow(K, p.y - 1.0) * inv);
      labs[t] = (K == 0.0 || !lossy) ? 0.f : float(std::pow(K, p.y - 2.0) * inv);
    }
  // FFT twiddles W_{Ns R}^{k r} per Stockham stage (radix R, Ns = product of
  // the earlier radices), stored as [stage][r - 1][k]; the stage blocks
  // telescope to n - R0 entries.
  // rev: the plan in reverse order (the inverse transforms of the fused
  // column passes; power-of-two lengths only, Ns stays a power of two).
  auto twid = [](int n, bool rev) {
    uint32_t rad = 0;
    int nst = 0;
    radix_plan(n, &rad, &nst, 8);
    std::vector<float2> t(n, make_float2(0.f, 0.f));
    if (rev && (n & (n - 1))) return t;
    auto radix = [&](int st) { return int((rad >> (4 * (rev ? nst - 1 - st : st))) & 15); };
    const int r0 = radix(0);
    int ns = 1;
    for (int st = 0; st < nst; ++st) {
      const int R = radix(st);
      if (st > 0)
        for (int r = 1; r < R; ++r)
          for (int k = 0; k < ns; ++k) {
            const double a = -2.0 * M_PI * double(k) * double(r) / double(ns * R);
            t[size_t(ns - r0 + (r - 1) * ns + k)] = make_float2(float(std::cos(a)), float(std::sin(a)));
          }
      ns *= R;
    }
    return t;
  };
  const std::vector<float2> twx = twid(nx, false), twy = twid(ny, false), twyr = twid(ny, true);
  std::vector<Tap> taps;
  std::vector<int> toff;
  build_taps(p, taps, toff);
  std::vector<int4> snodes;
  std::vector<int> snoff, scon;
  build_scatter(p, taps, toff, snodes, snoff, scon);
  if (taps.empty()) taps.push_back(Tap{});
  if (snodes.empty()) snodes.assign(2, make_int4(0, 0, 0, 0));
  if (scon.empty()) scon.push_back(0);

  // ---- upload (host checks are done; from here on a device is needed)
  {
    const hipError_t e = kernels_allow_lds(kMaxLds);
    if (e != hipSuccess) return fail(QPAT_E_HIP, std::string("LDS attribute: ") + hipGetErrorString(e));
  }
  Carver cv;
  const size_t o_c2 = cv.take<float>(N), o_c2eta = cv.take<float>(N), o_c2tau = cv.take<float>(N);
  const size_t o_r0 = cv.take<float>(N), o_bx = cv.take<float>(N), o_by = cv.take<float>(N);
  const size_t o_avx = cv.take<float>(nx), o_arx = cv.take<float>(nx);
  const size_t o_avy = cv.take<float>(ny), o_ary = cv.take<float>(ny);
  const size_t o_dxp = cv.take<float2>(nxh + 1), o_dxm = cv.take<float2>(nxh + 1);
  const size_t o_dyp = cv.take<float2>(ny), o_dym = cv.take<float2>(ny);
  const size_t o_kap = cv.take<float>(nt2), o_ldis = cv.take<float>(nt2), o_labs = cv.take<float>(nt2);
  const size_t o_twx = cv.take<float2>(nx), o_twy = cv.take<float2>(ny), o_twyr = cv.take<float2>(ny);
  const size_t o_toff = cv.take<int>(toff.size()), o_taps = cv.take<Tap>(taps.size());
  const size_t o_snoff = cv.take<int>(snoff.size()), o_snodes = cv.take<int4>(snodes.size()),
               o_scon = cv.take<int>(scon.size());
  const size_t total = cv.off;
  std::vector<char> host(total, 0);
  auto put = [&](size_t o, const void* src, size_t bytes) { std::memcpy(host.data() + o, src, bytes); };
  put(o_c2, c2.data(), N * 4);
  put(o_c2eta, c2eta.data(), N * 4);
  put(o_c2tau, c2tau.data(), N * 4);
  put(o_r0, r0.data(), N * 4);
  put(o_bx, bx.data(), N * 4);
  put(o_by, by.data(), N * 4);
  put(o_avx, avx.data(), nx * 4);
  put(o_arx, arx.data(), nx * 4);
  put(o_avy, avy.data(), ny * 4);
  put(o_ary, ary.data(), ny * 4);
  put(o_dxp, dxp.data(), (nxh + 1) * 8);
  put(o_dxm, dxm.data(), (nxh + 1) * 8);
  put(o_dyp, dyp.data(), ny * 8);
  put(o_dym, dym.data(), ny * 8);
  put(o_kap, kap.data(), nt2 * 4);
  put(o_ldis, ldis.data(), nt2 * 4);
  put(o_labs, labs.data(), nt2 * 4);
  put(o_twx, twx.data(), nx * 8);
  put(o_twy, twy.data(), ny * 8);
  put(o_twyr, twyr.data(), ny * 8);
  put(o_toff, toff.data(), toff.size() * 4);
  put(o_taps, taps.data(), taps.size() * sizeof(Tap));
  put(o_snoff, snoff.data(), snoff.size() * 4);
  put(o_snodes, snodes.data(), snodes.size() * sizeof(int4));
  put(o_scon, scon.data(), scon.size() * 4);
  char* d = nullptr;
  HIPCHK(hipMalloc(&d, total));
  P->d_med = d;
  P->med_bytes = total;
  HIPCHK(hipMemcpy(d, host.data(), total, hipMemcpyHostToDevice));

  Medium& M = P->med;
  M.nx = nx;
  M.ny = ny;
  M.nxh = nxh;
  M.nt = p.nt;
  M.ns = p.ns;
  M.lossy = lossy ? 1 : 0;
  M.dt = float(dt);
  M.ypow = float(p.y);
  radix_plan(nx, &M.radx, &M.nstx, 8);
  radix_plan(ny, &M.rady, &M.nsty, 8);
  M.c2 = (const float*)(d + o_c2);
  M.c2eta = (const float*)(d + o_c2eta);
  M.c2tau = (const float*)(d + o_c2tau);
  M.rho0 = (const float*)(d + o_r0);
  M.bx = (const float*)(d + o_bx);
  M.by = (const float*)(d + o_by);
  M.avx = (const float*)(d + o_avx);
  M.arx = (const float*)(d + o_arx);
  M.avy = (const float*)(d + o_avy);
  M.ary = (const float*)(d + o_ary);
  M.dxp = (const float2*)(d + o_dxp);
  M.dxm = (const float2*)(d + o_dxm);
  M.dyp = (const float2*)(d + o_dyp);
  M.dym = (const float2*)(d + o_dym);
  M.kap = (const float*)(d + o_kap);
  M.ldis = (const float*)(d + o_ldis);
  M.labs = (const float*)(d + o_labs);
  M.twx = (const float2*)(d + o_twx);
  M.twy = (const float2*)(d + o_twy);
  M.twyr = (const float2*)(d + o_twyr);
  M.tap_off = (const int*)(d + o_toff);
  M.taps = (const Tap*)(d + o_taps);
  M.node_off = (const int*)(d + o_snoff);
  M.nodes = (const int4*)(d + o_snodes);
  M.scon = (const int*)(d + o_scon);
  default_tiles(nx, ny, &P->rt, &P->ct, &P->rthr, &P->cthr);
  M.rt = P->rt;
  M.ct = P->ct;
  M.rthr = P->rthr;
  M.cthr = P->cthr;
  M.lrt = ilog2(P->rt);
  M.lct = ilog2(P->ct);
  M.srt = storage_rows(ny, P->rt);
  M.lsrt = ilog2(M.srt);
  return QPAT_OK;
}

// Work buffers for `count` vectors of a problem of the size of `p` in one
// allocation: per vector [f0 f1 f2 f3 q] fields, two half spectra, the sensor
// partials and a data buffer (used by jtjv).
qpat_status alloc_works(const qpat_params& p, int count, void** block, size_t* per_item,
                        std::vector<Work>& works, std::vector<float*>& datas) {
  const int nx = p.nx, ny = p.ny, N = nx * ny;
  const size_t ndata = size_t(p.nt) * p.ns;
  Carver cv;
  const size_t o_f = cv.take<float>(size_t(5) * N);
  const size_t o_s0 = cv.take<float2>(size_t(ny) * (nx / 2));
  const size_t o_s1 = cv.take<float2>(size_t(ny) * (nx / 2));
  const size_t o_part = cv.take<float>(2 * ndata);
  const size_t o_data = cv.take<float>(ndata);
  const size_t per = (cv.off + 255) & ~size_t(255);
  char* d = nullptr;
  HIPCHK(hipMalloc(&d, per * count));
  *block = d;
  *per_item = per;
  works.clear();
  datas.clear();
  for (int i = 0; i < count; ++i) {
    char* base = d + per * i;
    Work w{};
    float* f = (float*)(base + o_f);
    w.f0 = f;
    w.f1 = f + N;
    w.f2 = f + 2 * N;
    w.f3 = f + 3 * N;
    w.q = f + 4 * N;
    w.s0 = (float2*)(base + o_s0);
    w.s1 = (float2*)(base + o_s1);
    w.part = (float*)(base + o_part);
    works.push_back(w);
    datas.push_back((float*)(base + o_data));
  }
  return QPAT_OK;
}

// Make sure the plan has work buffers for `b` vectors.
qpat_status plan_reserve(qpat_plan P, int b) {
  if (b <= P->cap) return QPAT_OK;
  if (P->d_work) {
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipFree(P->d_work));
    P->d_work = nullptr;
  }
  P->clear_execs();
  P->cap = 0;
  STCHK(alloc_works(P->prm, b, &P->d_work, &P->work_item_bytes, P->works, P->datas));
  P->cap = b;
  return QPAT_OK;
}

qpat_status plan_exec(qpat_plan P, int b, Exec** out) {
  STCHK(plan_reserve(P, b));
  auto it = P->execs.find(b);
  if (it == P->execs.end()) {
    std::vector<Item> items(b);
    for (int i = 0; i < b; ++i) {
      items[i].m = P->med;
      items[i].w = P->works[i];
    }
    std::unique_ptr<Exec> E(new Exec());
    STCHK(exec_build(*E, items));
    it = P->execs.emplace(b, std::move(E)).first;
  }
  *out = it->second.get();
  return QPAT_OK;
}

qpat_status check_plan_call(qpat_plan P, const void* a, const void* b, int batch) {
  if (!P) return fail(QPAT_E_INVALID, "plan is NULL");
  if (!a || !b) return fail(QPAT_E_INVALID, "input / output pointer is NULL");
  if (batch < 1 || batch > 4096) return fail(QPAT_E_INVALID, "batch must be in [1, 4096]");
  return QPAT_OK;
}

size_t field_elems(qpat_plan P) { return size_t(P->prm.nx) * P->prm.ny; }
size_t data_elems(qpat_plan P) { return size_t(P->prm.nt) * P->prm.ns; }

qpat_status do_forward(qpat_plan P, const float* p0, float* data, int batch, hipStream_t st,
                       bool internal_data) {
  Exec* E = nullptr;
  STCHK(plan_exec(P, batch, &E));
  std::vector<IO> io(batch);
  for (int i = 0; i < batch; ++i) {
    io[i].in = p0 + field_elems(P) * i;
    io[i].out = internal_data ? P->datas[i] : data + data_elems(P) * i;
  }
  STCHK(exec_set_io(*E, io, st));
  STCHK(exec_run(*E, OP_FWD, P->graph, st));
  if (P->check && !internal_data) {
    hipError_t e = launch_finite(data, int64_t(data_elems(P)) * batch, P->d_flag, st);
    if (e != hipSuccess) return fail(QPAT_E_HIP, std::string("output check: ") + hipGetErrorString(e));
  }
  return QPAT_OK;
}

qpat_status do_adjoint(qpat_plan P, const float* res, float* grad, int batch, hipStream_t st,
                       bool internal_data) {
  Exec* E = nullptr;
  STCHK(plan_exec(P, batch, &E));
  std::vector<IO> io(batch);
  for (int i = 0; i < batch; ++i) {
    io[i].in = internal_data ? P->datas[i] : res + data_elems(P) * i;
    io[i].out = grad + field_elems(P) * i;
  }
  STCHK(exec_set_io(*E, io, st));
  STCHK(exec_run(*E, OP_ADJ, P->graph, st));
  if (P->check) {
    hipError_t e = launch_finite(grad, int64_t(field_elems(P)) * batch, P->d_flag, st);
    if (e != hipSuccess) return fail(QPAT_E_HIP, std::string("output check: ") + hipGetErrorString(e));
  }
  return QPAT_OK;
}

// ---- tuning cache
std::string tune_key(qpat_plan P, int batch) {
  char buf[128];
  std::snprintf(buf, sizeof buf, "%d %d %d %d %d", P->prm.nx, P->prm.ny, batch, P->med.lossy, int(P->graph));
  return buf;
}

bool tune_lookup(const std::string& key, int* rt, int* ct, int* rthr, int* cthr) {
  const char* path = std::getenv("QPAT_TUNE_CACHE");
  if (!path) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[256];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    int a, b, c, d, g, r, co, rh, ch;
    if (std::sscanf(line, "%d %d %d %d %d %d %d %d %d", &a, &b, &c, &d, &g, &r, &co, &rh, &ch) == 9) {
      char k[128];
      std::snprintf(k, sizeof k, "%d %d %d %d %d", a, b, c, d, g);
      if (key == k) {
        *rt = r;
        *ct = co;
        *rthr = rh;
        *cthr = ch;
        found = true;
      }
    }
  }
  std::fclose(f);
  return found;
}

void tune_store(const std::string& key, int rt, int ct, int rthr, int cthr) {
  const char* path = std::getenv("QPAT_TUNE_CACHE");
  if (!path) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%s %d %d %d %d\n", key.c_str(), rt, ct, rthr, cthr);
  std::fclose(f);
}

qpat_status set_tiles(qpat_plan P, int rt, int ct, int rthr, int cthr) {
  if (!row_tile_ok(P->prm.nx, P->prm.ny, rt, rthr))
    return fail(QPAT_E_INVALID, "row tile: rows must be an even power of two dividing ny (at most ny/8 for "
                                "power-of-two ny >= 128), threads 64/128/256/512, rows*nx <= 8*threads, within "
                                "the LDS limit");
  if (!col_tile_ok(P->prm.nx / 2, P->prm.ny, ct, cthr))
    return fail(QPAT_E_INVALID, "column tile: columns must be a power of two dividing nx/2, threads "
                                "64/128/256/512, columns*ny <= 4*threads, within the LDS limit");
  if (rt != P->rt || ct != P->ct || rthr != P->rthr || cthr != P->cthr) {
    P->rt = P->med.rt = rt;
    P->ct = P->med.ct = ct;
    P->med.lrt = ilog2(rt);
    P->med.lct = ilog2(ct);
    P->med.srt = storage_rows(P->prm.ny, rt);
    P->med.lsrt = ilog2(P->med.srt);
    P->rthr = P->med.rthr = rthr;
    P->cthr = P->med.cthr = cthr;
    HIPCHK(hipDeviceSynchronize());
    P->clear_execs();
  }
  return QPAT_OK;
}

// Time a short forward + adjoint with the current tiles: the first `steps`
// forward iterates, then the adjoint iterates of the same span (every pass
// kind of both sweeps), launched the way the plan's calls launch them -
// captured in a hipGraph and replayed when graph mode is on.  Best of three.
qpat_status time_pair(qpat_plan P, int batch, int steps, hipStream_t st, float* ms) {
  Exec* E = nullptr;
  STCHK(plan_exec(P, batch, &E));
  // The adjoint writes its gradient, a field, through IO::out at iterates 0
  // and -1: it needs a field-sized buffer of its own (the per-vector data
  // buffer holds only nt * ns floats).  The forward iterates below do not
  // write IO::out (no sensor-data combine).
  float* gout = nullptr;
  HIPCHK(hipMalloc(&gout, field_elems(P) * batch * sizeof(float)));
  std::vector<IO> io(batch);
  for (int i = 0; i < batch; ++i) {
    io[i].in = P->works[i].q;  // any field-sized buffer works as p0 for timing
    io[i].out = gout + field_elems(P) * i;
  }
  qpat_status rs = exec_set_io(*E, io, st);
  if (rs != QPAT_OK) {
    (void)hipFree(gout);
    return rs;
  }
  const int nl = std::min(P->prm.nt - 2, steps);
  auto body = [&](hipStream_t s) -> hipError_t {
    for (int n = -1; n <= nl; ++n) LCHK(fwd_iterate(*E, n, 0, s));
    for (int n = nl; n >= -1; --n) LCHK(adj_iterate(*E, n, 0, s));
    return hipSuccess;
  };
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  const bool use_graph = P->graph && st != nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess && use_graph) {
    e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      hipError_t e1 = body(st);
      e = hipStreamEndCapture(st, &g);
      if (e == hipSuccess) e = e1;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
  }
  auto launch = [&]() -> hipError_t { return use_graph ? hipGraphLaunch(ge, st) : body(st); };
  if (e == hipSuccess) e = launch();  // warm-up
  *ms = INFINITY;
  for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {  // best of three: the candidates differ by a few %
    float t = 0.f;
    e = hipEventRecord(a, st);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess) e = hipEventRecord(b, st);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
    if (e == hipSuccess) *ms = std::min(*ms, t);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);  // the launches are done with gout
  if (ge) (void)hipGraphExecDestroy(ge);
  if (g) (void)hipGraphDestroy(g);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipFree(gout);
  if (e != hipSuccess) return fail(QPAT_E_HIP, std::string("tune timing: ") + hipGetErrorString(e));
  return QPAT_OK;
}

}  // namespace

// ============================================================== C API
extern "C" {

const char* qpat_status_string(qpat_status s) {
  switch (s) {
    case QPAT_OK: return "ok";
    case QPAT_E_INVALID: return "invalid argument";
    case QPAT_E_UNSUPPORTED: return "unsupported configuration";
    case QPAT_E_UNSTABLE: return "time step above the stability bound";
    case QPAT_E_HIP: return "HIP runtime error";
    case QPAT_E_OOM: return "out of memory";
    case QPAT_E_NONFINITE: return "non-finite output";
  }
  return "unknown status";
}

const char* qpat_last_error(void) { return g_err.c_str(); }

qpat_status qpat_validate(const qpat_params* prm) { return validate(prm); }

qpat_status qpat_plan_create(const qpat_params* prm, const double* c0, const double* rho0, qpat_plan* out) {
  if (!out) return fail(QPAT_E_INVALID, "out is NULL");
  *out = nullptr;
  STCHK(validate(prm));
  if (!c0 || !rho0) return fail(QPAT_E_INVALID, "c0 / rho0 is NULL");
  qpat_plan P = new qpat_plan_s();
  P->prm = *prm;
  P->sensors.assign(prm->sensor_xy, prm->sensor_xy + 2 * size_t(prm->ns));
  P->prm.sensor_xy = P->sensors.data();
  qpat_status s = plan_build(P, c0, rho0);
  if (s != QPAT_OK) {
    qpat_plan_destroy(P);
    return s;
  }
  *out = P;
  return QPAT_OK;
}

void qpat_plan_destroy(qpat_plan P) {
  if (!P) return;
  (void)hipDeviceSynchronize();
  P->clear_execs();
  if (P->d_work) (void)hipFree(P->d_work);
  if (P->d_med) (void)hipFree(P->d_med);
  if (P->d_flag) (void)hipFree(P->d_flag);
  delete P;
}

qpat_status qpat_set_check(qpat_plan P, int32_t enable) {
  if (!P) return fail(QPAT_E_INVALID, "plan is NULL");
  if (enable && !P->d_flag) {
    HIPCHK(hipMalloc(&P->d_flag, sizeof(int)));
    HIPCHK(hipMemset(P->d_flag, 0, sizeof(int)));
  }
  P->check = enable != 0;
  return QPAT_OK;
}

qpat_status qpat_check(qpat_plan P, qpat_stream stream) {
  if (!P) return fail(QPAT_E_INVALID, "plan is NULL");
  if (!P->d_flag) return QPAT_OK;
  hipStream_t st = (hipStream_t)stream;
  int flag = 0;
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipMemcpy(&flag, P->d_flag, sizeof(int), hipMemcpyDeviceToHost));
  if (!flag) return QPAT_OK;
  HIPCHK(hipMemset(P->d_flag, 0, sizeof(int)));
  return fail(QPAT_E_NONFINITE, "a solve output held NaN or Inf values");
}

qpat_status qpat_forward(qpat_plan P, const float* p0, float* data, int32_t batch, qpat_stream stream) {
  const TraceRange trace_("qpat_forward");
  STCHK(check_plan_call(P, p0, data, batch));
  return do_forward(P, p0, data, batch, (hipStream_t)stream, false);
}

qpat_status qpat_jv(qpat_plan P, const float* v, float* data, int32_t batch, qpat_stream stream) {
  return qpat_forward(P, v, data, batch, stream);
}

qpat_status qpat_adjoint(qpat_plan P, const float* res, float* grad, int32_t batch, qpat_stream stream) {
  const TraceRange trace_("qpat_adjoint");
  STCHK(check_plan_call(P, res, grad, batch));
  return do_adjoint(P, res, grad, batch, (hipStream_t)stream, false);
}

qpat_status qpat_jtjv(qpat_plan P, const float* v, float* out, int32_t batch, qpat_stream stream) {
  const TraceRange trace_("qpat_jtjv");
  STCHK(check_plan_call(P, v, out, batch));
  STCHK(do_forward(P, v, nullptr, batch, (hipStream_t)stream, true));
  return do_adjoint(P, nullptr, out, batch, (hipStream_t)stream, true);
}

qpat_status qpat_jtjv_data(qpat_plan P, const float* v, float* jv, float* out, int32_t batch, qpat_stream stream) {
  const TraceRange trace_("qpat_jtjv_data");
  STCHK(check_plan_call(P, v, out, batch));
  if (!jv) return fail(QPAT_E_INVALID, "jv is NULL");
  STCHK(do_forward(P, v, jv, batch, (hipStream_t)stream, false));
  return do_adjoint(P, jv, out, batch, (hipStream_t)stream, false);
}

qpat_status qpat_apply(qpat_plan P, int32_t op, const float* in, float* out, int32_t batch, qpat_stream stream) {
  STCHK(check_plan_call(P, in, out, batch));
  static const int codes[6] = {MC_DXP, MC_DXM, MC_DYP, MC_DYM, MC_LDIS, MC_LABS};
  if (op < 0 || op > 5) return fail(QPAT_E_INVALID, "unknown operator");
  if ((op == QPAT_OP_YDIS || op == QPAT_OP_YABS) && !P->med.lossy)
    return fail(QPAT_E_INVALID, "Y_dis / Y_abs need a lossy plan (alpha0_db > 0)");
  hipStream_t st = (hipStream_t)stream;
  Exec* E = nullptr;
  STCHK(plan_exec(P, batch, &E));
  std::vector<IO> io(batch);
  for (int i = 0; i < batch; ++i) {
    io[i].in = in + field_elems(P) * i;
    io[i].out = out + field_elems(P) * i;
  }
  STCHK(exec_set_io(*E, io, st));
  hipError_t e = row(*E, RM_FWD1, -1, 0, st);
  if (e == hipSuccess) e = col(*E, CM_APPLY, -1, st, mpack(codes[op], 0, 0, 0));
  if (e == hipSuccess) e = row(*E, RM_INV1, -1, 0, st);
  if (e != hipSuccess) return fail(QPAT_E_HIP, std::string("apply: ") + hipGetErrorString(e));
  return QPAT_OK;
}

qpat_status qpat_ckpt_bytes(qpat_plan P, int32_t K, int32_t batch, size_t* bytes) {
  if (!P || !bytes) return fail(QPAT_E_INVALID, "plan / bytes is NULL");
  if (K < 1) return fail(QPAT_E_INVALID, "interval must be >= 1");
  if (batch < 1) return fail(QPAT_E_INVALID, "batch must be >= 1");
  const size_t nck = (size_t(P->prm.nt) + K - 1) / K;
  *bytes = size_t(batch) * nck * 5 * field_elems(P) * sizeof(float);
  return QPAT_OK;
}

qpat_status qpat_forward_ckpt(qpat_plan P, const float* p0, float* data, int32_t K, float* ckpt,
                              int32_t batch, qpat_stream stream) {
  const TraceRange trace_("qpat_forward_ckpt");
  STCHK(check_plan_call(P, p0, data, batch));
  if (!ckpt) return fail(QPAT_E_INVALID, "ckpt is NULL");
  if (K < 1) return fail(QPAT_E_INVALID, "interval must be >= 1");
  hipStream_t st = (hipStream_t)stream;
  Exec* E = nullptr;
  STCHK(plan_exec(P, batch, &E));
  std::vector<IO> io(batch);
  for (int i = 0; i < batch; ++i) {
    io[i].in = p0 + field_elems(P) * i;
    io[i].out = data + data_elems(P) * i;
  }
  STCHK(exec_set_io(*E, io, st));
  const size_t N = field_elems(P), nck = (size_t(P->prm.nt) + K - 1) / K;
  for (int n = -1; n <= P->prm.nt - 2; ++n) {
    const int m = n + 1;
    const bool store = (m % K) == 0;
    hipError_t e = fwd_iterate(*E, n, store ? FL_STORE_P : 0, st);
    if (e != hipSuccess) return fail(QPAT_E_HIP, std::string("forward_ckpt: ") + hipGetErrorString(e));
    if (store)
      for (int i = 0; i < batch; ++i)
        HIPCHK(hipMemcpyAsync(ckpt + (size_t(i) * nck + m / K) * 5 * N, P->works[i].f0, 5 * N * sizeof(float),
                              hipMemcpyDeviceToDevice, st));
  }
  hipError_t e = launch_combine(E->d_items, E->d_io, batch, E->max_data, st);
  if (e != hipSuccess) return fail(QPAT_E_HIP, std::string("forward_ckpt: ") + hipGetErrorString(e));
  return QPAT_OK;
}

qpat_status qpat_replay(qpat_plan P, const float* p0, const float* ckpt, int32_t K, int32_t seg,
                        float* states, int32_t batch, qpat_stream stream) {
  STCHK(check_plan_call(P, ckpt, states, batch));
  if (!p0) return fail(QPAT_E_INVALID, "p0 is NULL");
  if (K < 1) return fail(QPAT_E_INVALID, "interval must be >= 1");
  const int nt = P->prm.nt;
  const int nck = (nt + K - 1) / K;
  if (seg < 0 || seg >= nck) return fail(QPAT_E_INVALID, "segment out of range");
  hipStream_t st = (hipStream_t)stream;
  Exec* E = nullptr;
  STCHK(plan_exec(P, batch, &E));
  const size_t N = field_elems(P);
  const int m0 = seg * K, cnt = std::min(K, nt - m0);
  // restore z_{m0} and the spectrum of its pressure
  for (int i = 0; i < batch; ++i)
    HIPCHK(hipMemcpyAsync(P->works[i].f0, ckpt + (size_t(i) * nck + seg) * 5 * N, 5 * N * sizeof(float),
                          hipMemcpyDeviceToDevice, st));
  std::vector<IO> io(batch);
  for (int i = 0; i < batch; ++i) {
    io[i].in = P->works[i].q;
    io[i].out = nullptr;
  }
  STCHK(exec_set_io(*E, io, st));
  hipError_t e = row(*E, RM_FWD1, -1, 0, st);
  if (e != hipSuccess) return fail(QPAT_E_HIP, std::string("replay: ") + hipGetErrorString(e));
  for (int i = 0; i < batch; ++i) {
    io[i].in = p0 + N * i;
    io[i].out = nullptr;
  }
  STCHK(exec_set_io(*E, io, st));
  for (int c = 0; c < cnt; ++c) {
    if (c > 0) {
      e = fwd_iterate(*E, m0 + c - 1, FL_STORE_P | FL_NO_SENSORS, st);
      if (e != hipSuccess) return fail(QPAT_E_HIP, std::string("replay: ") + hipGetErrorString(e));
    }
    for (int i = 0; i < batch; ++i)
      HIPCHK(hipMemcpyAsync(states + (size_t(i) * cnt + c) * 5 * N, P->works[i].f0, 5 * N * sizeof(float),
                            hipMemcpyDeviceToDevice, st));
  }
  return QPAT_OK;
}

// ---- sound-speed gradient (checkpointed forward correlated with the adjoint)
namespace {

// Segment j of the time axis holds the pressures p^m, m in [lo_j, hi_j]:
// segment 0 starts at m = 0 (recomputed from p0 alone), segment j >= 1 at
// m = jK + 1 (recomputed from the checkpointed state at m = jK).  The
// sensitivity of p^m sits at slot m - jK.
struct GradLayout {
  int nseg = 0, slots = 0;
  size_t gc_off = 0, sens_off = 0, ck_off = 0, total = 0;
};

size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

GradLayout grad_layout(qpat_plan P, int K, int batch) {
  const int nt = P->prm.nt;
  const size_t N = field_elems(P), B = size_t(batch);
  GradLayout g;
  g.nseg = nt >= 2 ? 1 + (nt - 2) / K : 1;
  g.slots = std::min(K, nt - 1) + 1;
  g.gc_off = 0;
  g.sens_off = round256(B * N * sizeof(double));
  g.ck_off = round256(g.sens_off + B * size_t(g.slots) * N * sizeof(float));
  g.total = g.ck_off + B * size_t(g.nseg - 1) * 5 * N * sizeof(float);
  return g;
}

qpat_status grad_execs(qpat_plan P, int b, Exec** ef, Exec** ea) {
  STCHK(plan_reserve(P, 2 * b));
  auto it = P->grad_execs.find(b);
  if (it == P->grad_execs.end()) {
    std::vector<Item> fi(b), ai(b);
    for (int i = 0; i < b; ++i) {
      fi[i].m = ai[i].m = P->med;
      fi[i].w = P->works[i];
      ai[i].w = P->works[b + i];
    }
    std::unique_ptr<Exec> f(new Exec()), a(new Exec());
    STCHK(exec_build(*f, fi));
    STCHK(exec_build(*a, ai));
    it = P->grad_execs.emplace(b, std::make_pair(std::move(f), std::move(a))).first;
  }
  *ef = it->second.first.get();
  *ea = it->second.second.get();
  return QPAT_OK;
}

// The forward state that iterate m + 1 starts from: v_x, v_y, rho_x, rho_y
// (4 fields) and the half spectrum of p^m (ny * nx/2 complex = one field).
hipError_t state_copy(const Work& w, float* ck, size_t N, bool save, hipStream_t st) {
  const size_t fb = 4 * N * sizeof(float), sb = N * sizeof(float);
  hipError_t e = save ? hipMemcpyAsync(ck, w.f0, fb, hipMemcpyDeviceToDevice, st)
                      : hipMemcpyAsync(w.f0, ck, fb, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  return save ? hipMemcpyAsync(ck + 4 * N, w.s0, sb, hipMemcpyDeviceToDevice, st)
              : hipMemcpyAsync(w.s0, ck + 4 * N, sb, hipMemcpyDeviceToDevice, st);
}

}  // namespace

qpat_status qpat_medium_grad_bytes(qpat_plan P, int32_t K, int32_t batch, size_t* bytes) {
  if (!P || !bytes) return fail(QPAT_E_INVALID, "plan / bytes is NULL");
  if (K < 1) return fail(QPAT_E_INVALID, "interval must be >= 1");
  if (batch < 1 || batch > 4096) return fail(QPAT_E_INVALID, "batch must be in [1, 4096]");
  *bytes = grad_layout(P, K, batch).total;
  return QPAT_OK;
}

qpat_status qpat_medium_grad(qpat_plan P, const float* p0, const float* res, int32_t K, void* work,
                             float* grad_p0, float* grad_c, int32_t batch, qpat_stream stream) {
  const TraceRange trace_("qpat_medium_grad");
  STCHK(check_plan_call(P, p0, res, batch));
  if (!work || !grad_p0 || !grad_c) return fail(QPAT_E_INVALID, "work / grad_p0 / grad_c is NULL");
  if (K < 1) return fail(QPAT_E_INVALID, "interval must be >= 1");
  const GradLayout g = grad_layout(P, K, batch);
  if (g.slots >= (1 << (30 - kSlotShift))) return fail(QPAT_E_INVALID, "interval too long");
  hipStream_t st = (hipStream_t)stream;
  Exec *Ef = nullptr, *Ea = nullptr;
  STCHK(grad_execs(P, batch, &Ef, &Ea));
  const int nt = P->prm.nt;
  const size_t N = field_elems(P), D = data_elems(P);
  char* w = static_cast<char*>(work);
  double* gc = reinterpret_cast<double*>(w + g.gc_off);
  float* sens = reinterpret_cast<float*>(w + g.sens_off);
  float* ck = reinterpret_cast<float*>(w + g.ck_off);
  auto ckpt = [&](int i, int j) { return ck + (size_t(i) * (g.nseg - 1) + (j - 1)) * 5 * N; };
  std::vector<IO> iof(batch), ioa(batch);
  for (int i = 0; i < batch; ++i) {
    iof[i] = IO{p0 + N * i, nullptr, sens + size_t(i) * g.slots * N, nullptr};
    ioa[i] = IO{res + D * i, grad_p0 + N * i, sens + size_t(i) * g.slots * N, gc + N * i};
  }
  STCHK(exec_set_io(*Ef, iof, st));
  STCHK(exec_set_io(*Ea, ioa, st));
  auto run = [&]() -> hipError_t {
    // forward sweep: the states at m = jK, j = 1 .. nseg - 1
    for (int m = 0; m <= (g.nseg - 1) * K && g.nseg > 1; ++m) {
      LCHK(fwd_iterate(*Ef, m - 1, FL_NO_SENSORS, st));
      if (m > 0 && m % K == 0)
        for (int i = 0; i < batch; ++i) LCHK(state_copy(P->works[i], ckpt(i, m / K), N, true, st));
    }
    // reverse sweep, one segment at a time: recompute its sensitivities, then
    // run its adjoint iterates
    LCHK(launch_tap_order(Ea->d_items, Ea->d_io, batch, 2 * Ea->max_data, st));
    for (int j = g.nseg - 1; j >= 0; --j) {
      const int base = j * K, lo = j == 0 ? 0 : base + 1, hi = std::min(base + K, nt - 1);
      if (j > 0)
        for (int i = 0; i < batch; ++i) LCHK(state_copy(P->works[i], ckpt(i, j), N, false, st));
      for (int m = lo; m <= hi; ++m)
        LCHK(fwd_iterate(*Ef, m - 1, FL_NO_SENSORS | ((m - base) << kSlotShift), st, true));
      for (int m = hi; m >= lo; --m) LCHK(adj_iterate(*Ea, m - 1, (m - base) << kSlotShift, st, true));
    }
    return launch_grad_c(P->med.c2, p0, grad_p0, gc, (long long)N, batch, (long long)N, grad_c, st);
  };
  const hipError_t e = run();
  if (e != hipSuccess) return fail(QPAT_E_HIP, std::string("medium_grad: ") + hipGetErrorString(e));
  return QPAT_OK;
}

qpat_status qpat_set_tiles(qpat_plan P, int32_t rows, int32_t cols, int32_t row_threads,
                           int32_t col_threads) {
  if (!P) return fail(QPAT_E_INVALID, "plan is NULL");
  return set_tiles(P, rows, cols, row_threads, col_threads);
}

qpat_status qpat_get_tiles(qpat_plan P, int32_t* rows, int32_t* cols, int32_t* row_threads,
                           int32_t* col_threads) {
  if (!P || !rows || !cols) return fail(QPAT_E_INVALID, "NULL argument");
  *rows = P->rt;
  *cols = P->ct;
  if (row_threads) *row_threads = P->rthr;
  if (col_threads) *col_threads = P->cthr;
  return QPAT_OK;
}

qpat_status qpat_tune(qpat_plan P, int32_t batch, qpat_stream stream) {
  const TraceRange trace_("qpat_tune");
  if (!P) return fail(QPAT_E_INVALID, "plan is NULL");
  if (batch < 1) return fail(QPAT_E_INVALID, "batch must be >= 1");
  const std::string key = tune_key(P, batch);
  const int nx = P->prm.nx, ny = P->prm.ny;
  int rt, ct, rh, ch;
  if (tune_lookup(key, &rt, &ct, &rh, &ch) && row_tile_ok(nx, ny, rt, rh) && col_tile_ok(nx / 2, ny, ct, ch))
    return set_tiles(P, rt, ct, rh, ch);
  hipStream_t st = (hipStream_t)stream;
  const int steps = 16;
  int brt = P->rt, bct = P->ct, brh = P->rthr, bch = P->cthr;
  struct Cand {
    float ms;
    int rt, ct, rh, ch;
  };
  std::vector<Cand> seen;
  float best = INFINITY;
  // row shapes first (column shape fixed), then column shapes with the best row shape
  for (int r = 2; r <= 32; r *= 2)
    for (int h = 64; h <= kMaxThreads; h *= 2) {
      if (!row_tile_ok(nx, ny, r, h)) continue;
      STCHK(set_tiles(P, r, bct, h, bch));
      float ms;
      STCHK(time_pair(P, batch, steps, st, &ms));
      seen.push_back({ms, r, bct, h, bch});
      if (ms < best) {
        best = ms;
        brt = r;
        brh = h;
      }
    }
  best = INFINITY;
  for (int c = 1; c <= 32; c *= 2)
    for (int h = 64; h <= kMaxThreads; h *= 2) {
      if (!col_tile_ok(nx / 2, ny, c, h)) continue;
      STCHK(set_tiles(P, brt, c, brh, h));
      float ms;
      STCHK(time_pair(P, batch, steps, st, &ms));
      seen.push_back({ms, brt, c, brh, h});
      if (ms < best) {
        best = ms;
        bct = c;
        bch = h;
      }
    }
  // the sweeps' short runs separate shapes only to a few percent: the three
  // fastest distinct shapes are timed again over at least three times the
  // iterates and at least ~20 ms of work each (at 512^2, one vector, 48
  // iterates are 3.5 ms, too short to order shapes 0.7% apart)
  std::sort(seen.begin(), seen.end(), [](const Cand& a, const Cand& b) { return a.ms < b.ms; });
  std::vector<Cand> top;
  for (const Cand& c : seen) {
    bool dup = false;
    for (const Cand& t : top) dup = dup || (t.rt == c.rt && t.ct == c.ct && t.rh == c.rh && t.ch == c.ch);
    if (!dup) top.push_back(c);
    if (top.size() == 3) break;
  }
  best = INFINITY;
  const float ms0 = top.empty() ? 0.f : top[0].ms;
  const int steps2 = ms0 > 0.f ? std::max(3 * steps, int(std::min(4096.f, std::ceil(steps * 20.f / ms0)))) : 3 * steps;
  for (const Cand& c : top) {
    STCHK(set_tiles(P, c.rt, c.ct, c.rh, c.ch));
    float ms;
    STCHK(time_pair(P, batch, steps2, st, &ms));
    if (ms < best) {
      best = ms;
      brt = c.rt;
      bct = c.ct;
      brh = c.rh;
      bch = c.ch;
    }
  }
  STCHK(set_tiles(P, brt, bct, brh, bch));
  tune_store(key, brt, bct, brh, bch);
  return QPAT_OK;
}

// One pass kind of the forward (0-5) or adjoint (6-11) iterate, see qpat.h.
static hipError_t launch_pass(Exec& E, int pass, int n, hipStream_t st) {
  switch (pass) {
    case 0: return col(E, CM_GRADP1, n, st);
    case 1: return row(E, RM_F1, n, 0, st);
    case 2: return col(E, CM_GRADM2, n, st);
    case 3: return row(E, E.lossy ? RM_F2 : RM_F2L, n, 0, st);
    case 4: return col(E, CM_FRAC, n, st);
    case 5: return row(E, RM_F3, n, 0, st);
    case 6: return row(E, E.lossy ? RM_A1 : RM_A1L, n, 0, st);
    case 7: return col(E, CM_FRAC, n, st);
    case 8: return row(E, RM_A2, n, 0, st);
    case 9: return col(E, CM_GRADP2, n, st);
    case 10: return row(E, RM_A3, n, 0, st);
    case 11: return col(E, CM_DIVM, n, st);
    default: return hipErrorInvalidValue;
  }
}

qpat_status qpat_time_pass(qpat_plan P, int32_t pass, int32_t batch, int32_t reps, qpat_stream stream,
                           float* ms_per_launch) {
  if (!P || !ms_per_launch) return fail(QPAT_E_INVALID, "NULL argument");
  if (pass < 0 || pass > 11) return fail(QPAT_E_INVALID, "pass must be in [0, 11]");
  if (!P->med.lossy && (pass == 4 || pass == 5 || pass == 7 || pass == 8))
    return fail(QPAT_E_INVALID, "this pass exists only for lossy plans");
  if (batch < 1 || reps < 1) return fail(QPAT_E_INVALID, "batch and reps must be >= 1");
  hipStream_t st = (hipStream_t)stream;
  Exec* E = nullptr;
  STCHK(plan_exec(P, batch, &E));
  // IO::out of an adjoint pass is a field (written at iterates 0 and -1),
  // IO::in of a forward pass too (read at -1 and 0): field-sized buffers
  float* fbuf = nullptr;
  HIPCHK(hipMalloc(&fbuf, field_elems(P) * batch * sizeof(float)));
  HIPCHK(hipMemset(fbuf, 0, field_elems(P) * batch * sizeof(float)));
  std::vector<IO> io(batch);
  for (int i = 0; i < batch; ++i) {
    io[i].in = fbuf + field_elems(P) * i;
    io[i].out = fbuf + field_elems(P) * i;
  }
  qpat_status rs = exec_set_io(*E, io, st);
  if (rs != QPAT_OK) {
    (void)hipFree(fbuf);
    return rs;
  }
  const int n = std::min(1, P->prm.nt - 2);
  hipEvent_t a, b;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  hipError_t e = launch_pass(*E, pass, n, st);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(a, st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_pass(*E, pass, n, st);
  if (e == hipSuccess) e = hipEventRecord(b, st);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipFree(fbuf);
  if (e != hipSuccess) return fail(QPAT_E_HIP, std::string("time_pass: ") + hipGetErrorString(e));
  *ms_per_launch = ms / reps;
  return QPAT_OK;
}

qpat_status qpat_set_graph(qpat_plan P, int32_t enable) {
  if (!P) return fail(QPAT_E_INVALID, "plan is NULL");
  P->graph = enable != 0;
  return QPAT_OK;
}

qpat_status qpat_plan_info(qpat_plan P, int32_t* nx, int32_t* ny, int32_t* nt, int32_t* ns, size_t* bytes) {
  if (!P) return fail(QPAT_E_INVALID, "plan is NULL");
  if (nx) *nx = P->prm.nx;
  if (ny) *ny = P->prm.ny;
  if (nt) *nt = P->prm.nt;
  if (ns) *ns = P->prm.ns;
  if (bytes) *bytes = P->med_bytes + P->work_item_bytes * P->cap;
  return QPAT_OK;
}

// ---- uneven batches
// (Re)build the groups of a batch for its schedule from the plans' current
// media and launch shapes.
static qpat_status batch_build(qpat_batch B) {
  B->release_groups();
  const int count = int(B->plans.size());
  std::vector<std::vector<int>> members;
  if (B->schedule == 0) {
    members.emplace_back();
    for (int i = 0; i < count; ++i) members[0].push_back(i);
  } else {
    std::map<std::pair<int, int>, int> cls;
    for (int i = 0; i < count; ++i) {
      const auto key = std::make_pair(B->plans[i]->prm.nx, B->plans[i]->prm.ny);
      auto it = cls.find(key);
      if (it == cls.end()) {
        it = cls.emplace(key, int(members.size())).first;
        members.emplace_back();
      }
      members[it->second].push_back(i);
    }
  }
  for (auto& mem : members) {
    std::unique_ptr<qpat_batch_s::Group> g(new qpat_batch_s::Group());
    g->members = mem;
    std::vector<Item> items(mem.size());
    for (size_t k = 0; k < mem.size(); ++k) {
      items[k].m = B->plans[mem[k]]->med;
      items[k].w = B->works[mem[k]];
    }
    STCHK(exec_build(g->exec, items));
    if (members.size() > 1) {
      HIPCHK(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
      HIPCHK(hipEventCreateWithFlags(&g->done, hipEventDisableTiming));
    }
    B->groups.push_back(std::move(g));
  }
  return QPAT_OK;
}

qpat_status qpat_batch_create(const qpat_plan* plans, int32_t count, qpat_batch* out) {
  if (!out) return fail(QPAT_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!plans || count < 1) return fail(QPAT_E_INVALID, "need at least one plan");
  for (int i = 0; i < count; ++i) {
    if (!plans[i]) return fail(QPAT_E_INVALID, "plan " + std::to_string(i) + " is NULL");
    if (plans[i]->med.lossy != plans[0]->med.lossy)
      return fail(QPAT_E_UNSUPPORTED, "a batch must be all lossy or all lossless");
    for (int j = 0; j < i; ++j)
      if (plans[j] == plans[i]) return fail(QPAT_E_INVALID, "a plan may appear only once in a batch");
  }
  std::unique_ptr<qpat_batch_s> B(new qpat_batch_s());
  B->plans.assign(plans, plans + count);
  for (int i = 0; i < count; ++i) {
    void* blk = nullptr;
    size_t per = 0;
    std::vector<Work> w;
    std::vector<float*> dd;
    STCHK(alloc_works(plans[i]->prm, 1, &blk, &per, w, dd));
    B->blocks.push_back(blk);
    B->works.push_back(w[0]);
    B->datas.push_back(dd[0]);
  }
  HIPCHK(hipEventCreateWithFlags(&B->fork, hipEventDisableTiming));
  STCHK(batch_build(B.get()));
  *out = B.release();
  return QPAT_OK;
}

void qpat_batch_destroy(qpat_batch B) {
  if (!B) return;
  (void)hipDeviceSynchronize();
  delete B;
}

static qpat_status batch_io(qpat_batch B, const float* const* in, float* const* out, bool internal_in,
                            bool internal_out, hipStream_t st) {
  for (auto& g : B->groups) {
    std::vector<IO> io(g->members.size());
    for (size_t k = 0; k < g->members.size(); ++k) {
      const int i = g->members[k];
      io[k].in = internal_in ? B->datas[i] : in[i];
      io[k].out = internal_out ? B->datas[i] : out[i];
      if (!io[k].in || !io[k].out) return fail(QPAT_E_INVALID, "NULL pointer in batch arrays");
    }
    STCHK(exec_set_io(g->exec, io, st));
  }
  return QPAT_OK;
}

// The forward or adjoint sweep of every group: on `st` for one group, else
// forked onto the groups' streams and joined back into `st`.
static hipError_t batch_body(qpat_batch B, int op, hipStream_t st) {
  auto sweep = [&](Exec& E, hipStream_t s) {
    return op == OP_FWD ? seq_forward(E, E.max_nt - 2, s) : seq_adjoint(E, s);
  };
  if (B->groups.size() == 1) return sweep(B->groups[0]->exec, st);
  LCHK(hipEventRecord(B->fork, st));
  for (auto& g : B->groups) {
    LCHK(hipStreamWaitEvent(g->stream, B->fork, 0));
    LCHK(sweep(g->exec, g->stream));
    LCHK(hipEventRecord(g->done, g->stream));
  }
  for (auto& g : B->groups) LCHK(hipStreamWaitEvent(st, g->done, 0));
  return hipSuccess;
}

static qpat_status batch_run(qpat_batch B, int op, hipStream_t st) {
  if (!B->graph || st == nullptr) {
    hipError_t e = batch_body(B, op, st);
    if (e != hipSuccess) return fail(QPAT_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
    return QPAT_OK;
  }
  auto it = B->graphs.find(op);
  if (it == B->graphs.end()) {
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    hipError_t e = batch_body(B, op, st);
    hipError_t e2 = hipStreamEndCapture(st, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(QPAT_E_HIP, std::string("graph capture: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    HIPCHK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
    it = B->graphs.emplace(op, std::make_pair(g, ge)).first;
  }
  HIPCHK(hipGraphLaunch(it->second.second, st));
  return QPAT_OK;
}

qpat_status qpat_batch_forward(qpat_batch B, const float* const* p0, float* const* data, qpat_stream stream) {
  const TraceRange trace_("qpat_batch_forward");
  if (!B || !p0 || !data) return fail(QPAT_E_INVALID, "NULL argument");
  STCHK(batch_io(B, p0, data, false, false, (hipStream_t)stream));
  return batch_run(B, OP_FWD, (hipStream_t)stream);
}

qpat_status qpat_batch_adjoint(qpat_batch B, const float* const* res, float* const* grad, qpat_stream stream) {
  const TraceRange trace_("qpat_batch_adjoint");
  if (!B || !res || !grad) return fail(QPAT_E_INVALID, "NULL argument");
  STCHK(batch_io(B, res, grad, false, false, (hipStream_t)stream));
  return batch_run(B, OP_ADJ, (hipStream_t)stream);
}

qpat_status qpat_batch_jtjv(qpat_batch B, const float* const* v, float* const* out, qpat_stream stream) {
  const TraceRange trace_("qpat_batch_jtjv");
  if (!B || !v || !out) return fail(QPAT_E_INVALID, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  STCHK(batch_io(B, v, nullptr, false, true, st));
  STCHK(batch_run(B, OP_FWD, st));
  STCHK(batch_io(B, nullptr, out, true, false, st));
  return batch_run(B, OP_ADJ, st);
}

qpat_status qpat_batch_set_graph(qpat_batch B, int32_t enable) {
  if (!B) return fail(QPAT_E_INVALID, "batch is NULL");
  B->graph = enable != 0;
  return QPAT_OK;
}

qpat_status qpat_batch_set_schedule(qpat_batch B, int32_t schedule) {
  if (!B) return fail(QPAT_E_INVALID, "batch is NULL");
  if (schedule != 0 && schedule != 1) return fail(QPAT_E_INVALID, "schedule must be 0 or 1");
  (void)hipDeviceSynchronize();  // the groups' buffers may still be in use
  B->schedule = schedule;
  return batch_build(B);
}

qpat_status qpat_batch_get_schedule(qpat_batch B, int32_t* schedule) {
  if (!B || !schedule) return fail(QPAT_E_INVALID, "NULL argument");
  *schedule = B->schedule;
  return QPAT_OK;
}

qpat_status qpat_batch_tune(qpat_batch B, qpat_stream stream) {
  const TraceRange trace_("qpat_batch_tune");
  if (!B) return fail(QPAT_E_INVALID, "batch is NULL");
  hipStream_t st = (hipStream_t)stream;
  // launch shapes: per grid size, tuned on its first plan for the number of
  // problems of that size and given to every plan of that size
  std::map<std::pair<int, int>, std::vector<qpat_plan>> cls;
  for (qpat_plan P : B->plans) cls[{P->prm.nx, P->prm.ny}].push_back(P);
  for (auto& c : cls) {
    qpat_plan P0 = c.second[0];
    const bool g0 = P0->graph;
    P0->graph = B->graph;
    qpat_status s = qpat_tune(P0, int32_t(c.second.size()), stream);
    P0->graph = g0;
    STCHK(s);
    for (qpat_plan P : c.second) STCHK(set_tiles(P, P0->rt, P0->ct, P0->rthr, P0->cthr));
  }
  // schedule: a full forward + adjoint of the batch under each, best of two
  std::vector<size_t> goff(B->plans.size());
  size_t gtot = 0;
  for (size_t i = 0; i < B->plans.size(); ++i) {
    goff[i] = gtot;
    gtot += size_t(B->plans[i]->prm.nx) * B->plans[i]->prm.ny;
  }
  float* gbuf = nullptr;
  HIPCHK(hipMalloc(&gbuf, gtot * sizeof(float)));
  float best = INFINITY;
  int best_s = 0;
  hipEvent_t a = nullptr, b = nullptr;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  qpat_status rc = QPAT_OK;
  for (int sch = 0; sch < 2 && rc == QPAT_OK; ++sch) {
    B->schedule = sch;
    (void)hipStreamSynchronize(st);
    rc = batch_build(B);
    if (rc != QPAT_OK) break;
    std::vector<const float*> in(B->plans.size());
    std::vector<float*> outp(B->plans.size());
    for (size_t i = 0; i < B->plans.size(); ++i) {
      in[i] = B->works[i].q;        // any field-sized buffer works as p0 for timing
      outp[i] = gbuf + goff[i];     // gradients: field-sized buffers of their own
    }
    for (int rep = 0; rep < 3 && rc == QPAT_OK; ++rep) {  // warm-up (and graph capture), then two timed
      float t = 0.f;
      hipError_t e = hipEventRecord(a, st);
      if (e == hipSuccess) {
        rc = batch_io(B, in.data(), nullptr, false, true, st);
        if (rc == QPAT_OK) rc = batch_run(B, OP_FWD, st);
        if (rc == QPAT_OK) rc = batch_io(B, nullptr, outp.data(), true, false, st);
        if (rc == QPAT_OK) rc = batch_run(B, OP_ADJ, st);
      }
      if (rc != QPAT_OK) break;
      if (e == hipSuccess) e = hipEventRecord(b, st);
      if (e == hipSuccess) e = hipEventSynchronize(b);
      if (e == hipSuccess) e = hipEventElapsedTime(&t, a, b);
      if (e != hipSuccess) rc = fail(QPAT_E_HIP, std::string("batch tune timing: ") + hipGetErrorString(e));
      if (rc == QPAT_OK && rep > 0 && t < best) {
        best = t;
        best_s = sch;
      }
    }
  }
  (void)hipStreamSynchronize(st);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipFree(gbuf);
  STCHK(rc);
  B->schedule = best_s;
  return batch_build(B);
}

// ---- reductions
qpat_status qpat_dot(const float* a, const float* b, int64_t n, double* out, qpat_stream stream) {
  if (!out) return fail(QPAT_E_INVALID, "out is NULL");
  if (n < 0) return fail(QPAT_E_INVALID, "n must be >= 0");
  if (n > 0 && (!a || !b)) return fail(QPAT_E_INVALID, "NULL input with n > 0");
  // partial sums: one buffer per (device, stream), so calls on different
  // streams never share one; calls on one stream are ordered by it
  static std::mutex mu;
  static std::map<std::pair<int, void*>, double*> partials;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  double* part = nullptr;
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = partials.find({dev, stream});
    if (it == partials.end()) {
      HIPCHK(hipMalloc(&part, kDotBlocks * sizeof(double)));
      partials[{dev, stream}] = part;
    } else {
      part = it->second;
    }
  }
  const int nblk = dot_blocks(n);
  hipError_t e = launch_dot(a, b, n, part, nblk, out, (hipStream_t)stream);
  if (e != hipSuccess) return fail(QPAT_E_HIP, std::string("dot: ") + hipGetErrorString(e));
  return QPAT_OK;
}

qpat_status qpat_dot_noalloc(const float* a, const float* b, int64_t n, double* out, qpat_stream stream) {
  if (!out) return fail(QPAT_E_INVALID, "out is NULL");
  if (n < 0) return fail(QPAT_E_INVALID, "n must be >= 0");
  if (n > kDotNoallocMaxN) return fail(QPAT_E_INVALID, "n exceeds 2^40, the largest length qpat_dot_noalloc takes");
  if (n > 0 && (!a || !b)) return fail(QPAT_E_INVALID, "NULL input with n > 0");
  double* part = nullptr;
  hipError_t e = dot_scratch(&part);
  if (e != hipSuccess) return fail(QPAT_E_HIP, std::string("dot_noalloc: symbol lookup: ") + hipGetErrorString(e));
  e = launch_dot(a, b, n, part, dot_blocks(n), out, (hipStream_t)stream);
  if (e != hipSuccess) return fail(QPAT_E_HIP, std::string("dot_noalloc: ") + hipGetErrorString(e));
  return QPAT_OK;
}

}  // extern "C"
