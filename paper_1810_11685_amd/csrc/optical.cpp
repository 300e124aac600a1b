// Host side of the optical operators (the qpat_optical_* entry points of
// include/qpat.h): device state of a batch of problems on one grid-matched
// mesh, the conjugate-gradient driver with a convergence check every 32
// iterations, and the forward / J_o / J_o^* / pixel-map calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/qpat.h"
#include "optical_internal.hpp"

namespace qpat {
qpat_status set_error(qpat_status s, const std::string& msg);
}

using namespace qpat;

namespace {

#define OPCHK(expr)                                                                             \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return set_error(e_ == hipErrorOutOfMemory ? QPAT_E_OOM : QPAT_E_HIP,                      \
                       std::string(#expr) + ": " + hipGetErrorString(e_));                      \
  } while (0)

constexpr int kCheckEvery = 8;   // CG iterations between host convergence checks
static_assert(kCheckEvery % 2 == 0, "full chunks must start at an even iteration");

}  // namespace

struct qpat_optical_s {
  int cap = 0;
  void* mem = nullptr;
  OptCg c{};
  std::vector<OptLevel> lv;   // multigrid levels, finest first
  bool solved = false;
  std::vector<double> h_rr, h_bb;
  // hipGraph of one chunk of kCheckEvery CG iterations (chunks start at an
  // even iteration, so every full chunk launches the same kernels) for the
  // batch and tolerance it was captured with; the buffers never move
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  int g_batch = 0;
  double g_tol2 = 0.0;
  void drop_graph() {
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    graph_exec = nullptr;
    graph = nullptr;
  }
  ~qpat_optical_s() {
    drop_graph();
    if (mem) (void)hipFree(mem);
  }
};

namespace {

qpat_status check(qpat_optical o, int batch) {
  if (!o) return set_error(QPAT_E_INVALID, "optical handle is NULL");
  if (batch < 1 || batch > o->cap) return set_error(QPAT_E_INVALID, "batch must be in [1, capacity]");
  return QPAT_OK;
}

bool opt_ok(double tol, int max_iter) { return std::isfinite(tol) && tol > 0.0 && tol < 1.0 && max_iter >= 1; }

// One full chunk of CG iterations: replayed from a captured graph on a
// non-default stream (a chunk of small launches is bound by their issue
// rate), launched one by one on the default stream, which cannot be captured.
hipError_t cg_chunk(qpat_optical o, const OptCg& c, double tol2, hipStream_t st) {
  if (st == nullptr) {
    for (int k = 0; k < kCheckEvery; ++k) {
      const hipError_t e = opt_launch_cg_iteration(c, o->lv.data(), int(o->lv.size()), k & 1, tol2, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  if (!o->graph_exec || o->g_batch != c.batch || o->g_tol2 != tol2) {
    o->drop_graph();
    hipError_t e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t el = hipSuccess;
    for (int k = 0; k < kCheckEvery && el == hipSuccess; ++k)
      el = opt_launch_cg_iteration(c, o->lv.data(), int(o->lv.size()), k & 1, tol2, st);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(st, &g);
    if (el != hipSuccess || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return el != hipSuccess ? el : e;
    }
    o->graph = g;
    e = hipGraphInstantiate(&o->graph_exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      o->drop_graph();
      return e;
    }
    o->g_batch = c.batch;
    o->g_tol2 = tol2;
  }
  return hipGraphLaunch(o->graph_exec, st);
}

// Solve A x = rhs (already in c.rhs) for `batch` problems.
qpat_status solve(qpat_optical o, int batch, double tol, int max_iter, int* iters, hipStream_t st) {
  OptCg c = o->c;
  c.batch = batch;
  const double tol2 = tol * tol;
  OPCHK(opt_launch_mg_setup(c, o->lv.data(), int(o->lv.size()), st));
  OPCHK(opt_launch_cg_start(c, o->lv.data(), int(o->lv.size()), st));
  int it = 0;
  while (it < max_iter) {
    const int chunk = std::min(kCheckEvery, max_iter - it);
    if (chunk == kCheckEvery) {
      OPCHK(cg_chunk(o, c, tol2, st));
      it += chunk;
    } else {
      for (int k = 0; k < chunk; ++k, ++it)
        OPCHK(opt_launch_cg_iteration(c, o->lv.data(), int(o->lv.size()), it & 1, tol2, st));
    }
    OPCHK(hipMemcpyAsync(o->h_rr.data(), c.rr_next, sizeof(double) * batch, hipMemcpyDeviceToHost, st));
    OPCHK(hipMemcpyAsync(o->h_bb.data(), c.bb, sizeof(double) * batch, hipMemcpyDeviceToHost, st));
    OPCHK(hipStreamSynchronize(st));
    bool done = true;
    for (int b = 0; b < batch; ++b) done = done && !(o->h_rr[b] > tol2 * o->h_bb[b]);
    if (done) break;
  }
  OPCHK(opt_launch_cg_finish(c, st));
  if (iters) *iters = it;
  return QPAT_OK;
}

OptCg with_batch(qpat_optical o, int batch) {
  OptCg c = o->c;
  c.batch = batch;
  return c;
}

}  // namespace

extern "C" {

qpat_status qpat_optical_create(int32_t nx, int32_t ny, double dx, int32_t batch, qpat_optical* out) {
  if (!out) return set_error(QPAT_E_INVALID, "out is NULL");
  *out = nullptr;
  if (nx < 1 || ny < 1 || int64_t(nx + 1) * (ny + 1) > (int64_t(1) << 26))
    return set_error(QPAT_E_INVALID, "mesh must have 1..2^26 nodes");
  if (!(std::isfinite(dx) && dx > 0.0)) return set_error(QPAT_E_INVALID, "dx must be finite and > 0");
  if (batch < 1 || batch > 64) return set_error(QPAT_E_INVALID, "batch must be in [1, 64]");
  qpat_optical o = new qpat_optical_s();
  OptCg& c = o->c;
  c.nx = nx;
  c.ny = ny;
  c.nn = (nx + 1) * (ny + 1);
  c.ne = 2 * nx * ny;
  c.batch = batch;
  c.h = dx;
  c.nblk = std::min(kOptBlocks, (c.nn + kOptThreads - 1) / kOptThreads);
  const size_t nn = size_t(c.nn) * batch, ne = size_t(c.ne) * batch, np = size_t(kOptBlocks) * batch;
  // multigrid levels on the node grid: 2 x 2 aggregates down to a single node
  std::vector<std::pair<int, int>> dims{{nx + 1, ny + 1}};
  while (int64_t(dims.back().first) * dims.back().second > 1)
    dims.push_back({(dims.back().first + 1) / 2, (dims.back().second + 1) / 2});
  if (int(dims.size()) > kOptMgMaxLevels) {
    delete o;
    return set_error(QPAT_E_UNSUPPORTED, "mesh needs too many multigrid levels");
  }
  size_t coarse = 0;
  for (size_t l = 1; l < dims.size(); ++l) coarse += size_t(dims[l].first) * dims[l].second * batch;
  const size_t total = 4 * ne + 7 * nn + 3 * np + 5 * size_t(batch) + 4 * size_t(batch) + 6 * nn + 8 * coarse;
  void* mem = nullptr;
  hipError_t e = hipMalloc(&mem, total * sizeof(double));
  if (e != hipSuccess) {
    delete o;
    return set_error(QPAT_E_OOM, "optical work space");
  }
  o->mem = mem;
  double* p = static_cast<double*>(mem);
  auto take = [&](size_t n) {
    double* r = p;
    p += n;
    return r;
  };
  c.ka = take(ne);
  c.mu = take(ne);
  c.ek = take(ne);
  c.em = take(ne);
  c.phi = take(nn);
  c.rhs = take(nn);
  c.x = take(nn);
  c.r = take(nn);
  c.p = take(nn);
  c.q = take(nn);
  c.dinv = take(nn);
  c.part_rz = take(np);
  c.part_rr = take(np);
  c.part_pq = take(np);
  c.rz = take(2 * size_t(batch));
  c.rr = take(batch);
  c.rr_next = take(batch);
  c.bb = take(batch);
  c.cur = take(4 * size_t(batch));
  c.z = take(nn);
  {
    // level 0 works on the CG vectors: b = r, result t = z
    OptLevel L{nx + 1, ny + 1, take(nn), take(nn), take(nn), take(nn), c.dinv, c.r, take(nn), c.z};
    o->lv.push_back(L);
  }
  for (size_t l = 1; l < dims.size(); ++l) {
    const size_t m = size_t(dims[l].first) * dims[l].second * batch;
    OptLevel L{dims[l].first, dims[l].second, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    L.sc = take(m);
    L.se = take(m);
    L.sn = take(m);
    L.sd = take(m);
    L.dinv = take(m);
    L.b = take(m);
    L.x = take(m);
    L.t = take(m);
    o->lv.push_back(L);
  }
  o->cap = batch;
  o->h_rr.resize(batch);
  o->h_bb.resize(batch);
  *out = o;
  return QPAT_OK;
}

void qpat_optical_destroy(qpat_optical o) {
  if (!o) return;
  (void)hipDeviceSynchronize();
  delete o;
}

qpat_status qpat_optical_forward(qpat_optical o, const float* kappa, const float* mu, const double* currents,
                                 float* H, int32_t batch, double tol, int32_t max_iter, int32_t* iters,
                                 qpat_stream stream) {
  qpat_status s = check(o, batch);
  if (s != QPAT_OK) return s;
  if (!kappa || !mu || !currents || !H) return set_error(QPAT_E_INVALID, "NULL argument");
  if (!opt_ok(tol, max_iter)) return set_error(QPAT_E_INVALID, "tol must be in (0, 1) and max_iter >= 1");
  hipStream_t st = (hipStream_t)stream;
  const OptCg c = with_batch(o, batch);
  OPCHK(hipMemcpyAsync(c.cur, currents, sizeof(double) * 4 * batch, hipMemcpyHostToDevice, st));
  OPCHK(opt_launch_set(c, kappa, mu, st));
  OPCHK(opt_launch_rhs(c, 0, c.cur, nullptr, st));
  s = solve(o, batch, tol, max_iter, iters, st);
  if (s != QPAT_OK) return s;
  OPCHK(opt_launch_out(c, 0, nullptr, H, nullptr, st));
  o->solved = true;
  return QPAT_OK;
}

qpat_status qpat_optical_jv(qpat_optical o, const float* dkappa, const float* dmu, float* dH, int32_t batch,
                            double tol, int32_t max_iter, int32_t* iters, qpat_stream stream) {
  qpat_status s = check(o, batch);
  if (s != QPAT_OK) return s;
  if (!dkappa || !dmu || !dH) return set_error(QPAT_E_INVALID, "NULL argument");
  if (!o->solved) return set_error(QPAT_E_INVALID, "qpat_optical_forward has not been called");
  if (!opt_ok(tol, max_iter)) return set_error(QPAT_E_INVALID, "tol must be in (0, 1) and max_iter >= 1");
  hipStream_t st = (hipStream_t)stream;
  const OptCg c = with_batch(o, batch);
  OPCHK(opt_launch_stage(c, dkappa, dmu, st));
  OPCHK(opt_launch_rhs(c, 1, nullptr, nullptr, st));
  s = solve(o, batch, tol, max_iter, iters, st);
  if (s != QPAT_OK) return s;
  OPCHK(opt_launch_out(c, 1, nullptr, dH, nullptr, st));
  return QPAT_OK;
}

qpat_status qpat_optical_jtv(qpat_optical o, const float* H, float* gkappa, float* gmu, int32_t batch, double tol,
                             int32_t max_iter, int32_t* iters, qpat_stream stream) {
  qpat_status s = check(o, batch);
  if (s != QPAT_OK) return s;
  if (!H || !gkappa || !gmu) return set_error(QPAT_E_INVALID, "NULL argument");
  if (!o->solved) return set_error(QPAT_E_INVALID, "qpat_optical_forward has not been called");
  if (!opt_ok(tol, max_iter)) return set_error(QPAT_E_INVALID, "tol must be in (0, 1) and max_iter >= 1");
  hipStream_t st = (hipStream_t)stream;
  const OptCg c = with_batch(o, batch);
  OPCHK(opt_launch_rhs(c, 2, nullptr, H, st));
  s = solve(o, batch, tol, max_iter, iters, st);
  if (s != QPAT_OK) return s;
  OPCHK(opt_launch_out(c, 2, H, gkappa, gmu, st));
  return QPAT_OK;
}

qpat_status qpat_optical_pixels(qpat_optical o, const float* in, float* out, int32_t transpose, int32_t batch,
                                qpat_stream stream) {
  if (!o) return set_error(QPAT_E_INVALID, "optical handle is NULL");
  if (!in || !out) return set_error(QPAT_E_INVALID, "NULL argument");
  if (batch < 1) return set_error(QPAT_E_INVALID, "batch must be >= 1");
  OPCHK(opt_launch_pixels(in, out, o->c.nx * o->c.ny, batch, transpose != 0, (hipStream_t)stream));
  return QPAT_OK;
}

}  // extern "C"
