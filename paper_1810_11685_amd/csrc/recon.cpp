// Host side of the TV priorconditioner and the PCG vector update (the
// extern "C" entry points qpat_tv_* and qpat_axpby declared in include/qpat.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/qpat.h"
#include "recon_internal.hpp"

namespace qpat {
qpat_status set_error(qpat_status s, const std::string& msg);
}

using namespace qpat;

namespace {

#define TVCHK(expr)                                                                             \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return set_error(e_ == hipErrorOutOfMemory ? QPAT_E_OOM : QPAT_E_HIP,                      \
                       std::string(#expr) + ": " + hipGetErrorString(e_));                      \
  } while (0)

constexpr int kCheckEvery = 8;  // CG iterations between host convergence checks

}  // namespace

struct qpat_tv_s {
  int nx = 0, ny = 0, cap = 0;
  void* mem = nullptr;
  TvCg c{};
  std::vector<MgLevel> lv;   // multigrid levels, finest first
  bool weights = false;
  std::vector<double> h_rr, h_bb, h_part;
  ~qpat_tv_s() {
    if (mem) (void)hipFree(mem);
  }
};

extern "C" {

qpat_status qpat_tv_create(int32_t nx, int32_t ny, int32_t batch, qpat_tv* out) {
  if (!out) return set_error(QPAT_E_INVALID, "out is NULL");
  *out = nullptr;
  if (nx < 2 || ny < 2 || int64_t(nx) * ny > (int64_t(1) << 24))
    return set_error(QPAT_E_INVALID, "grid must be at least 2 x 2 and at most 2^24 nodes");
  if (batch < 1 || batch > 64) return set_error(QPAT_E_INVALID, "batch must be in [1, 64]");
  qpat_tv t = new qpat_tv_s();
  t->nx = nx;
  t->ny = ny;
  t->cap = batch;
  const size_t n = size_t(nx) * ny * batch;
  const size_t parts = size_t(batch) * kRedBlocks;
  // multigrid levels: 2 x 2 aggregates down to a single node
  std::vector<std::pair<int, int>> dims{{nx, ny}};
  while (int64_t(dims.back().first) * dims.back().second > 1)
    dims.push_back({(dims.back().first + 1) / 2, (dims.back().second + 1) / 2});
  if (int(dims.size()) > kMgMaxLevels) {
    delete t;
    return set_error(QPAT_E_UNSUPPORTED, "grid needs too many multigrid levels");
  }
  size_t coarse = 0;
  for (size_t l = 1; l < dims.size(); ++l) coarse += size_t(dims[l].first) * dims[l].second * batch;
  const size_t words = 8 * n + 3 * parts + 2 * size_t(batch) + 3 * size_t(batch) + 2 * n + 7 * coarse;
  hipError_t e = hipMalloc(&t->mem, words * sizeof(double));
  if (e != hipSuccess) {
    delete t;
    return set_error(e == hipErrorOutOfMemory ? QPAT_E_OOM : QPAT_E_HIP,
                     std::string("qpat_tv_create: ") + hipGetErrorString(e));
  }
  double* d = static_cast<double*>(t->mem);
  auto take = [&](size_t cnt) {
    double* p = d;
    d += cnt;
    return p;
  };
  t->c.x = take(n);
  t->c.r = take(n);
  t->c.z = take(n);
  t->c.p = take(n);
  t->c.q = take(n);
  t->c.dinv = take(n);
  t->c.wh = take(n);
  t->c.wv = take(n);
  t->c.part_rz = take(parts);
  t->c.part_rr = take(parts);
  t->c.part_pq = take(parts);
  t->c.rz = take(2 * size_t(batch));
  t->c.rr = take(batch);
  t->c.rr_next = take(batch);
  t->c.bb = take(batch);
  // level 0 works on the CG vectors: b = r, result t = z
  t->lv.push_back(MgLevel{nx, ny, t->c.wh, t->c.wv, take(n), t->c.dinv, t->c.r, take(n), t->c.z});
  for (size_t l = 1; l < dims.size(); ++l) {
    const size_t m = size_t(dims[l].first) * dims[l].second * batch;
    MgLevel L{dims[l].first, dims[l].second, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    L.wh = take(m);
    L.wv = take(m);
    L.g = take(m);
    L.dinv = take(m);
    L.b = take(m);
    L.x = take(m);
    L.t = take(m);
    t->lv.push_back(L);
  }
  t->h_rr.resize(batch);
  t->h_bb.resize(batch);
  t->h_part.resize(parts);
  *out = t;
  return QPAT_OK;
}

void qpat_tv_destroy(qpat_tv tv) {
  if (!tv) return;
  (void)hipDeviceSynchronize();
  delete tv;
}

static qpat_status tv_check(qpat_tv tv, int32_t batch) {
  if (!tv) return set_error(QPAT_E_INVALID, "tv is NULL");
  if (batch < 1 || batch > tv->cap) return set_error(QPAT_E_INVALID, "batch must be in [1, capacity]");
  return QPAT_OK;
}

qpat_status qpat_tv_set_weights(qpat_tv tv, const float* x, double beta, int32_t batch, qpat_stream stream) {
  qpat_status s = tv_check(tv, batch);
  if (s != QPAT_OK) return s;
  if (!x) return set_error(QPAT_E_INVALID, "x is NULL");
  if (!(std::isfinite(beta) && beta > 0.0)) return set_error(QPAT_E_INVALID, "beta must be finite and > 0");
  TVCHK(launch_tv_weights(x, tv->nx, tv->ny, batch, beta, tv->c.wh, tv->c.wv, (hipStream_t)stream));
  tv->weights = true;
  return QPAT_OK;
}

qpat_status qpat_tv_apply(qpat_tv tv, double gamma, const float* x, float* y, int32_t batch, qpat_stream stream) {
  qpat_status s = tv_check(tv, batch);
  if (s != QPAT_OK) return s;
  if (!x || !y) return set_error(QPAT_E_INVALID, "NULL field");
  if (!tv->weights) return set_error(QPAT_E_INVALID, "qpat_tv_set_weights has not been called");
  if (!(std::isfinite(gamma) && gamma >= 0.0)) return set_error(QPAT_E_INVALID, "gamma must be finite and >= 0");
  TVCHK(launch_tv_apply(x, y, tv->c.wh, tv->c.wv, tv->nx, tv->ny, batch, gamma, (hipStream_t)stream));
  return QPAT_OK;
}

qpat_status qpat_tv_solve(qpat_tv tv, double gamma, const float* r, float* z, int32_t batch, double tol,
                          int32_t max_iter, int32_t* iters, qpat_stream stream) {
  qpat_status s = tv_check(tv, batch);
  if (s != QPAT_OK) return s;
  if (!r || !z) return set_error(QPAT_E_INVALID, "NULL field");
  if (!tv->weights) return set_error(QPAT_E_INVALID, "qpat_tv_set_weights has not been called");
  if (!(std::isfinite(gamma) && gamma > 0.0)) return set_error(QPAT_E_INVALID, "gamma must be finite and > 0");
  if (!(std::isfinite(tol) && tol > 0.0 && tol < 1.0)) return set_error(QPAT_E_INVALID, "tol must be in (0, 1)");
  if (max_iter < 1) return set_error(QPAT_E_INVALID, "max_iter must be >= 1");
  hipStream_t st = (hipStream_t)stream;
  const double tol2 = tol * tol;
  const int nlev = int(tv->lv.size());
  TVCHK(launch_mg_setup(tv->lv.data(), nlev, batch, gamma, st));
  TVCHK(launch_cg_start(r, tv->c, tv->lv.data(), nlev, tv->nx, tv->ny, batch, st));
  int it = 0;
  while (it < max_iter) {
    const int chunk = std::min(kCheckEvery, max_iter - it);
    for (int k = 0; k < chunk; ++k, ++it)
      TVCHK(launch_cg_iteration(tv->c, tv->lv.data(), nlev, tv->nx, tv->ny, batch, gamma, it & 1, tol2, st));
    // the pending r.r of the last iteration is published by the next cg_q or by the finish
    TVCHK(hipMemcpyAsync(tv->h_rr.data(), tv->c.rr_next, sizeof(double) * batch, hipMemcpyDeviceToHost, st));
    TVCHK(hipMemcpyAsync(tv->h_bb.data(), tv->c.bb, sizeof(double) * batch, hipMemcpyDeviceToHost, st));
    TVCHK(hipStreamSynchronize(st));
    bool done = true;
    for (int b = 0; b < batch; ++b) done = done && !(tv->h_rr[b] > tol2 * tv->h_bb[b]);
    if (done) break;
  }
  TVCHK(launch_cg_finish(tv->c, z, tv->nx, tv->ny, batch, st));
  if (iters) *iters = it;
  return QPAT_OK;
}

qpat_status qpat_tv_value(qpat_tv tv, const float* x, double beta, int32_t batch, double* out, qpat_stream stream) {
  qpat_status s = tv_check(tv, batch);
  if (s != QPAT_OK) return s;
  if (!x || !out) return set_error(QPAT_E_INVALID, "NULL argument");
  if (!(std::isfinite(beta) && beta > 0.0)) return set_error(QPAT_E_INVALID, "beta must be finite and > 0");
  hipStream_t st = (hipStream_t)stream;
  TVCHK(launch_tv_value(x, tv->nx, tv->ny, batch, beta, tv->c.part_pq, st));
  TVCHK(hipMemcpyAsync(tv->h_part.data(), tv->c.part_pq, sizeof(double) * batch * kRedBlocks,
                       hipMemcpyDeviceToHost, st));
  TVCHK(hipStreamSynchronize(st));
  for (int b = 0; b < batch; ++b) {
    double acc = 0.0;
    for (int i = 0; i < kRedBlocks; ++i) acc += tv->h_part[size_t(b) * kRedBlocks + i];
    out[b] = acc;
  }
  return QPAT_OK;
}

qpat_status qpat_axpby(int64_t n, float a, const float* x, float b, float* y, qpat_stream stream) {
  if (n < 0) return set_error(QPAT_E_INVALID, "n must be >= 0");
  if (n == 0) return QPAT_OK;
  if (!x || !y) return set_error(QPAT_E_INVALID, "NULL vector with n > 0");
  TVCHK(launch_axpby(n, a, x, b, y, (hipStream_t)stream));
  return QPAT_OK;
}

}  // extern "C"
