// Host side of the TV priorconditioner and the PCG vector update (the
// extern "C" entry points qpat_tv_* and qpat_axpby declared in include/qpat.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <memory>
#include <string>
#include <vector>

#include "../../include/qpat.h"
#include "qpat_internal.hpp"
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

#define STCHK(expr)                   \
  do {                                \
    qpat_status s_ = (expr);          \
    if (s_ != QPAT_OK) return s_;     \
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

// ---- inexact-Newton driver (Algorithm 5 with the PCG of Algorithm 4)
struct qpat_ld_s {
  qpat_plan plan = nullptr;
  qpat_tv tv = nullptr;
  int batch = 0, nx = 0, ny = 0, nt = 0, ns = 0;
  size_t N = 0, D = 0;
  int rzs = 0;                       // row stride of the rz history (i_max + 2 of the last run)
  void* mem = nullptr;
  float *res = nullptr, *grad = nullptr, *r = nullptr, *z = nullptr, *d = nullptr, *sol = nullptr, *hd = nullptr;
  float *jd = nullptr, *hsol = nullptr;  // data [B][nt][ns]: H_a d of the current direction, H_a sol
  double *part = nullptr, *rz = nullptr, *dhd = nullptr, *eps = nullptr;
  int *live = nullptr, *done = nullptr, *flag = nullptr;
  int* h_int = nullptr;              // pinned: flags to and from the device
  double* h_eps = nullptr;           // pinned: misfits
  ~qpat_ld_s() {
    if (tv) qpat_tv_destroy(tv);
    if (mem) (void)hipFree(mem);
    if (h_int) (void)hipHostFree(h_int);
    if (h_eps) (void)hipHostFree(h_eps);
  }
};

namespace {

// the FP64 scalars and the rz history are sized for i_max iterations
qpat_status ld_reserve_rz(qpat_ld L, int i_max) {
  const int want = i_max + 2;
  if (want <= L->rzs) return QPAT_OK;
  if (L->rz) (void)hipFree(L->rz);
  L->rz = nullptr;
  TVCHK(hipMalloc(&L->rz, sizeof(double) * size_t(L->batch) * want));
  L->rzs = want;
  return QPAT_OK;
}

// res = H x - data, eps_f = 0.5 |res_f|^2 (device) and grad = H^* res (eq gr).
// When every x_f is zero, H x = 0 exactly and the forward solve is skipped
// (res = -data, the value the solve would give).
qpat_status ld_misfit(qpat_ld L, const float* data, const float* x, hipStream_t st) {
  const int B = L->batch;
  const int64_t nd = int64_t(L->D) * B;
  TVCHK(launch_ld_dots(x, x, L->N, B, L->part, L->eps, 1, 1.0, st));
  TVCHK(hipMemcpyAsync(L->h_eps, L->eps, sizeof(double) * B, hipMemcpyDeviceToHost, st));
  TVCHK(hipStreamSynchronize(st));
  bool zero = true;
  for (int b = 0; b < B; ++b) zero = zero && L->h_eps[b] == 0.0;
  if (zero) {
    TVCHK(hipMemcpyAsync(L->res, data, sizeof(float) * nd, hipMemcpyDeviceToDevice, st));
    TVCHK(launch_axpby(nd, 0.0f, data, -1.0f, L->res, st));
  } else {
    qpat_status s = qpat_forward(L->plan, x, L->res, B, st);
    if (s != QPAT_OK) return s;
    TVCHK(launch_axpby(nd, -1.0f, data, 1.0f, L->res, st));
  }
  TVCHK(launch_ld_dots(L->res, L->res, L->D, B, L->part, L->eps, 1, 0.5, st));
  return qpat_adjoint(L->plan, L->res, L->grad, B, st);
}

qpat_status ld_read_eps(qpat_ld L, hipStream_t st) {
  TVCHK(hipMemcpyAsync(L->h_eps, L->eps, sizeof(double) * L->batch, hipMemcpyDeviceToHost, st));
  TVCHK(hipStreamSynchronize(st));
  return QPAT_OK;
}

}  // namespace

qpat_status qpat_ld_create(qpat_plan plan, int32_t batch, qpat_ld* out) {
  if (!out) return set_error(QPAT_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!plan) return set_error(QPAT_E_INVALID, "plan is NULL");
  if (batch < 1 || batch > 64) return set_error(QPAT_E_INVALID, "batch must be in [1, 64]");
  int32_t nx = 0, ny = 0, nt = 0, ns = 0;
  qpat_status s = qpat_plan_info(plan, &nx, &ny, &nt, &ns, nullptr);
  if (s != QPAT_OK) return s;
  std::unique_ptr<qpat_ld_s> L(new qpat_ld_s());
  L->plan = plan;
  L->batch = batch;
  L->nx = nx;
  L->ny = ny;
  L->nt = nt;
  L->ns = ns;
  L->N = size_t(nx) * ny;
  L->D = size_t(nt) * ns;
  s = qpat_tv_create(nx, ny, batch, &L->tv);
  if (s != QPAT_OK) return s;
  const size_t fields = L->N * batch, datas = L->D * batch;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  };
  const size_t o_res = take(datas * 4), o_grad = take(fields * 4), o_r = take(fields * 4), o_z = take(fields * 4),
               o_d = take(fields * 4), o_sol = take(fields * 4), o_hd = take(fields * 4),
               o_jd = take(datas * 4), o_hsol = take(datas * 4),
               o_part = take(sizeof(double) * kRedBlocks * batch), o_dhd = take(sizeof(double) * batch),
               o_eps = take(sizeof(double) * batch), o_live = take(sizeof(int) * batch),
               o_done = take(sizeof(int) * batch), o_flag = take(sizeof(int) * batch);
  TVCHK(hipMalloc(&L->mem, off));
  char* m = static_cast<char*>(L->mem);
  L->res = reinterpret_cast<float*>(m + o_res);
  L->grad = reinterpret_cast<float*>(m + o_grad);
  L->r = reinterpret_cast<float*>(m + o_r);
  L->z = reinterpret_cast<float*>(m + o_z);
  L->d = reinterpret_cast<float*>(m + o_d);
  L->sol = reinterpret_cast<float*>(m + o_sol);
  L->hd = reinterpret_cast<float*>(m + o_hd);
  L->jd = reinterpret_cast<float*>(m + o_jd);
  L->hsol = reinterpret_cast<float*>(m + o_hsol);
  L->part = reinterpret_cast<double*>(m + o_part);
  L->dhd = reinterpret_cast<double*>(m + o_dhd);
  L->eps = reinterpret_cast<double*>(m + o_eps);
  L->live = reinterpret_cast<int*>(m + o_live);
  L->done = reinterpret_cast<int*>(m + o_done);
  L->flag = reinterpret_cast<int*>(m + o_flag);
  TVCHK(hipHostMalloc(&L->h_int, sizeof(int) * batch, hipHostMallocDefault));
  TVCHK(hipHostMalloc(&L->h_eps, sizeof(double) * batch, hipHostMallocDefault));
  *out = L.release();
  return QPAT_OK;
}

void qpat_ld_destroy(qpat_ld L) {
  if (!L) return;
  (void)hipDeviceSynchronize();
  if (L->rz) (void)hipFree(L->rz);
  delete L;
}

qpat_status qpat_ld_run(qpat_ld L, const float* data, float* x, const qpat_ld_params* p, double* eps_hist,
                        int32_t* pcg_iters, int32_t* outer_steps, int32_t* solve_iters, qpat_stream stream) {
  const TraceRange trace_("qpat_ld_run");
  if (!L || !p) return set_error(QPAT_E_INVALID, "NULL argument");
  if (!data || !x) return set_error(QPAT_E_INVALID, "data and x must not be NULL");
  if (!eps_hist || !pcg_iters) return set_error(QPAT_E_INVALID, "eps_hist and pcg_iters must not be NULL");
  if (!(std::isfinite(p->beta) && p->beta > 0.0) || !(std::isfinite(p->gamma) && p->gamma > 0.0))
    return set_error(QPAT_E_INVALID, "beta and gamma must be finite and > 0");
  if (p->i_max < 0 || p->i_max > 100000 || p->i_m < 1 || p->outer_max < 0 || p->outer_max > 100000)
    return set_error(QPAT_E_INVALID, "need 0 <= i_max <= 1e5, i_m >= 1, 0 <= outer_max <= 1e5");
  if (!(std::isfinite(p->solve_tol) && p->solve_tol > 0.0 && p->solve_tol < 1.0) || p->solve_max_iter < 1)
    return set_error(QPAT_E_INVALID, "solve_tol must be in (0, 1) and solve_max_iter >= 1");
  if (std::isnan(p->tol_in) || std::isnan(p->tol_out)) return set_error(QPAT_E_INVALID, "tolerances must not be NaN");
  hipStream_t st = (hipStream_t)stream;
  const int B = L->batch, K = p->outer_max;
  const size_t N = L->N;
  STCHK(ld_reserve_rz(L, p->i_max));
  const int rzs = L->rzs;
  int solves = 0;
  for (int b = 0; b < B; ++b) {
    for (int k = 0; k <= K; ++k) eps_hist[size_t(b) * (K + 1) + k] = 0.0;
    for (int k = 0; k < K; ++k) pcg_iters[size_t(b) * K + k] = -1;
  }
  // eps^0 and the gradient at X^0
  STCHK(ld_misfit(L, data, x, st));
  STCHK(ld_read_eps(L, st));
  for (int b = 0; b < B; ++b) eps_hist[size_t(b) * (K + 1)] = L->h_eps[b];
  std::vector<int> active(B, 1);
  int k = 0;
  while (k < K) {
    if (k > 0) {
      for (int b = 0; b < B; ++b) {
        const double* h = eps_hist + size_t(b) * (K + 1);
        active[b] = active[b] && (1.0 - h[k] / h[k - 1] > p->tol_out);
      }
    }
    if (std::none_of(active.begin(), active.end(), [](int a) { return a != 0; })) break;
    // ---- Algorithm 4 on H d = -grad with the preconditioner M_gamma[X^k]
    STCHK(qpat_tv_set_weights(L->tv, x, p->beta, B, stream));
    TVCHK(hipMemcpyAsync(L->r, L->grad, sizeof(float) * N * B, hipMemcpyDeviceToDevice, st));
    TVCHK(launch_axpby(int64_t(N) * B, 0.0f, L->grad, -1.0f, L->r, st));  // r_0 = -grad
    int it = 0;
    STCHK(qpat_tv_solve(L->tv, p->gamma, L->r, L->z, B, p->solve_tol, p->solve_max_iter, &it, stream));
    solves += it;
    TVCHK(hipMemcpyAsync(L->d, L->z, sizeof(float) * N * B, hipMemcpyDeviceToDevice, st));
    TVCHK(hipMemsetAsync(L->sol, 0, sizeof(float) * N * B, st));
    TVCHK(hipMemsetAsync(L->hsol, 0, sizeof(float) * L->D * B, st));
    TVCHK(launch_ld_dots(L->r, L->z, N, B, L->part, L->rz, rzs, 1.0, st));   // rz_0
    for (int b = 0; b < B; ++b) L->h_int[b] = active[b] ? 0 : 1;          // done = not active
    TVCHK(hipMemcpyAsync(L->done, L->h_int, sizeof(int) * B, hipMemcpyHostToDevice, st));
    std::vector<int> count(B, 0);
    for (int i = 0;; ++i) {
      TVCHK(launch_ld_live(B, L->rz, rzs, i, p->i_max, p->i_m, p->tol_in, L->done, L->live, st));
      TVCHK(hipMemcpyAsync(L->h_int, L->live, sizeof(int) * B, hipMemcpyDeviceToHost, st));
      TVCHK(hipStreamSynchronize(st));   // one host read per iteration: which fields go on
      bool any = false;
      for (int b = 0; b < B; ++b) {
        any = any || L->h_int[b] != 0;
        count[b] += L->h_int[b] != 0;
      }
      if (!any) break;
      STCHK(qpat_jtjv_data(L->plan, L->d, L->jd, L->hd, B, stream));     // H_a d and H d, one batched call
      TVCHK(launch_ld_dots(L->d, L->hd, N, B, L->part, L->dhd, 1, 1.0, st));
      TVCHK(launch_ld_step(N, B, L->rz, rzs, i, L->dhd, L->live, L->d, L->hd, L->sol, L->r, st));
      TVCHK(launch_ld_data_step(L->D, B, L->rz, rzs, i, L->dhd, L->live, L->jd, L->hsol, st));
      STCHK(qpat_tv_solve(L->tv, p->gamma, L->r, L->z, B, p->solve_tol, p->solve_max_iter, &it, stream));
      solves += it;
      TVCHK(launch_ld_dots(L->r, L->z, N, B, L->part, L->rz + i + 1, rzs, 1.0, st));
      TVCHK(launch_ld_dir(N, B, L->rz, rzs, i, L->live, L->z, L->d, st));
    }
    // X^{k+1} = X^k + d^k for the fields still iterating (step length 1)
    for (int b = 0; b < B; ++b) L->h_int[b] = active[b];
    TVCHK(hipMemcpyAsync(L->flag, L->h_int, sizeof(int) * B, hipMemcpyHostToDevice, st));
    TVCHK(launch_ld_add(N, B, L->flag, L->sol, x, st));
    for (int b = 0; b < B; ++b)
      if (active[b]) pcg_iters[size_t(b) * K + k] = count[b];
    // eps^{k+1}: the residual H_a X^{k+1} - data = res + H_a sol (H_a linear), with
    // H_a sol accumulated from the PCG's products; the gradient only if another
    // outer step can follow
    TVCHK(launch_ld_add(L->D, B, L->flag, L->hsol, L->res, st));
    TVCHK(launch_ld_dots(L->res, L->res, L->D, B, L->part, L->eps, 1, 0.5, st));
    STCHK(ld_read_eps(L, st));
    for (int b = 0; b < B; ++b) {
      double* h = eps_hist + size_t(b) * (K + 1);
      h[k + 1] = active[b] ? L->h_eps[b] : h[k];
    }
    ++k;
    bool more = false;
    if (k < K)
      for (int b = 0; b < B; ++b) {
        const double* h = eps_hist + size_t(b) * (K + 1);
        more = more || (active[b] && 1.0 - h[k] / h[k - 1] > p->tol_out);
      }
    if (more) STCHK(qpat_adjoint(L->plan, L->res, L->grad, B, stream));
  }
  // entries past the last step repeat the last misfit
  for (int b = 0; b < B; ++b) {
    double* h = eps_hist + size_t(b) * (K + 1);
    for (int j = k + 1; j <= K; ++j) h[j] = h[k];
  }
  if (outer_steps) *outer_steps = k;
  if (solve_iters) *solve_iters = solves;
  TVCHK(hipStreamSynchronize(st));
  return QPAT_OK;
}

}  // extern "C"
