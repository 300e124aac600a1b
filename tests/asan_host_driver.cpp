// Host-side checks of libqpat under AddressSanitizer (host code only; the
// device code is built as usual).  Without a GPU every call below stops at its
// argument checks or at its first device allocation; before that, plan
// creation runs the whole FP64 construction of the medium tables, k-space
// multipliers, FFT twiddles and sensor taps on the host, which is what the
// sanitizer watches.  Prints "host checks ok" and exits 0 when every call
// returned the expected kind of status.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../include/qpat.h"

static int failures = 0;
static void expect(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAILED: %s (last error: %s)\n", what, qpat_last_error());
    ++failures;
  }
}

static qpat_params params2d(int nx, int ny, std::vector<double>& xy, int ns) {
  xy.resize(2 * ns);
  for (int s = 0; s < ns; ++s) {
    const double a = 2.0 * M_PI * s / ns;
    xy[2 * s] = 0.3 * nx * 1e-4 * std::cos(a) + 0.37e-4;  // off the nodes
    xy[2 * s + 1] = 0.3 * ny * 1e-4 * std::sin(a) - 0.21e-4;
  }
  qpat_params p{};
  p.nx = nx;
  p.ny = ny;
  p.dx = p.dy = 1e-4;
  p.dt = 0.3 * 1e-4 / 1600.0;
  p.nt = 40;
  p.c_ref = 1600.0;
  p.pml_size = std::min(6, std::min(nx, ny) / 2 - 1);
  p.pml_alpha = 2.0;
  p.alpha0_db = 0.75;
  p.y = 1.5;
  p.ns = ns;
  p.sensor_xy = xy.data();
  return p;
}

int main() {
  for (int s = 0; s <= 6; ++s) expect(qpat_status_string(qpat_status(s)) != nullptr, "status string");
  std::vector<double> xy;
  // 2-D: valid parameter sets, then plan creation up to the first device allocation
  const int sizes[][2] = {{64, 48}, {96, 64}, {128, 128}, {1024, 256}, {8, 8}};
  for (const auto& n : sizes) {
    qpat_params p = params2d(n[0], n[1], xy, 17);
    expect(qpat_validate(&p) == QPAT_OK, "validate 2-D");
    std::vector<double> c0(size_t(n[0]) * n[1]), rho0(c0.size());
    for (size_t i = 0; i < c0.size(); ++i) {
      c0[i] = 1500.0 + 80.0 * std::sin(0.01 * double(i));
      rho0[i] = 1000.0 + 60.0 * std::cos(0.013 * double(i));
    }
    qpat_plan plan = nullptr;
    const qpat_status st = qpat_plan_create(&p, c0.data(), rho0.data(), &plan);
    if (st == QPAT_OK) {
      qpat_plan_destroy(plan);  // a machine with a GPU
    } else {
      expect(plan == nullptr, "failed plan is NULL");
      expect(st == QPAT_E_HIP || st == QPAT_E_OOM, "plan fails only at the device");
    }
    p.alpha0_db = 0.0;  // lossless
    expect(qpat_validate(&p) == QPAT_OK, "validate lossless");
  }
  // 2-D: invalid parameter sets
  {
    qpat_params p = params2d(64, 48, xy, 5);
    qpat_params q = p;
    q.nx = 100;
    expect(qpat_validate(&q) != QPAT_OK, "nx 100");
    q = p;
    q.y = 1.0;
    expect(qpat_validate(&q) != QPAT_OK, "y = 1");
    q = p;
    q.sensor_xy = nullptr;
    expect(qpat_validate(&q) != QPAT_OK, "NULL sensors");
    q = p;
    std::vector<double> far = {1.0, 1.0};
    q.ns = 1;
    q.sensor_xy = far.data();
    expect(qpat_validate(&q) != QPAT_OK, "sensor outside");
    q = p;
    q.dt = 1e-3;
    q.c_ref = 100.0;
    std::vector<double> c0(64 * 48, 1500.0), rho0(64 * 48, 1000.0);
    qpat_plan plan = nullptr;
    expect(qpat_plan_create(&q, c0.data(), rho0.data(), &plan) != QPAT_OK && plan == nullptr, "unstable dt");
    c0[7] = -1.0;
    expect(qpat_plan_create(&p, c0.data(), rho0.data(), &plan) == QPAT_E_INVALID, "negative c0");
    expect(qpat_plan_create(&p, nullptr, rho0.data(), &plan) == QPAT_E_INVALID, "NULL c0");
  }
  // 3-D: the paper's 49-point axes (7 x 7) and a prime axis
  {
    const int n3[][3] = {{49, 49, 49}, {53, 13, 11}, {16, 12, 10}};
    for (const auto& n : n3) {
      std::vector<double> sxyz = {0.11e-4, -0.23e-4, 0.31e-4, 1.3e-4, 0.7e-4, -0.9e-4};
      qpat_params3d p{};
      p.nx = n[0];
      p.ny = n[1];
      p.nz = n[2];
      p.dx = p.dy = p.dz = 1e-4;
      p.dt = 0.3 * 1e-4 / 1600.0;
      p.nt = 20;
      p.c_ref = 1600.0;
      p.pml_size = 3;
      p.pml_alpha = 2.0;
      p.alpha0_db = 0.75;
      p.y = 1.5;
      p.ns = 2;
      p.sensor_xyz = sxyz.data();
      expect(qpat3d_validate(&p) == QPAT_OK, "validate 3-D");
      const size_t N = size_t(n[0]) * n[1] * n[2];
      std::vector<double> c0(N, 1500.0), rho0(N, 1000.0);
      qpat_plan3d plan = nullptr;
      const qpat_status st = qpat3d_plan_create(&p, c0.data(), rho0.data(), &plan);
      if (st == QPAT_OK) qpat3d_plan_destroy(plan);
      else expect(plan == nullptr && (st == QPAT_E_HIP || st == QPAT_E_OOM), "3-D plan fails only at the device");
    }
  }
  // the other handles: argument checks, then the device
  {
    qpat_optical o = nullptr;
    expect(qpat_optical_create(0, 4, 1e-4, 1, &o) == QPAT_E_INVALID, "optical size");
    const qpat_status st = qpat_optical_create(16, 12, 1e-4, 2, &o);
    if (st == QPAT_OK) qpat_optical_destroy(o);
    qpat_tv tv = nullptr;
    expect(qpat_tv_create(1, 4, 1, &tv) == QPAT_E_INVALID, "tv size");
    qpat_ld ld = nullptr;
    expect(qpat_ld_create(nullptr, 1, &ld) == QPAT_E_INVALID && ld == nullptr, "ld NULL plan");
    qpat_batch b = nullptr;
    expect(qpat_batch_create(nullptr, 0, &b) == QPAT_E_INVALID, "batch NULL");
    float us = 0.f;
    int32_t to = 0;
    expect(qpat_probe_barrier(5, 256, 256, 10, 0, nullptr, &us, &to) == QPAT_E_INVALID, "probe design");
    expect(qpat_dot_noalloc(nullptr, nullptr, -1, nullptr, nullptr) == QPAT_E_INVALID, "dot_noalloc n");
  }
  if (failures) return 1;
  std::printf("host checks ok\n");
  return 0;
}
