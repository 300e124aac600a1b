// Lagged-diffusivity TV priorconditioner of the inexact-Newton driver
// (Section 5.2: eqs tvm, dd, jm, m, m1, pre) and the vector update of its PCG
// loop (Algorithm 4), for fields on the acoustic grid.
//
// D takes differences across the internal edges between horizontally and
// vertically adjacent grid nodes (unit edge length); C[x] = diag((|D x|^2 +
// beta)^(-1/2)); M_gamma = D^T C D + gamma I.  Edge weights are stored per
// node: wh[j][i] for the edge (j, i)-(j, i+1), wv[j][i] for (j, i)-(j+1, i)
// (zero past the last column / row).  M_gamma z = r is solved by conjugate
// gradients in FP64, preconditioned by one multigrid V-cycle: 2 x 2
// aggregation with piecewise-constant prolongation P, whose Galerkin coarse
// operators P^T A P keep the same five-point form (a coarse edge weighs the
// sum of the fine edges between its two aggregates, the diagonal term sums
// over the aggregate), and one damped Jacobi sweep before and after each
// coarse correction, which keeps the preconditioner symmetric.  The scalars of
// every field stay in device memory; the reductions are deterministic (fixed
// block partition, fixed order; every block re-reduces the block partials
// itself).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "recon_internal.hpp"

namespace qpat {

namespace {

__device__ __forceinline__ double wave_sum_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Block sum of one value per thread (blockDim.x = kRedThreads); result in thread 0.
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum_d(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kRedThreads / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

// Sum of the kRedBlocks partials of field b, in a fixed order (every block
// computes the same value).
__device__ __forceinline__ double partial_total(const double* __restrict__ part, int b, double* red) {
  double v = 0.0;
  for (int i = threadIdx.x; i < kRedBlocks; i += blockDim.x) v += part[size_t(b) * kRedBlocks + i];
  __shared__ double tot;
  const double s = block_sum(v, red);
  if (threadIdx.x == 0) tot = s;
  __syncthreads();
  return tot;
}

__global__ void __launch_bounds__(kRedThreads)
tv_weights_kernel(const float* __restrict__ x, int nx, int ny, double beta, double* __restrict__ wh,
                  double* __restrict__ wv) {
  const int b = blockIdx.y;
  const size_t n = size_t(nx) * ny, base = size_t(b) * n;
  for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += size_t(gridDim.x) * blockDim.x) {
    const int j = int(k / nx), i = int(k - size_t(j) * nx);
    const double xc = x[base + k];
    double h = 0.0, v = 0.0;
    if (i + 1 < nx) {
      const double g = xc - double(x[base + k + 1]);
      h = 1.0 / sqrt(g * g + beta);
    }
    if (j + 1 < ny) {
      const double g = xc - double(x[base + k + nx]);
      v = 1.0 / sqrt(g * g + beta);
    }
    wh[base + k] = h;
    wv[base + k] = v;
  }
}

// (M_gamma u)_k for node k = (j, i) of field b.
template <typename T>
__device__ __forceinline__ double mgamma_at(const T* __restrict__ u, const double* __restrict__ wh,
                                            const double* __restrict__ wv, size_t base, size_t k, int i, int j,
                                            int nx, int ny, double gamma) {
  const double uc = double(u[base + k]);
  double y = gamma * uc;
  if (i + 1 < nx) y += wh[base + k] * (uc - double(u[base + k + 1]));
  if (i > 0) y += wh[base + k - 1] * (uc - double(u[base + k - 1]));
  if (j + 1 < ny) y += wv[base + k] * (uc - double(u[base + k + nx]));
  if (j > 0) y += wv[base + k - nx] * (uc - double(u[base + k - nx]));
  return y;
}

__global__ void __launch_bounds__(kRedThreads)
tv_apply_kernel(const float* __restrict__ x, float* __restrict__ y, const double* __restrict__ wh,
                const double* __restrict__ wv, int nx, int ny, double gamma) {
  const int b = blockIdx.y;
  const size_t n = size_t(nx) * ny, base = size_t(b) * n;
  for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += size_t(gridDim.x) * blockDim.x) {
    const int j = int(k / nx), i = int(k - size_t(j) * nx);
    y[base + k] = float(mgamma_at(x, wh, wv, base, k, i, j, nx, ny, gamma));
  }
}

// smoothed TV value: block partials of sum_l sqrt((D x)_l^2 + beta)
__global__ void __launch_bounds__(kRedThreads)
tv_value_kernel(const float* __restrict__ x, int nx, int ny, double beta, double* __restrict__ part) {
  __shared__ double red[kRedThreads / 64];
  const int b = blockIdx.y;
  const size_t n = size_t(nx) * ny, base = size_t(b) * n;
  double acc = 0.0;
  for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += size_t(gridDim.x) * blockDim.x) {
    const int j = int(k / nx), i = int(k - size_t(j) * nx);
    const double xc = x[base + k];
    if (i + 1 < nx) {
      const double g = xc - double(x[base + k + 1]);
      acc += sqrt(g * g + beta);
    }
    if (j + 1 < ny) {
      const double g = xc - double(x[base + k + nx]);
      acc += sqrt(g * g + beta);
    }
  }
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) part[size_t(b) * kRedBlocks + blockIdx.x] = s;
}

// ---- multigrid V-cycle (levels as in MgLevel)
// y = (A u)_k at node (j, i) of a level: diagonal term plus edge differences
template <typename U>
__device__ __forceinline__ double level_op(const MgLevel& L, size_t base, int k, int i, int j, U u) {
  const double uc = u(k, i, j);
  double y = L.g[base + k] * uc;
  if (i + 1 < L.nx) y += L.wh[base + k] * (uc - u(k + 1, i + 1, j));
  if (i > 0) y += L.wh[base + k - 1] * (uc - u(k - 1, i - 1, j));
  if (j + 1 < L.ny) y += L.wv[base + k] * (uc - u(k + L.nx, i, j + 1));
  if (j > 0) y += L.wv[base + k - L.nx] * (uc - u(k - L.nx, i, j - 1));
  return y;
}

__global__ void __launch_bounds__(kRedThreads) mg_fill_kernel(double* __restrict__ a, size_t n, double v) {
  for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += size_t(gridDim.x) * blockDim.x) a[k] = v;
}

// coarse level operator from the finer one (one thread per coarse node)
__global__ void __launch_bounds__(kRedThreads) mg_coarsen_kernel(MgLevel f, MgLevel c) {
  const int b = blockIdx.y, nc = c.nx * c.ny;
  const size_t bf = size_t(b) * f.nx * f.ny, bc = size_t(b) * nc;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nc; k += gridDim.x * blockDim.x) {
    const int J = k / c.nx, I = k - J * c.nx, j0 = 2 * J, i0 = 2 * I;
    double g = 0.0, h = 0.0, v = 0.0;
    for (int j = j0; j < j0 + 2 && j < f.ny; ++j) {
      for (int i = i0; i < i0 + 2 && i < f.nx; ++i) g += f.g[bf + size_t(j) * f.nx + i];
      if (I + 1 < c.nx) h += f.wh[bf + size_t(j) * f.nx + i0 + 1];   // edge (j, i0+1)-(j, i0+2)
    }
    if (J + 1 < c.ny)
      for (int i = i0; i < i0 + 2 && i < f.nx; ++i) v += f.wv[bf + size_t(j0 + 1) * f.nx + i];
    c.g[bc + k] = g;
    c.wh[bc + k] = h;
    c.wv[bc + k] = v;
  }
}

__global__ void __launch_bounds__(kRedThreads) mg_diag_kernel(MgLevel L) {
  const int b = blockIdx.y, n = L.nx * L.ny;
  const size_t base = size_t(b) * n;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const int j = k / L.nx, i = k - j * L.nx;
    double d = L.g[base + k];
    if (i + 1 < L.nx) d += L.wh[base + k];
    if (i > 0) d += L.wh[base + k - 1];
    if (j + 1 < L.ny) d += L.wv[base + k];
    if (j > 0) d += L.wv[base + k - L.nx];
    L.dinv[base + k] = 1.0 / d;
  }
}

// first sweep from x = 0: x = om dinv b
__global__ void __launch_bounds__(kRedThreads) mg_scale_kernel(MgLevel L, double om) {
  const int b = blockIdx.y, n = L.nx * L.ny;
  const size_t base = size_t(b) * n;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
    L.x[base + k] = om * L.dinv[base + k] * L.b[base + k];
}

// coarse right-hand side: the aggregate sums of the residual b - A x of the
// first sweep from x = 0, x = om dinv b (recomputed where it is needed)
__global__ void __launch_bounds__(kRedThreads) mg_restrict_kernel(MgLevel f, MgLevel c, double om) {
  const int b = blockIdx.y, nc = c.nx * c.ny;
  const size_t bf = size_t(b) * f.nx * f.ny, bc = size_t(b) * nc;
  auto xf = [&](int kk, int, int) { return om * f.dinv[bf + kk] * f.b[bf + kk]; };
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nc; k += gridDim.x * blockDim.x) {
    const int J = k / c.nx, I = k - J * c.nx;
    double acc = 0.0;
    for (int j = 2 * J; j < 2 * J + 2 && j < f.ny; ++j)
      for (int i = 2 * I; i < 2 * I + 2 && i < f.nx; ++i) {
        const int kf = j * f.nx + i;
        acc += f.b[bf + kf] - level_op(f, bf, kf, i, j, xf);
      }
    c.b[bc + k] = acc;
  }
}

// coarse correction and post-smoothing: with x' = om dinv b + P xc (the
// first sweep's x, recomputed), t = x' + om dinv (b - A x')
__global__ void __launch_bounds__(kRedThreads) mg_post_kernel(MgLevel f, const double* __restrict__ xc, int nxc,
                                                               int nyc, double om) {
  const int b = blockIdx.y, n = f.nx * f.ny;
  const size_t bf = size_t(b) * n, bc = size_t(b) * nxc * nyc;
  auto xp = [&](int kk, int ii, int jj) {
    return om * f.dinv[bf + kk] * f.b[bf + kk] + xc[bc + size_t(jj >> 1) * nxc + (ii >> 1)];
  };
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const int j = k / f.nx, i = k - j * f.nx;
    const double y = level_op(f, bf, k, i, j, xp);
    f.t[bf + k] = xp(k, i, j) + om * f.dinv[bf + k] * (f.b[bf + k] - y);
  }
}

// ---- conjugate gradients for M_gamma z = r, per field (FP64)
// start: x = 0, r = rhs; partials of r.r (z and r.z follow the V-cycle)
__global__ void __launch_bounds__(kRedThreads)
cg_start_kernel(const float* __restrict__ rhs, TvCg c, int nx, int ny) {
  __shared__ double red[kRedThreads / 64];
  const int b = blockIdx.y;
  const size_t n = size_t(nx) * ny, base = size_t(b) * n;
  double rr = 0.0;
  for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += size_t(gridDim.x) * blockDim.x) {
    const double r = rhs[base + k];
    c.x[base + k] = 0.0;
    c.r[base + k] = r;
    rr += r * r;
  }
  const double s = block_sum(rr, red);
  if (threadIdx.x == 0) c.part_rr[size_t(b) * kRedBlocks + blockIdx.x] = s;
}

// partials of r.z for the z the V-cycle left; at the start also p = z
__global__ void __launch_bounds__(kRedThreads) cg_rz_kernel(TvCg c, int nx, int ny, int set_p) {
  __shared__ double red[kRedThreads / 64];
  const int b = blockIdx.y;
  const size_t n = size_t(nx) * ny, base = size_t(b) * n;
  double rz = 0.0;
  for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += size_t(gridDim.x) * blockDim.x) {
    const double z = c.z[base + k];
    rz += c.r[base + k] * z;
    if (set_p) c.p[base + k] = z;
  }
  const double s = block_sum(rz, red);
  if (threadIdx.x == 0) c.part_rz[size_t(b) * kRedBlocks + blockIdx.x] = s;
}

// totals of the start partials: rz[0][b], rr[b], bb[b] = r.r of the right-hand side
__global__ void __launch_bounds__(kRedThreads) cg_start_total_kernel(TvCg c) {
  __shared__ double red[kRedThreads / 64];
  const int b = blockIdx.x;
  const double rz = partial_total(c.part_rz, b, red);
  const double rr = partial_total(c.part_rr, b, red);
  if (threadIdx.x == 0) {
    c.rz[b] = rz;
    c.rr[b] = rr;
    c.rr_next[b] = rr;
    c.bb[b] = rr;
  }
}

// q = M_gamma p; partials of p.q.  Block (0, 0) also publishes the r.r of the
// previous iteration (nothing reads rr while this kernel runs).
__global__ void __launch_bounds__(kRedThreads) cg_q_kernel(TvCg c, int nx, int ny, double gamma) {
  __shared__ double red[kRedThreads / 64];
  const int b = blockIdx.y;
  if (blockIdx.x == 0 && blockIdx.y == 0)
    for (int t = threadIdx.x; t < int(gridDim.y); t += blockDim.x) c.rr[t] = c.rr_next[t];
  const size_t n = size_t(nx) * ny, base = size_t(b) * n;
  double pq = 0.0;
  for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += size_t(gridDim.x) * blockDim.x) {
    const int j = int(k / nx), i = int(k - size_t(j) * nx);
    const double q = mgamma_at(c.p, c.wh, c.wv, base, k, i, j, nx, ny, gamma);
    c.q[base + k] = q;
    pq += c.p[base + k] * q;
  }
  const double s = block_sum(pq, red);
  if (threadIdx.x == 0) c.part_pq[size_t(b) * kRedBlocks + blockIdx.x] = s;
}

// alpha = r.z / p.q (0 once the field has converged: r.r <= tol^2 b.b);
// x += alpha p; r -= alpha q; partials of the new r.r.  rz[par] holds the
// current r.z, the new one goes to rz[1 - par] (cg_dir).
__global__ void __launch_bounds__(kRedThreads)
cg_update_kernel(TvCg c, int nx, int ny, int par, double tol2) {
  __shared__ double red[kRedThreads / 64];
  const int b = blockIdx.y, nb = gridDim.y;
  const size_t n = size_t(nx) * ny, base = size_t(b) * n;
  const double pq = partial_total(c.part_pq, b, red);
  const double rz = c.rz[size_t(par) * nb + b];
  const bool live = c.rr[b] > tol2 * c.bb[b] && pq > 0.0;
  const double alpha = live ? rz / pq : 0.0;
  double rr = 0.0;
  for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += size_t(gridDim.x) * blockDim.x) {
    c.x[base + k] += alpha * c.p[base + k];
    const double r = c.r[base + k] - alpha * c.q[base + k];
    c.r[base + k] = r;
    rr += r * r;
  }
  const double s2 = block_sum(rr, red);
  if (threadIdx.x == 0) c.part_rr[size_t(b) * kRedBlocks + blockIdx.x] = s2;
}

// beta = r.z(new) / r.z(old); p = z + beta p; block 0 stores the new r.z and r.r.
__global__ void __launch_bounds__(kRedThreads)
cg_dir_kernel(TvCg c, int nx, int ny, int par, double tol2) {
  __shared__ double red[kRedThreads / 64];
  const int b = blockIdx.y, nb = gridDim.y;
  const size_t n = size_t(nx) * ny, base = size_t(b) * n;
  const double rzn = partial_total(c.part_rz, b, red);
  const double rr = partial_total(c.part_rr, b, red);
  const double rz = c.rz[size_t(par) * nb + b];
  const bool live = c.rr[b] > tol2 * c.bb[b];
  const double beta = (live && rz > 0.0) ? rzn / rz : 0.0;
  for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += size_t(gridDim.x) * blockDim.x)
    c.p[base + k] = c.z[base + k] + beta * c.p[base + k];
  // every block has read rz[par] and rr[b] above; the new values go to rz[1 - par]
  // and to rr_next, which the next cg_q publishes as rr
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c.rz[size_t(1 - par) * nb + b] = live ? rzn : rz;
    c.rr_next[b] = live ? rr : c.rr[b];
  }
}

__global__ void __launch_bounds__(kRedThreads)
cg_finish_kernel(TvCg c, float* __restrict__ out, int nx, int ny) {
  const int b = blockIdx.y;
  if (blockIdx.x == 0 && blockIdx.y == 0)
    for (int t = threadIdx.x; t < int(gridDim.y); t += blockDim.x) c.rr[t] = c.rr_next[t];
  const size_t n = size_t(nx) * ny, base = size_t(b) * n;
  for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += size_t(gridDim.x) * blockDim.x)
    out[base + k] = float(c.x[base + k]);
}

__global__ void __launch_bounds__(kRedThreads)
axpby_kernel(int64_t n, float a, const float* __restrict__ x, float b, float* __restrict__ y) {
  for (int64_t k = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += int64_t(gridDim.x) * blockDim.x)
    y[k] = a * x[k] + b * y[k];
}

// ---- PCG of Algorithm 4 with its scalars on the device, for `batch` fields
// of n values ([batch][n]); rz is the history r_i.z_i, [batch][rzs]
__global__ void __launch_bounds__(kRedThreads)
ld_dot_kernel(const float* __restrict__ a, const float* __restrict__ b, size_t n, double* __restrict__ part) {
  __shared__ double red[kRedThreads / 64];
  const size_t base = size_t(blockIdx.y) * n;
  double acc = 0.0;
  for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += size_t(gridDim.x) * blockDim.x)
    acc += double(a[base + k]) * double(b[base + k]);
  const double s = block_sum(acc, red);
  if (threadIdx.x == 0) part[size_t(blockIdx.y) * kRedBlocks + blockIdx.x] = s;
}

__global__ void __launch_bounds__(kRedThreads)
ld_total_kernel(const double* __restrict__ part, double* __restrict__ out, int ostride, double scale) {
  __shared__ double red[kRedThreads / 64];
  const double t = partial_total(part, blockIdx.x, red);
  if (threadIdx.x == 0) out[size_t(blockIdx.x) * ostride] = scale * t;
}

// which fields run PCG iteration i: not finished, i < i_max and (i < i_m or
// 1 - rz_i / rz_{i - i_m} > tol_in); a field that does not run is finished
__global__ void ld_live_kernel(int batch, const double* __restrict__ rz, int rzs, int i, int i_max, int i_m,
                               double tol_in, int* __restrict__ done, int* __restrict__ live) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= batch) return;
  bool l = !done[f] && i < i_max;
  if (l && i >= i_m) l = 1.0 - rz[size_t(f) * rzs + i] / rz[size_t(f) * rzs + i - i_m] > tol_in;
  live[f] = l ? 1 : 0;
  if (!l) done[f] = 1;
}

// alpha = rz_i / (d . H d);  sol += alpha d;  r -= alpha H d   (live fields)
__global__ void __launch_bounds__(kRedThreads)
ld_step_kernel(size_t n, const double* __restrict__ rz, int rzs, int i, const double* __restrict__ dhd,
               const int* __restrict__ live, const float* __restrict__ d, const float* __restrict__ hd,
               float* __restrict__ sol, float* __restrict__ r) {
  const int f = blockIdx.y;
  if (!live[f]) return;
  const float a = float(rz[size_t(f) * rzs + i] / dhd[f]);
  const size_t base = size_t(f) * n;
  for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += size_t(gridDim.x) * blockDim.x) {
    sol[base + k] = a * d[base + k] + sol[base + k];
    r[base + k] = -a * hd[base + k] + r[base + k];
  }
}

// hsol += alpha jd (live data sets): the data of the step that ld_step_kernel
// adds to sol, with the same FP32 alpha
__global__ void __launch_bounds__(kRedThreads)
ld_data_step_kernel(size_t nd, const double* __restrict__ rz, int rzs, int i, const double* __restrict__ dhd,
                    const int* __restrict__ live, const float* __restrict__ jd, float* __restrict__ hsol) {
  const int f = blockIdx.y;
  if (!live[f]) return;
  const float a = float(rz[size_t(f) * rzs + i] / dhd[f]);
  const size_t base = size_t(f) * nd;
  for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < nd; k += size_t(gridDim.x) * blockDim.x)
    hsol[base + k] = a * jd[base + k] + hsol[base + k];
}

// d = z + (rz_{i+1} / rz_i) d   (live fields)
__global__ void __launch_bounds__(kRedThreads)
ld_dir_kernel(size_t n, const double* __restrict__ rz, int rzs, int i, const int* __restrict__ live,
              const float* __restrict__ z, float* __restrict__ d) {
  const int f = blockIdx.y;
  if (!live[f]) return;
  const float bt = float(rz[size_t(f) * rzs + i + 1] / rz[size_t(f) * rzs + i]);
  const size_t base = size_t(f) * n;
  for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += size_t(gridDim.x) * blockDim.x)
    d[base + k] = 1.0f * z[base + k] + bt * d[base + k];
}

// x += sol for the fields whose flag is set (the outer step of Algorithm 5)
__global__ void __launch_bounds__(kRedThreads)
ld_add_kernel(size_t n, const int* __restrict__ flag, const float* __restrict__ sol, float* __restrict__ x) {
  const int f = blockIdx.y;
  if (!flag[f]) return;
  const size_t base = size_t(f) * n;
  for (size_t k = size_t(blockIdx.x) * blockDim.x + threadIdx.x; k < n; k += size_t(gridDim.x) * blockDim.x)
    x[base + k] = 1.0f * sol[base + k] + 1.0f * x[base + k];
}

}  // namespace

hipError_t launch_ld_dots(const float* a, const float* b, size_t n, int batch, double* part, double* out,
                          int ostride, double scale, hipStream_t st) {
  hipLaunchKernelGGL(ld_dot_kernel, dim3(kRedBlocks, batch), dim3(kRedThreads), 0, st, a, b, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(ld_total_kernel, dim3(batch), dim3(kRedThreads), 0, st, part, out, ostride, scale);
  return hipGetLastError();
}

hipError_t launch_ld_live(int batch, const double* rz, int rzs, int i, int i_max, int i_m, double tol_in, int* done,
                          int* live, hipStream_t st) {
  hipLaunchKernelGGL(ld_live_kernel, dim3((batch + 63) / 64), dim3(64), 0, st, batch, rz, rzs, i, i_max, i_m, tol_in,
                     done, live);
  return hipGetLastError();
}

hipError_t launch_ld_step(size_t n, int batch, const double* rz, int rzs, int i, const double* dhd, const int* live,
                          const float* d, const float* hd, float* sol, float* r, hipStream_t st) {
  hipLaunchKernelGGL(ld_step_kernel, dim3(kRedBlocks, batch), dim3(kRedThreads), 0, st, n, rz, rzs, i, dhd, live, d,
                     hd, sol, r);
  return hipGetLastError();
}

hipError_t launch_ld_data_step(size_t nd, int batch, const double* rz, int rzs, int i, const double* dhd,
                               const int* live, const float* jd, float* hsol, hipStream_t st) {
  hipLaunchKernelGGL(ld_data_step_kernel, dim3(kRedBlocks, batch), dim3(kRedThreads), 0, st, nd, rz, rzs, i, dhd, live,
                     jd, hsol);
  return hipGetLastError();
}

hipError_t launch_ld_dir(size_t n, int batch, const double* rz, int rzs, int i, const int* live, const float* z,
                         float* d, hipStream_t st) {
  hipLaunchKernelGGL(ld_dir_kernel, dim3(kRedBlocks, batch), dim3(kRedThreads), 0, st, n, rz, rzs, i, live, z, d);
  return hipGetLastError();
}

hipError_t launch_ld_add(size_t n, int batch, const int* flag, const float* sol, float* x, hipStream_t st) {
  hipLaunchKernelGGL(ld_add_kernel, dim3(kRedBlocks, batch), dim3(kRedThreads), 0, st, n, flag, sol, x);
  return hipGetLastError();
}

hipError_t launch_tv_weights(const float* x, int nx, int ny, int batch, double beta, double* wh, double* wv,
                             hipStream_t st) {
  hipLaunchKernelGGL(tv_weights_kernel, dim3(kRedBlocks, batch), dim3(kRedThreads), 0, st, x, nx, ny, beta, wh, wv);
  return hipGetLastError();
}

hipError_t launch_tv_apply(const float* x, float* y, const double* wh, const double* wv, int nx, int ny, int batch,
                           double gamma, hipStream_t st) {
  hipLaunchKernelGGL(tv_apply_kernel, dim3(kRedBlocks, batch), dim3(kRedThreads), 0, st, x, y, wh, wv, nx, ny, gamma);
  return hipGetLastError();
}

hipError_t launch_tv_value(const float* x, int nx, int ny, int batch, double beta, double* part, hipStream_t st) {
  hipLaunchKernelGGL(tv_value_kernel, dim3(kRedBlocks, batch), dim3(kRedThreads), 0, st, x, nx, ny, beta, part);
  return hipGetLastError();
}

namespace {

// blocks per field for a level of n nodes (grid-stride loops cover the rest)
dim3 level_grid(const MgLevel& L, int batch) {
  const int n = L.nx * L.ny;
  return dim3(unsigned(std::min(kRedBlocks, (n + kRedThreads - 1) / kRedThreads)), unsigned(batch));
}

// z = V-cycle applied to level 0's b; the result lands in level 0's t
hipError_t launch_vcycle(const MgLevel* lv, int nlev, int batch, hipStream_t st) {
  for (int l = 0; l + 1 < nlev; ++l)
    hipLaunchKernelGGL(mg_restrict_kernel, level_grid(lv[l + 1], batch), dim3(kRedThreads), 0, st, lv[l], lv[l + 1],
                       kMgOmega);
  // coarsest level: one node per field, solved exactly (x = b / diag)
  hipLaunchKernelGGL(mg_scale_kernel, level_grid(lv[nlev - 1], batch), dim3(kRedThreads), 0, st, lv[nlev - 1], 1.0);
  for (int l = nlev - 2; l >= 0; --l) {
    const double* xc = (l + 1 == nlev - 1) ? lv[l + 1].x : lv[l + 1].t;
    hipLaunchKernelGGL(mg_post_kernel, level_grid(lv[l], batch), dim3(kRedThreads), 0, st, lv[l], xc, lv[l + 1].nx,
                       lv[l + 1].ny, kMgOmega);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_mg_setup(const MgLevel* lv, int nlev, int batch, double gamma, hipStream_t st) {
  const size_t n0 = size_t(lv[0].nx) * lv[0].ny * batch;
  hipLaunchKernelGGL(mg_fill_kernel, dim3(unsigned(std::min<size_t>(4096, (n0 + kRedThreads - 1) / kRedThreads))),
                     dim3(kRedThreads), 0, st, lv[0].g, n0, gamma);
  for (int l = 0; l + 1 < nlev; ++l)
    hipLaunchKernelGGL(mg_coarsen_kernel, level_grid(lv[l + 1], batch), dim3(kRedThreads), 0, st, lv[l], lv[l + 1]);
  for (int l = 0; l < nlev; ++l)
    hipLaunchKernelGGL(mg_diag_kernel, level_grid(lv[l], batch), dim3(kRedThreads), 0, st, lv[l]);
  return hipGetLastError();
}

hipError_t launch_cg_start(const float* rhs, const TvCg& c, const MgLevel* lv, int nlev, int nx, int ny, int batch,
                           hipStream_t st) {
  hipLaunchKernelGGL(cg_start_kernel, dim3(kRedBlocks, batch), dim3(kRedThreads), 0, st, rhs, c, nx, ny);
  hipError_t e = launch_vcycle(lv, nlev, batch, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cg_rz_kernel, dim3(kRedBlocks, batch), dim3(kRedThreads), 0, st, c, nx, ny, 1);
  hipLaunchKernelGGL(cg_start_total_kernel, dim3(batch), dim3(kRedThreads), 0, st, c);
  return hipGetLastError();
}

hipError_t launch_cg_iteration(const TvCg& c, const MgLevel* lv, int nlev, int nx, int ny, int batch, double gamma,
                               int par, double tol2, hipStream_t st) {
  hipLaunchKernelGGL(cg_q_kernel, dim3(kRedBlocks, batch), dim3(kRedThreads), 0, st, c, nx, ny, gamma);
  hipLaunchKernelGGL(cg_update_kernel, dim3(kRedBlocks, batch), dim3(kRedThreads), 0, st, c, nx, ny, par, tol2);
  hipError_t e = launch_vcycle(lv, nlev, batch, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(cg_rz_kernel, dim3(kRedBlocks, batch), dim3(kRedThreads), 0, st, c, nx, ny, 0);
  hipLaunchKernelGGL(cg_dir_kernel, dim3(kRedBlocks, batch), dim3(kRedThreads), 0, st, c, nx, ny, par, tol2);
  return hipGetLastError();
}

// publishes the last r.r (the convergence test reads rr) and writes the solution
hipError_t launch_cg_finish(const TvCg& c, float* out, int nx, int ny, int batch, hipStream_t st) {
  hipLaunchKernelGGL(cg_finish_kernel, dim3(kRedBlocks, batch), dim3(kRedThreads), 0, st, c, out, nx, ny);
  return hipGetLastError();
}

hipError_t launch_axpby(int64_t n, float a, const float* x, float b, float* y, hipStream_t st) {
  int64_t blocks = (n + kRedThreads - 1) / kRedThreads;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(axpby_kernel, dim3(unsigned(blocks)), dim3(kRedThreads), 0, st, n, a, x, b, y);
  return hipGetLastError();
}

}  // namespace qpat
