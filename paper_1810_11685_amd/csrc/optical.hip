// Optical operators of Section 3.1 on the GPU: the P1 Galerkin system
// A_o = K[kappa] + C[mu] + R of the diffusion approximation with its Robin
// condition (eqs var_fo, system_forward2) on the grid-matched triangulation,
// its solution by FP64 conjugate gradients (preconditioned by one multigrid
// V-cycle of 2 x 2 node aggregation with Galerkin coarse stencils), the
// heating map H = mu o I Phi (eq forward_out), J_o (eq dh_des) and J_o^*
// (eqs system_adjoint, system_adjoint1, prodtproj).
//
// Mesh: nx x ny square pixels of side h; FEM nodes are the pixel corners,
// node (r, c) = r (nx + 1) + c; pixel (j, i) holds element 2 (j nx + i) with
// corners (j,i), (j,i+1), (j+1,i+1) and element 2 (j nx + i) + 1 with corners
// (j,i), (j+1,i+1), (j+1,i).  A is applied matrix-free by gathering, at every
// node, the rows of the (at most six) incident element matrices and of the
// boundary edges: no atomics, a fixed summation order.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "optical_internal.hpp"

namespace qpat {

namespace {

constexpr double kGamma2 = 0.31830988618379067154;  // gamma_2 = 1/pi

// P1 stiffness of the two element shapes without kappa (S grad phi_a . grad phi_b,
// independent of h in 2-D) and the P1 mass pattern (times S/12).
__device__ __forceinline__ double kloc(int shape, int a, int b) {
  // shape 0: [[1,-1,0],[-1,2,-1],[0,-1,1]] / 2; shape 1: [[1,0,-1],[0,1,-1],[-1,-1,2]] / 2
  if (shape == 0) {
    const int d = a > b ? a - b : b - a;
    if (a == b) return a == 1 ? 1.0 : 0.5;
    return d == 1 ? -0.5 : 0.0;
  }
  if (a == b) return a == 2 ? 1.0 : 0.5;
  return (a == 2 || b == 2) ? -0.5 : 0.0;
}
__device__ __forceinline__ double mloc(int a, int b) { return a == b ? 2.0 / 12.0 : 1.0 / 12.0; }

// local index of pixel corner (lr, lc) in element shape 0 / 1 (-1: not a vertex)
__device__ __forceinline__ int local0(int lr, int lc) { return lr == 0 ? (lc == 0 ? 0 : 1) : (lc == 1 ? 2 : -1); }
__device__ __forceinline__ int local1(int lr, int lc) { return lr == 0 ? (lc == 0 ? 0 : -1) : (lc == 1 ? 1 : 2); }

struct Pix {
  int n[4];  // corners (j,i), (j,i+1), (j+1,i+1), (j+1,i)
};
__device__ __forceinline__ Pix pixel(int j, int i, int nx) {
  const int w = nx + 1;
  return Pix{{j * w + i, j * w + i + 1, (j + 1) * w + i + 1, (j + 1) * w + i}};
}
// vertex b of element shape s as a pixel corner index
__device__ __forceinline__ int vert(int s, int b) { return s == 0 ? b : (b == 0 ? 0 : b == 1 ? 2 : 3); }

// (K[ka] + C[mu] (+ R)) x at node (r, c); ka, mu elemental; with `robin` the
// boundary term 2 gamma int phi_k phi_p ds is added (edge mass h/6 [[2,1],[1,2]]).
template <typename T>
__device__ double apply_at(const T* __restrict__ x, const double* __restrict__ ka, const double* __restrict__ mu,
                           int r, int c, int nx, int ny, double h, bool robin) {
  double y = 0.0;
  const double ms = 0.5 * h * h;  // element area
  for (int dj = -1; dj <= 0; ++dj) {
    const int j = r + dj;
    if (j < 0 || j >= ny) continue;
    for (int di = -1; di <= 0; ++di) {
      const int i = c + di;
      if (i < 0 || i >= nx) continue;
      const Pix P = pixel(j, i, nx);
      const int lr = r - j, lc = c - i;
      const int e = 2 * (j * nx + i);
      const int a0 = local0(lr, lc), a1 = local1(lr, lc);
      if (a0 >= 0) {
        double k = 0.0, m = 0.0;
        for (int b = 0; b < 3; ++b) {
          const double xb = double(x[P.n[vert(0, b)]]);
          k += kloc(0, a0, b) * xb;
          m += mloc(a0, b) * xb;
        }
        y += ka[e] * k + mu[e] * ms * m;
      }
      if (a1 >= 0) {
        double k = 0.0, m = 0.0;
        for (int b = 0; b < 3; ++b) {
          const double xb = double(x[P.n[vert(1, b)]]);
          k += kloc(1, a1, b) * xb;
          m += mloc(a1, b) * xb;
        }
        y += ka[e + 1] * k + mu[e + 1] * ms * m;
      }
    }
  }
  if (robin) {
    const double w = 2.0 * kGamma2 * h / 6.0;
    const int W = nx + 1;
    const double xc = double(x[r * W + c]);
    if (r == 0 || r == ny) {  // bottom / top edges along x
      if (c > 0) y += w * (2.0 * xc + double(x[r * W + c - 1]));
      if (c < nx) y += w * (2.0 * xc + double(x[r * W + c + 1]));
    }
    if (c == 0 || c == nx) {  // left / right edges along y
      if (r > 0) y += w * (2.0 * xc + double(x[(r - 1) * W + c]));
      if (r < ny) y += w * (2.0 * xc + double(x[(r + 1) * W + c]));
    }
  }
  return y;
}

__device__ double diag_at(const double* __restrict__ ka, const double* __restrict__ mu, int r, int c, int nx,
                          int ny, double h) {
  double d = 0.0;
  const double ms = 0.5 * h * h;
  for (int dj = -1; dj <= 0; ++dj) {
    const int j = r + dj;
    if (j < 0 || j >= ny) continue;
    for (int di = -1; di <= 0; ++di) {
      const int i = c + di;
      if (i < 0 || i >= nx) continue;
      const int lr = r - j, lc = c - i, e = 2 * (j * nx + i);
      const int a0 = local0(lr, lc), a1 = local1(lr, lc);
      if (a0 >= 0) d += ka[e] * kloc(0, a0, a0) + mu[e] * ms * mloc(a0, a0);
      if (a1 >= 0) d += ka[e + 1] * kloc(1, a1, a1) + mu[e + 1] * ms * mloc(a1, a1);
    }
  }
  const double w = 2.0 * kGamma2 * h / 6.0;
  if (r == 0 || r == ny) d += w * (2.0 * (c > 0) + 2.0 * (c < nx));
  if (c == 0 || c == nx) d += w * (2.0 * (r > 0) + 2.0 * (r < ny));
  return d;
}

__device__ __forceinline__ double wave_sum_d(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum_d(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kOptThreads / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}
__device__ __forceinline__ double partial_total(const double* __restrict__ part, int b, int nblk, double* red) {
  double v = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) v += part[size_t(b) * kOptBlocks + i];
  __shared__ double tot;
  const double s = block_sum(v, red);
  if (threadIdx.x == 0) tot = s;
  __syncthreads();
  return tot;
}

#define FOR_NODES(k)                                                                         \
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < c.nn; k += gridDim.x * blockDim.x)
#define FOR_ELEMS(e)                                                                         \
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < c.ne; e += gridDim.x * blockDim.x)

// coefficients of field b in FP64
__global__ void __launch_bounds__(kOptThreads) opt_set_kernel(OptCg c, const float* __restrict__ kappa,
                                                              const float* __restrict__ mu) {
  const int b = blockIdx.y;
  const size_t be = size_t(b) * c.ne;
  FOR_ELEMS(e) {
    c.ka[be + e] = kappa[be + e];
    c.mu[be + e] = mu[be + e];
  }
}

// right-hand sides.  mode 0: G of constant side currents cur[b][4] (bottom,
// top, left, right): int 2 I phi_p ds = I h per edge end;  mode 1:
// -(K[dka] + C[dmu]) Phi0;  mode 2: -I^+(mu o H) = -(S/3) sum_{e at p} mu_e H_e.
__global__ void __launch_bounds__(kOptThreads)
opt_rhs_kernel(OptCg c, int mode, const double* __restrict__ cur, const float* __restrict__ Hin) {
  const int b = blockIdx.y;
  const size_t bn = size_t(b) * c.nn, be = size_t(b) * c.ne;
  const int W = c.nx + 1;
  FOR_NODES(k) {
    const int r = k / W, col = k - r * W;
    double v = 0.0;
    if (mode == 0) {
      const double* I = cur + 4 * b;
      if (r == 0) v += I[0] * c.h * ((col > 0) + (col < c.nx));
      if (r == c.ny) v += I[1] * c.h * ((col > 0) + (col < c.nx));
      if (col == 0) v += I[2] * c.h * ((r > 0) + (r < c.ny));
      if (col == c.nx) v += I[3] * c.h * ((r > 0) + (r < c.ny));
    } else if (mode == 1) {
      // the perturbations, staged in FP64 by opt_stage_kernel
      v = -apply_at(c.phi + bn, c.ek + be, c.em + be, r, col, c.nx, c.ny, c.h, false);
    } else {
      const double s3 = 0.5 * c.h * c.h / 3.0;
      for (int dj = -1; dj <= 0; ++dj) {
        const int j = r + dj;
        if (j < 0 || j >= c.ny) continue;
        for (int di = -1; di <= 0; ++di) {
          const int i = col + di;
          if (i < 0 || i >= c.nx) continue;
          const int lr = r - j, lc = col - i, e = 2 * (j * c.nx + i);
          if (local0(lr, lc) >= 0) v -= s3 * c.mu[be + e] * double(Hin[be + e]);
          if (local1(lr, lc) >= 0) v -= s3 * c.mu[be + e + 1] * double(Hin[be + e + 1]);
        }
      }
    }
    c.rhs[bn + k] = v;
  }
}

// element perturbations to FP64 scratch (mode 1 of opt_rhs_kernel)
__global__ void __launch_bounds__(kOptThreads) opt_stage_kernel(OptCg c, const float* __restrict__ da,
                                                                const float* __restrict__ dm) {
  const int b = blockIdx.y;
  const size_t be = size_t(b) * c.ne;
  FOR_ELEMS(e) {
    c.ek[be + e] = da[be + e];
    c.em[be + e] = dm[be + e];
  }
}

// ---- multigrid V-cycle (levels as in OptLevel)
// fine-mesh element indices of pixel (j, i)
__device__ __forceinline__ int elem0(int j, int i, int nx) { return 2 * (j * nx + i); }

// Level 0 stencil of A_o at node (r, col): the diagonal (diag_at), and the
// entries for the east edge (bottom edge of pixel (r, col), element shape 0;
// top edge of pixel (r - 1, col), shape 1), the north edge (left edge of
// pixel (r, col), shape 1; right edge of pixel (r, col - 1), shape 0) and the
// north-east diagonal of pixel (r, col) (mass of both elements; the P1
// stiffness across a right angle's hypotenuse is 0); boundary edges add the
// Robin edge mass.
__global__ void __launch_bounds__(kOptThreads) opt_mg_stencil_kernel(OptCg c, OptLevel L) {
  const int b = blockIdx.y;
  const size_t bn = size_t(b) * c.nn, be = size_t(b) * c.ne;
  const double* ka = c.ka + be;
  const double* mu = c.mu + be;
  const int W = c.nx + 1, nx = c.nx, ny = c.ny;
  const double ms = 0.5 * c.h * c.h, w = 2.0 * kGamma2 * c.h / 6.0;
  FOR_NODES(k) {
    const int r = k / W, col = k - r * W;
    const double d = diag_at(ka, mu, r, col, nx, ny, c.h);
    double e = 0.0, n = 0.0, g = 0.0;
    if (col < nx) {
      if (r < ny) e += -0.5 * ka[elem0(r, col, nx)] + ms / 12.0 * mu[elem0(r, col, nx)];
      if (r > 0) e += -0.5 * ka[elem0(r - 1, col, nx) + 1] + ms / 12.0 * mu[elem0(r - 1, col, nx) + 1];
      if (r == 0 || r == ny) e += w;
    }
    if (r < ny) {
      if (col < nx) n += -0.5 * ka[elem0(r, col, nx) + 1] + ms / 12.0 * mu[elem0(r, col, nx) + 1];
      if (col > 0) n += -0.5 * ka[elem0(r, col - 1, nx)] + ms / 12.0 * mu[elem0(r, col - 1, nx)];
      if (col == 0 || col == nx) n += w;
    }
    if (r < ny && col < nx) g = ms / 12.0 * (mu[elem0(r, col, nx)] + mu[elem0(r, col, nx) + 1]);
    L.sc[bn + k] = d;
    L.se[bn + k] = e;
    L.sn[bn + k] = n;
    L.sd[bn + k] = g;
    L.dinv[bn + k] = 1.0 / d;
  }
}

// (A u)_k at node (j, i) of a level, u(k, i, j) the iterate
template <typename U>
__device__ __forceinline__ double stencil_op(const OptLevel& L, size_t base, int k, int i, int j, U u) {
  const int nx = L.nx;
  double y = L.sc[base + k] * u(k, i, j);
  if (i + 1 < nx) y += L.se[base + k] * u(k + 1, i + 1, j);
  if (i > 0) y += L.se[base + k - 1] * u(k - 1, i - 1, j);
  if (j + 1 < L.ny) y += L.sn[base + k] * u(k + nx, i, j + 1);
  if (j > 0) y += L.sn[base + k - nx] * u(k - nx, i, j - 1);
  if (j + 1 < L.ny && i + 1 < nx) y += L.sd[base + k] * u(k + nx + 1, i + 1, j + 1);
  if (j > 0 && i > 0) y += L.sd[base + k - nx - 1] * u(k - nx - 1, i - 1, j - 1);
  return y;
}

// Galerkin coarse stencil P^T A P of 2 x 2 aggregates (one thread per coarse
// node): the diagonal sums the aggregate's diagonal and twice its inner
// couplings; a coarse coupling sums the fine couplings between two aggregates
__global__ void __launch_bounds__(kOptThreads) opt_mg_coarsen_kernel(OptLevel f, OptLevel c) {
  const int b = blockIdx.y, nc = c.nx * c.ny;
  const size_t bf = size_t(b) * f.nx * f.ny, bc = size_t(b) * nc;
  auto F = [&](const double* a, int j, int i) { return (j < f.ny && i < f.nx) ? a[bf + size_t(j) * f.nx + i] : 0.0; };
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nc; k += gridDim.x * blockDim.x) {
    const int J = k / c.nx, I = k - J * c.nx, j = 2 * J, i = 2 * I;
    const double d = F(f.sc, j, i) + F(f.sc, j, i + 1) + F(f.sc, j + 1, i) + F(f.sc, j + 1, i + 1) +
                     2.0 * (F(f.se, j, i) + F(f.se, j + 1, i) + F(f.sn, j, i) + F(f.sn, j, i + 1) + F(f.sd, j, i));
    const bool east = I + 1 < c.nx, north = J + 1 < c.ny;
    c.sc[bc + k] = d;
    c.se[bc + k] = east ? F(f.se, j, i + 1) + F(f.se, j + 1, i + 1) + F(f.sd, j, i + 1) : 0.0;
    c.sn[bc + k] = north ? F(f.sn, j + 1, i) + F(f.sn, j + 1, i + 1) + F(f.sd, j + 1, i) : 0.0;
    c.sd[bc + k] = (east && north) ? F(f.sd, j + 1, i + 1) : 0.0;
    c.dinv[bc + k] = 1.0 / d;
  }
}

// first sweep from x = 0: x = om dinv b
__global__ void __launch_bounds__(kOptThreads) opt_mg_scale_kernel(OptLevel L, double om) {
  const int b = blockIdx.y, n = L.nx * L.ny;
  const size_t base = size_t(b) * n;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x)
    L.x[base + k] = om * L.dinv[base + k] * L.b[base + k];
}

// coarse right-hand side: aggregate sums of the residual b - A x of the first
// sweep from x = 0, x = om dinv b (recomputed where it is needed rather than stored)
__global__ void __launch_bounds__(kOptThreads) opt_mg_restrict_kernel(OptLevel f, OptLevel c, double om) {
  const int b = blockIdx.y, nc = c.nx * c.ny;
  const size_t bf = size_t(b) * f.nx * f.ny, bc = size_t(b) * nc;
  auto xf = [&](int kk, int, int) { return om * f.dinv[bf + kk] * f.b[bf + kk]; };
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nc; k += gridDim.x * blockDim.x) {
    const int J = k / c.nx, I = k - J * c.nx;
    double acc = 0.0;
    for (int j = 2 * J; j < 2 * J + 2 && j < f.ny; ++j)
      for (int i = 2 * I; i < 2 * I + 2 && i < f.nx; ++i) {
        const int kf = j * f.nx + i;
        acc += f.b[bf + kf] - stencil_op(f, bf, kf, i, j, xf);
      }
    c.b[bc + k] = acc;
  }
}

// coarse correction and post-smoothing: x' = om dinv b + P xc (the first
// sweep's x, recomputed); t = x' + om dinv (b - A x')
__global__ void __launch_bounds__(kOptThreads) opt_mg_post_kernel(OptLevel f, const double* __restrict__ xc,
                                                                   int nxc, int nyc, double om) {
  const int b = blockIdx.y, n = f.nx * f.ny;
  const size_t bf = size_t(b) * n, bc = size_t(b) * nxc * nyc;
  auto xp = [&](int kk, int ii, int jj) {
    return om * f.dinv[bf + kk] * f.b[bf + kk] + xc[bc + size_t(jj >> 1) * nxc + (ii >> 1)];
  };
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) {
    const int j = k / f.nx, i = k - j * f.nx;
    const double y = stencil_op(f, bf, k, i, j, xp);
    f.t[bf + k] = xp(k, i, j) + om * f.dinv[bf + k] * (f.b[bf + k] - y);
  }
}

// CG start: x = 0, r = rhs; partials of r.r (z and r.z follow the V-cycle)
__global__ void __launch_bounds__(kOptThreads) opt_cg_start_kernel(OptCg c) {
  __shared__ double red[kOptThreads / 64];
  const int b = blockIdx.y;
  const size_t bn = size_t(b) * c.nn;
  double rr = 0.0;
  FOR_NODES(k) {
    const double rv = c.rhs[bn + k];
    c.x[bn + k] = 0.0;
    c.r[bn + k] = rv;
    rr += rv * rv;
  }
  const double s = block_sum(rr, red);
  if (threadIdx.x == 0) c.part_rr[size_t(b) * kOptBlocks + blockIdx.x] = s;
}

// partials of r.z for the z the V-cycle left; at the start also p = z
__global__ void __launch_bounds__(kOptThreads) opt_cg_rz_kernel(OptCg c, int set_p) {
  __shared__ double red[kOptThreads / 64];
  const int b = blockIdx.y;
  const size_t bn = size_t(b) * c.nn;
  double rz = 0.0;
  FOR_NODES(k) {
    const double z = c.z[bn + k];
    rz += c.r[bn + k] * z;
    if (set_p) c.p[bn + k] = z;
  }
  const double s = block_sum(rz, red);
  if (threadIdx.x == 0) c.part_rz[size_t(b) * kOptBlocks + blockIdx.x] = s;
}

__global__ void __launch_bounds__(kOptThreads) opt_cg_start_total_kernel(OptCg c) {
  __shared__ double red[kOptThreads / 64];
  const int b = blockIdx.x;
  const double rz = partial_total(c.part_rz, b, c.nblk, red);
  const double rr = partial_total(c.part_rr, b, c.nblk, red);
  if (threadIdx.x == 0) {
    c.rz[b] = rz;
    c.rr[b] = rr;
    c.rr_next[b] = rr;
    c.bb[b] = rr;
  }
}

// q = A p, partials of p.q; block (0, 0) publishes the previous r.r
__global__ void __launch_bounds__(kOptThreads) opt_cg_q_kernel(OptCg c) {
  __shared__ double red[kOptThreads / 64];
  const int b = blockIdx.y;
  if (blockIdx.x == 0 && blockIdx.y == 0)
    for (int t = threadIdx.x; t < int(gridDim.y); t += blockDim.x) c.rr[t] = c.rr_next[t];
  const size_t bn = size_t(b) * c.nn, be = size_t(b) * c.ne;
  const int W = c.nx + 1;
  double pq = 0.0;
  FOR_NODES(k) {
    const int r = k / W, col = k - r * W;
    const double q = apply_at(c.p + bn, c.ka + be, c.mu + be, r, col, c.nx, c.ny, c.h, true);
    c.q[bn + k] = q;
    pq += c.p[bn + k] * q;
  }
  const double s = block_sum(pq, red);
  if (threadIdx.x == 0) c.part_pq[size_t(b) * kOptBlocks + blockIdx.x] = s;
}

// alpha = r.z / p.q (0 once converged); x += alpha p; r -= alpha q; partials of the new r.r
__global__ void __launch_bounds__(kOptThreads) opt_cg_update_kernel(OptCg c, int par, double tol2) {
  __shared__ double red[kOptThreads / 64];
  const int b = blockIdx.y, nb = gridDim.y;
  const size_t bn = size_t(b) * c.nn;
  const double pq = partial_total(c.part_pq, b, c.nblk, red);
  const double rz = c.rz[size_t(par) * nb + b];
  const bool live = c.rr[b] > tol2 * c.bb[b] && pq > 0.0;
  const double alpha = live ? rz / pq : 0.0;
  double rr = 0.0;
  FOR_NODES(k) {
    c.x[bn + k] += alpha * c.p[bn + k];
    const double rv = c.r[bn + k] - alpha * c.q[bn + k];
    c.r[bn + k] = rv;
    rr += rv * rv;
  }
  const double s2 = block_sum(rr, red);
  if (threadIdx.x == 0) c.part_rr[size_t(b) * kOptBlocks + blockIdx.x] = s2;
}

// beta = rz_new / rz; p = z + beta p; block (0, b) stores rz_new, rr_next
__global__ void __launch_bounds__(kOptThreads) opt_cg_dir_kernel(OptCg c, int par) {
  __shared__ double red[kOptThreads / 64];
  const int b = blockIdx.y, nb = gridDim.y;
  const size_t bn = size_t(b) * c.nn;
  const double rzn = partial_total(c.part_rz, b, c.nblk, red);
  const double rrn = partial_total(c.part_rr, b, c.nblk, red);
  const double rz = c.rz[size_t(par) * nb + b];
  const double beta = rz > 0.0 ? rzn / rz : 0.0;
  FOR_NODES(k) c.p[bn + k] = c.z[bn + k] + beta * c.p[bn + k];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    c.rz[size_t(1 - par) * nb + b] = rzn;
    c.rr_next[b] = rrn;
  }
}

__global__ void __launch_bounds__(kOptThreads) opt_cg_finish_kernel(OptCg c) {
  for (int t = threadIdx.x; t < c.batch; t += blockDim.x) c.rr[t] = c.rr_next[t];
}

// outputs. mode 0 (forward): phi = x; H = mu o I phi.  mode 1 (J_o): dH =
// dmu o I phi + mu o I x.  mode 2 (J_o^*): gk = grad x . grad phi,
// gm = (1/12) x_e^T [[2,1,1],[1,2,1],[1,1,2]] phi_e + H o I phi.
__global__ void __launch_bounds__(kOptThreads)
opt_out_kernel(OptCg c, int mode, const float* __restrict__ Hin, float* __restrict__ o1, float* __restrict__ o2) {
  const int b = blockIdx.y;
  const size_t bn = size_t(b) * c.nn, be = size_t(b) * c.ne;
  if (mode == 0) FOR_NODES(k) c.phi[bn + k] = c.x[bn + k];
  FOR_ELEMS(e) {
    const int pix = e >> 1, s = e & 1, j = pix / c.nx, i = pix - j * c.nx;
    const Pix P = pixel(j, i, c.nx);
    const int v0 = P.n[vert(s, 0)], v1 = P.n[vert(s, 1)], v2 = P.n[vert(s, 2)];
    const double f0 = mode == 0 ? c.x[bn + v0] : c.phi[bn + v0];
    const double f1 = mode == 0 ? c.x[bn + v1] : c.phi[bn + v1];
    const double f2 = mode == 0 ? c.x[bn + v2] : c.phi[bn + v2];
    const double If = (f0 + f1 + f2) / 3.0;
    if (mode == 0) {
      o1[be + e] = float(c.mu[be + e] * If);
    } else if (mode == 1) {
      const double Ix = (c.x[bn + v0] + c.x[bn + v1] + c.x[bn + v2]) / 3.0;
      o1[be + e] = float(c.em[be + e] * If + c.mu[be + e] * Ix);
    } else {
      const double x0 = c.x[bn + v0], x1 = c.x[bn + v1], x2 = c.x[bn + v2];
      // element gradients (h = side): shape 0 (x-step, y-step) = (u1 - u0, u2 - u1)/h,
      // shape 1 = (u1 - u2, u2 - u0)/h
      double gx0, gy0, gx1, gy1;
      if (s == 0) {
        gx0 = x1 - x0; gy0 = x2 - x1; gx1 = f1 - f0; gy1 = f2 - f1;
      } else {
        gx0 = x1 - x2; gy0 = x2 - x0; gx1 = f1 - f2; gy1 = f2 - f0;
      }
      o1[be + e] = float((gx0 * gx1 + gy0 * gy1) / (c.h * c.h));
      const double m = (2.0 * x0 * f0 + 2.0 * x1 * f1 + 2.0 * x2 * f2 + x0 * (f1 + f2) + x1 * (f0 + f2) +
                        x2 * (f0 + f1)) / 12.0;
      o2[be + e] = float(m + double(Hin[be + e]) * If);
    }
  }
}

// pixel maps: p = mean of the pixel's two elements; transpose: half to each
__global__ void __launch_bounds__(kOptThreads) opt_pixels_kernel(const float* __restrict__ H, float* __restrict__ p,
                                                                 int npix, int transpose) {
  const size_t b = blockIdx.y;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < npix; k += gridDim.x * blockDim.x) {
    if (!transpose) {
      p[b * npix + k] = 0.5f * (H[b * 2 * npix + 2 * k] + H[b * 2 * npix + 2 * k + 1]);
    } else {
      const float v = 0.5f * H[b * npix + k];
      p[b * 2 * npix + 2 * k] = v;
      p[b * 2 * npix + 2 * k + 1] = v;
    }
  }
}

}  // namespace

hipError_t opt_launch_set(const OptCg& c, const float* kappa, const float* mu, hipStream_t st) {
  hipLaunchKernelGGL(opt_set_kernel, dim3(c.nblk, c.batch), dim3(kOptThreads), 0, st, c, kappa, mu);
  return hipGetLastError();
}
hipError_t opt_launch_stage(const OptCg& c, const float* da, const float* dm, hipStream_t st) {
  hipLaunchKernelGGL(opt_stage_kernel, dim3(c.nblk, c.batch), dim3(kOptThreads), 0, st, c, da, dm);
  return hipGetLastError();
}
hipError_t opt_launch_rhs(const OptCg& c, int mode, const double* cur, const float* Hin, hipStream_t st) {
  hipLaunchKernelGGL(opt_rhs_kernel, dim3(c.nblk, c.batch), dim3(kOptThreads), 0, st, c, mode, cur, Hin);
  return hipGetLastError();
}
namespace {

// blocks per field for a level of n nodes (grid-stride loops cover the rest)
dim3 level_grid(const OptLevel& L, int batch) {
  const int n = L.nx * L.ny;
  return dim3(unsigned(n < kOptBlocks * kOptThreads ? (n + kOptThreads - 1) / kOptThreads : kOptBlocks),
              unsigned(batch));
}

// z = V-cycle applied to level 0's b; the result lands in level 0's t
void launch_vcycle(const OptLevel* lv, int nlev, int batch, hipStream_t st) {
  for (int l = 0; l + 1 < nlev; ++l)
    hipLaunchKernelGGL(opt_mg_restrict_kernel, level_grid(lv[l + 1], batch), dim3(kOptThreads), 0, st, lv[l],
                       lv[l + 1], kOptMgOmega);
  // coarsest level: one node per field, solved exactly (x = b / diag)
  hipLaunchKernelGGL(opt_mg_scale_kernel, level_grid(lv[nlev - 1], batch), dim3(kOptThreads), 0, st, lv[nlev - 1],
                     1.0);
  for (int l = nlev - 2; l >= 0; --l) {
    const double* xc = (l + 1 == nlev - 1) ? lv[l + 1].x : lv[l + 1].t;
    hipLaunchKernelGGL(opt_mg_post_kernel, level_grid(lv[l], batch), dim3(kOptThreads), 0, st, lv[l], xc,
                       lv[l + 1].nx, lv[l + 1].ny, kOptMgOmega);
  }
}

}  // namespace

hipError_t opt_launch_mg_setup(const OptCg& c, const OptLevel* lv, int nlev, hipStream_t st) {
  hipLaunchKernelGGL(opt_mg_stencil_kernel, dim3(c.nblk, c.batch), dim3(kOptThreads), 0, st, c, lv[0]);
  for (int l = 0; l + 1 < nlev; ++l)
    hipLaunchKernelGGL(opt_mg_coarsen_kernel, level_grid(lv[l + 1], c.batch), dim3(kOptThreads), 0, st, lv[l],
                       lv[l + 1]);
  return hipGetLastError();
}
hipError_t opt_launch_cg_start(const OptCg& c, const OptLevel* lv, int nlev, hipStream_t st) {
  hipLaunchKernelGGL(opt_cg_start_kernel, dim3(c.nblk, c.batch), dim3(kOptThreads), 0, st, c);
  launch_vcycle(lv, nlev, c.batch, st);
  hipLaunchKernelGGL(opt_cg_rz_kernel, dim3(c.nblk, c.batch), dim3(kOptThreads), 0, st, c, 1);
  hipLaunchKernelGGL(opt_cg_start_total_kernel, dim3(c.batch), dim3(kOptThreads), 0, st, c);
  return hipGetLastError();
}
hipError_t opt_launch_cg_iteration(const OptCg& c, const OptLevel* lv, int nlev, int par, double tol2,
                                   hipStream_t st) {
  hipLaunchKernelGGL(opt_cg_q_kernel, dim3(c.nblk, c.batch), dim3(kOptThreads), 0, st, c);
  hipLaunchKernelGGL(opt_cg_update_kernel, dim3(c.nblk, c.batch), dim3(kOptThreads), 0, st, c, par, tol2);
  launch_vcycle(lv, nlev, c.batch, st);
  hipLaunchKernelGGL(opt_cg_rz_kernel, dim3(c.nblk, c.batch), dim3(kOptThreads), 0, st, c, 0);
  hipLaunchKernelGGL(opt_cg_dir_kernel, dim3(c.nblk, c.batch), dim3(kOptThreads), 0, st, c, par);
  return hipGetLastError();
}
hipError_t opt_launch_cg_finish(const OptCg& c, hipStream_t st) {
  hipLaunchKernelGGL(opt_cg_finish_kernel, dim3(1), dim3(kOptThreads), 0, st, c);
  return hipGetLastError();
}
hipError_t opt_launch_out(const OptCg& c, int mode, const float* Hin, float* o1, float* o2, hipStream_t st) {
  hipLaunchKernelGGL(opt_out_kernel, dim3(c.nblk, c.batch), dim3(kOptThreads), 0, st, c, mode, Hin, o1, o2);
  return hipGetLastError();
}
hipError_t opt_launch_pixels(const float* in, float* out, int npix, int batch, bool transpose, hipStream_t st) {
  const int nb = (npix + kOptThreads - 1) / kOptThreads;
  hipLaunchKernelGGL(opt_pixels_kernel, dim3(nb < kOptBlocks ? nb : kOptBlocks, batch), dim3(kOptThreads), 0, st, in, out, npix,
                     transpose ? 1 : 0);
  return hipGetLastError();
}

}  // namespace qpat
