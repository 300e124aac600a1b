// Internal structures of the optical operators (optical.hip, optical.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace qpat {

constexpr int kOptThreads = 256;  // threads per block of the optical kernels
constexpr int kOptBlocks = 256;   // most blocks per field (a fixed count per mesh: deterministic reductions)

// Device state of up to `batch` optical problems on one mesh (FP64).
struct OptCg {
  int nx, ny, nn, ne, batch;
  int nblk;                    // blocks per field, min(kOptBlocks, ceil(nn / kOptThreads))
  double h;
  double *ka, *mu;             // [batch][ne] coefficients of the last forward solve
  double *ek, *em;             // [batch][ne] staged perturbations (J_o)
  double* phi;                 // [batch][nn] Phi0 of the last forward solve
  double *rhs, *x, *r, *p, *q, *dinv;  // [batch][nn] conjugate-gradient work
  double* z;                   // [batch][nn] preconditioned residual
  double *part_rz, *part_rr, *part_pq;  // [batch][kOptBlocks] block partials
  double *rz, *rr, *rr_next, *bb;       // rz [2][batch]; others [batch]
  double* cur;                 // [batch][4] side currents
};

hipError_t opt_launch_set(const OptCg& c, const float* kappa, const float* mu, hipStream_t st);
hipError_t opt_launch_stage(const OptCg& c, const float* da, const float* dm, hipStream_t st);
hipError_t opt_launch_rhs(const OptCg& c, int mode, const double* cur, const float* Hin, hipStream_t st);
// One level of the multigrid preconditioner of the CG solve, on the node
// grid ([batch][ny][nx] fields; level 0 is the mesh's (ny + 1) x (nx + 1)
// nodes, level l + 1 aggregates 2 x 2 nodes of level l).  The operator is a
// symmetric 7-point stencil: diagonal and the couplings to the east, north
// and north-east neighbours (the mesh diagonals run south-west to north-east,
// and 2 x 2 aggregation keeps that pattern).  Level 0's b is the CG residual
// and its t receives the preconditioned residual.
struct OptLevel {
  int nx, ny;
  double *sc, *se, *sn, *sd, *dinv;  // stencil and inverse diagonal
  double *b, *x, *t;                 // right-hand side, iterate (coarsest level), post-smoothed iterate
};
constexpr int kOptMgMaxLevels = 32;
constexpr double kOptMgOmega = 0.8;  // damping of the Jacobi sweeps

// Stencils of every level for the current coefficients (c.ka, c.mu).
hipError_t opt_launch_mg_setup(const OptCg& c, const OptLevel* lv, int nlev, hipStream_t st);
hipError_t opt_launch_cg_start(const OptCg& c, const OptLevel* lv, int nlev, hipStream_t st);
hipError_t opt_launch_cg_iteration(const OptCg& c, const OptLevel* lv, int nlev, int par, double tol2,
                                   hipStream_t st);
hipError_t opt_launch_cg_finish(const OptCg& c, hipStream_t st);
hipError_t opt_launch_out(const OptCg& c, int mode, const float* Hin, float* o1, float* o2, hipStream_t st);
hipError_t opt_launch_pixels(const float* in, float* out, int npix, int batch, bool transpose, hipStream_t st);

}  // namespace qpat
