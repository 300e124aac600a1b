// Internal interface of the TV priorconditioner kernels (recon.hip) and their
// host side (recon.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace qpat {

constexpr int kRedThreads = 256;  // threads per block of the TV / CG kernels
constexpr int kRedBlocks = 256;   // blocks per field (fixed: the reductions run in a fixed order)

// Device buffers of the FP64 conjugate-gradient solve of M_gamma z = r for
// `batch` fields of n = nx*ny nodes each ([batch][n] unless noted).
struct TvCg {
  double *x, *r, *z, *p, *q, *dinv;  // iterate, residual, preconditioned residual, direction, M p, 1/diag
  double *wh, *wv;                   // edge weights C (horizontal / vertical edge of each node)
  double *part_rz, *part_rr, *part_pq;  // block partials [batch][kRedBlocks]
  double* rz;                        // r.z [2][batch] (current and next, alternating)
  double *rr, *rr_next, *bb;         // r.r (published / pending), r.r of the right-hand side [batch]
};

// One level of the multigrid preconditioner of the CG solve, [batch][ny][nx]
// fields.  Level 0 is the grid itself (b is the CG residual, t receives the
// preconditioned residual); level l + 1 aggregates 2 x 2 blocks of level l.
struct MgLevel {
  int nx, ny;
  double *wh, *wv, *g, *dinv;  // operator: edge weights, diagonal (gamma) term, inverse diagonal
  double *b, *x, *t;           // right-hand side, iterate (coarsest level), post-smoothed iterate
};
constexpr int kMgMaxLevels = 32;
constexpr double kMgOmega = 0.8;  // damping of the Jacobi sweeps

hipError_t launch_tv_weights(const float* x, int nx, int ny, int batch, double beta, double* wh, double* wv,
                             hipStream_t st);
hipError_t launch_tv_apply(const float* x, float* y, const double* wh, const double* wv, int nx, int ny, int batch,
                           double gamma, hipStream_t st);
hipError_t launch_tv_value(const float* x, int nx, int ny, int batch, double beta, double* part, hipStream_t st);
// Operators of every level for this gamma (level 0's edge weights are the TV
// weights; its inverse diagonal goes to c.dinv).
hipError_t launch_mg_setup(const MgLevel* lv, int nlev, int batch, double gamma, hipStream_t st);
hipError_t launch_cg_start(const float* rhs, const TvCg& c, const MgLevel* lv, int nlev, int nx, int ny, int batch,
                           hipStream_t st);
hipError_t launch_cg_iteration(const TvCg& c, const MgLevel* lv, int nlev, int nx, int ny, int batch, double gamma,
                               int par, double tol2, hipStream_t st);
hipError_t launch_cg_finish(const TvCg& c, float* out, int nx, int ny, int batch, hipStream_t st);
hipError_t launch_axpby(int64_t n, float a, const float* x, float b, float* y, hipStream_t st);

// PCG of Algorithm 4 with device scalars, `batch` fields of n values:
// out[f * ostride] = scale * a_f . b_f (FP64; part holds [batch][kRedBlocks]);
// live / done flags of iteration i; the alpha step; the beta direction update;
// x += sol for the flagged fields.
hipError_t launch_ld_dots(const float* a, const float* b, size_t n, int batch, double* part, double* out,
                          int ostride, double scale, hipStream_t st);
hipError_t launch_ld_live(int batch, const double* rz, int rzs, int i, int i_max, int i_m, double tol_in, int* done,
                          int* live, hipStream_t st);
hipError_t launch_ld_step(size_t n, int batch, const double* rz, int rzs, int i, const double* dhd, const int* live,
                          const float* d, const float* hd, float* sol, float* r, hipStream_t st);
hipError_t launch_ld_dir(size_t n, int batch, const double* rz, int rzs, int i, const int* live, const float* z,
                         float* d, hipStream_t st);
hipError_t launch_ld_add(size_t n, int batch, const int* flag, const float* sol, float* x, hipStream_t st);
// hsol += alpha_i jd per live data set, alpha_i = rz_i / dhd (the step of launch_ld_step on data vectors)
hipError_t launch_ld_data_step(size_t nd, int batch, const double* rz, int rzs, int i, const double* dhd,
                               const int* live, const float* jd, float* hsol, hipStream_t st);

}  // namespace qpat
