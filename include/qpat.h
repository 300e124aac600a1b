/*
 * qpat.h - C ABI of the MI355X k-space acoustic operator library (libqpat.so).
 *
 * The library computes the discrete acoustic forward operator H_a of
 * Javaherian & Holman, "Direct quantitative photoacoustic tomography for
 * realistic acoustic media" (arXiv 1810.11685), Section 3.2.3 and Definition 4
 * (k-space PSTD solve of eqs num-vel, num-rho, num-p, num-m with the two-step
 * additive source of eq s1), and its discretise-then-adjoint H_a^* (Section
 * 3.2.4, Lemma 2), on a 2-D grid, in FP32, with hand-written HIP kernels for
 * gfx950.
 *
 * Conventions shared by every entry point
 *  - Fields are row-major [ny][nx] float arrays, x fastest.  Node (j, i) sits at
 *    x = (i - nx/2) dx, y = (j - ny/2) dy (centre node at the origin).
 *  - Sensor data are time-major [nt][ns] (Definition 4): row m holds
 *    P_m = M p_m, m = 0 .. nt-1.
 *  - A batch of B vectors of the same plan is laid out contiguously:
 *    fields [B][ny][nx], data [B][nt][ns].
 *  - Device pointers are HIP device memory owned by the caller; the library
 *    never frees them.  Host pointers are read during the call only.
 *  - `stream` is a hipStream_t (NULL = default stream).  Calls enqueue work on
 *    it and return without waiting for the device; no hidden device-wide
 *    synchronisation.  A plan is not re-entrant: calls that use one plan from
 *    several streams at once race on its work buffers.
 *  - Every call returns a qpat_status.  Argument checks happen on the host
 *    before any device work; a failing check enqueues nothing.  The message of
 *    the last failure of the calling thread is in qpat_last_error().
 *  - Readings of points the paper leaves open (PML profile, staggered density,
 *    sensor interpolation, Nyquist bin, sinc convention, alpha0 units) are
 *    listed with the parameters below.
 */
#ifndef QPAT_H
#define QPAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QPAT_OK = 0,
  QPAT_E_INVALID = 1,     /* bad argument (null pointer, bad size, non-positive medium, ...) */
  QPAT_E_UNSUPPORTED = 2, /* grid size not 2^a or 3*2^a in [8, 1024], y odd with loss, mixed batch */
  QPAT_E_UNSTABLE = 3,    /* dt above the k-space stability bound for c_ref < max(c0) */
  QPAT_E_HIP = 4,         /* a HIP runtime call failed (message has the HIP error) */
  QPAT_E_OOM = 5,         /* device or pinned host allocation failed */
  QPAT_E_NONFINITE = 6    /* qpat_check: a checked output held NaN or Inf */
} qpat_status;

typedef struct qpat_plan_s* qpat_plan;
typedef struct qpat_batch_s* qpat_batch;
typedef void* qpat_stream; /* hipStream_t */

/*
 * Problem parameters (host struct, copied by qpat_plan_create).
 *  nx, ny      grid nodes (each 2^a or 3*2^a, 8 <= n <= 1024); the PML lies
 *              inside this grid.
 *  dx, dy, dt  grid spacing [m] and time step [s].
 *  nt          number of time samples (the loop runs n = -1 .. nt-2).
 *  c_ref       reference speed of the k-space correction sinc(c_ref k dt/2),
 *              eq grr [m/s].  The stability bound is checked against max(c0).
 *  pml_size    PML thickness in cells on every side (0 = none); profile
 *              sigma = pml_alpha (c_ref/dx) (xi/pml_size)^4 [1/s], A = exp(-sigma dt/2)
 *              (eq dis-pml); velocities use it at half-node positions.
 *  pml_alpha   PML maximum attenuation in nepers per cell.
 *  alpha0_db   power-law absorption prefactor in dB MHz^-y cm^-1 (0 = lossless);
 *              tau and eta follow eq Twelve after conversion to Np (rad/s)^-y m^-1.
 *  y           power-law exponent (y != 1 when alpha0_db > 0).
 *  ns          number of point sensors.
 *  sensor_xy   host [ns][2] (x, y) positions in metres; each must lie inside the
 *              node grid; M interpolates bilinearly from the 4 nearest nodes.
 */
typedef struct {
  int32_t nx, ny;
  double dx, dy, dt;
  int32_t nt;
  double c_ref;
  int32_t pml_size;
  double pml_alpha;
  double alpha0_db;
  double y;
  int32_t ns;
  const double* sensor_xy;
} qpat_params;

/* Spectral operators for qpat_apply (Section 3.2.2): k-space staggered
 * gradients of eq grr and the fractional Laplacians Y_dis, Y_abs. */
typedef enum {
  QPAT_OP_DX_PLUS = 0,  /* d/dx^+ : F^-1 { i kx e^{+i kx dx/2} sinc(c_ref k dt/2) F } */
  QPAT_OP_DX_MINUS = 1, /* d/dx^- */
  QPAT_OP_DY_PLUS = 2,  /* d/dy^+ */
  QPAT_OP_DY_MINUS = 3, /* d/dy^- */
  QPAT_OP_YDIS = 4,     /* F^-1 { |k|^(y-1) F }, 0 at k = 0 */
  QPAT_OP_YABS = 5      /* F^-1 { |k|^(y-2) F }, 0 at k = 0 */
} qpat_op;

/* Host-only check of a parameter set (no device work, no allocation).
 * Returns QPAT_E_INVALID / QPAT_E_UNSUPPORTED for bad sizes or values. */
qpat_status qpat_validate(const qpat_params* prm);

/* Build a plan: validates `prm` and the medium, derives every medium diagonal,
 * multiplier, PML profile and sensor tap in FP64 on the host, rounds them to
 * FP32 and uploads them (synchronously) to the current HIP device.
 *  c0, rho0  host [ny][nx] sound speed [m/s] and ambient density [kg/m^3],
 *            all > 0 and finite.
 * Returns QPAT_E_UNSTABLE when dt exceeds 2 asin(c_ref/max c0)/(c_ref k_max)
 * with c_ref < max c0.  On failure *out is NULL. */
qpat_status qpat_plan_create(const qpat_params* prm, const double* c0, const double* rho0,
                             qpat_plan* out);
void qpat_plan_destroy(qpat_plan plan);

/* Forward operator H_a (Definition 4): p0 [B][ny][nx] -> data [B][nt][ns].
 * `batch` vectors run in one set of launches. */
qpat_status qpat_forward(qpat_plan plan, const float* p0, float* data, int32_t batch,
                         qpat_stream stream);

/* Adjoint H_a^* (Lemma 2): residual [B][nt][ns] -> gradient in p0 [B][ny][nx]. */
qpat_status qpat_adjoint(qpat_plan plan, const float* res, float* grad, int32_t batch,
                         qpat_stream stream);

/* Jacobian-vector product.  H_a is linear in p0 (eq acoust_map), so J v = H_a v. */
qpat_status qpat_jv(qpat_plan plan, const float* v, float* data, int32_t batch,
                    qpat_stream stream);

/* Gauss-Newton normal operator J^T J v = H_a^* H_a v (Section 4, eq apj):
 * v [B][ny][nx] -> out [B][ny][nx]; the intermediate data stay in plan memory. */
qpat_status qpat_jtjv(qpat_plan plan, const float* v, float* out, int32_t batch,
                      qpat_stream stream);

/* qpat_jtjv that also hands back the intermediate J v = H_a v: v [B][ny][nx]
 * -> jv [B][nt][ns] and out [B][ny][nx] (device, caller-owned, not
 * overlapping).  The same launches as qpat_jv followed by qpat_adjoint on its
 * output, so jv is bitwise qpat_jv's and out bitwise qpat_jtjv's.  A
 * Gauss-Newton solver that keeps J d for each search direction d can form
 * J (x + sum a_i d_i) - y from the residual at x without another forward
 * solve (J is linear in p0). */
qpat_status qpat_jtjv_data(qpat_plan plan, const float* v, float* jv, float* out, int32_t batch,
                           qpat_stream stream);

/* One spectral operator on B fields: in [B][ny][nx] -> out [B][ny][nx]. */
qpat_status qpat_apply(qpat_plan plan, int32_t op, const float* in, float* out, int32_t batch,
                       qpat_stream stream);

/* Wavefield checkpointing.  The stacked state z_m = (v_x, v_y at t_{m-1/2},
 * rho_x, rho_y, p at t_m) of the paper's eq t is stored at m = 0, K, 2K, ...
 * A checkpoint buffer holds [B][ceil(nt/K)][5][ny][nx] floats.
 *  qpat_ckpt_bytes     size in bytes of that buffer.
 *  qpat_forward_ckpt   qpat_forward that also fills `ckpt` (device, caller-owned).
 *  qpat_replay         recomputes the states of segment `seg` from its checkpoint:
 *                      states [B][cnt][5][ny][nx] for m = seg*K .. seg*K+cnt-1,
 *                      cnt = min(K, nt - seg*K); bitwise equal to the states of
 *                      the uninterrupted forward run.  p0 is needed again because
 *                      the source of eq s1 is also injected at iterate n = 0.
 * Memory is O(nt/K) for the checkpoints plus O(K) for one replayed segment. */
qpat_status qpat_ckpt_bytes(qpat_plan plan, int32_t interval, int32_t batch, size_t* bytes);
qpat_status qpat_forward_ckpt(qpat_plan plan, const float* p0, float* data, int32_t interval,
                              float* ckpt, int32_t batch, qpat_stream stream);
qpat_status qpat_replay(qpat_plan plan, const float* p0, const float* ckpt, int32_t interval,
                        int32_t seg, float* states, int32_t batch, qpat_stream stream);

/* Sound-speed gradient (towards the joint sound-speed reconstruction that the
 * paper's Discussion names as future work): for residuals r [B][nt][ns] and initial pressures p0 [B][ny][nx],
 *   grad_c = d <r, H_a[c0] p0> / d c0   [B][ny][nx],
 *   grad_p0 = H_a^* r                   [B][ny][nx] (as qpat_adjoint),
 * with c_ref (hence kappa and the PML, eqs kappa and pml) held fixed.  c0
 * enters the discrete operator through the equation of state (eq num-p: c^2,
 * and c^2 eta ~ c^(y+2), c^2 tau ~ c^(y+1) by eq Twelve) and through the
 * source scaling p0 / (4 c^2) of eq s1, so
 *   grad_c = sum_m p*^m dp^m/dc - (2/c) p0 grad_p0,
 * p*^m being the adjoint of p^m.  The forward wavefield is checkpointed every
 * `interval` = K iterates; the reverse sweep recomputes one segment of K
 * pressures at a time from its checkpoint, storing only dp^m/dc, and
 * correlates it with the adjoint of that segment (FP64 sum).  K >= nt - 1
 * keeps every sensitivity (one forward and one adjoint sweep); a smaller K
 * costs one more forward sweep.  Per vector the workspace holds one FP64
 * field, min(K, nt - 1) + 1 sensitivity fields and floor((nt - 2) / K)
 * checkpoints of 5 fields (memory O(nt/K + K)).
 *  qpat_medium_grad_bytes  size of the device workspace `work` (caller-owned,
 *                          256-byte aligned, contents need not be initialised).
 * Uses plan work space for 2B vectors.  Calls on one plan must not overlap. */
qpat_status qpat_medium_grad_bytes(qpat_plan plan, int32_t interval, int32_t batch, size_t* bytes);
qpat_status qpat_medium_grad(qpat_plan plan, const float* p0, const float* res, int32_t interval, void* work,
                             float* grad_p0, float* grad_c, int32_t batch, qpat_stream stream);

/* Launch shape of the FFT passes: rows per row-pass block, spectrum columns
 * per column-pass block (powers of two dividing ny and nx/2; rows even, and at
 * most ny/8 when ny is a power of two of 128 or more) and
 * threads per block of each pass (64, 128, 256 or 512; rows*nx at most 8 and
 * cols*ny at most 4 times the threads; a block's LDS within the 160 KB of a gfx950
 * work-group).  qpat_tune times the candidates on `stream` for
 * `batch` vectors and keeps the fastest: each candidate runs 16 forward
 * iterates and the 16 adjoint iterates that undo them (every pass kind of a
 * forward + adjoint pair), launched the way the plan's calls launch them
 * (captured and replayed as a hipGraph when graph mode is on; the stream is
 * synchronised); the three fastest are then timed again, each over the same
 * number of iterates each way: 48, or more where 16 took under ~7 ms, so that
 * each timing covers ~20 ms of work (at most 4096, and at most nt - 2).  Results are cached per (nx, ny, batch, lossy, graph mode)
 * in the file named by QPAT_TUNE_CACHE, if set, one line
 * "nx ny batch lossy graph rows cols row_threads col_threads" per shape; a
 * plan whose key is in the file takes that shape without timing.  row_threads / col_threads may be NULL in
 * qpat_get_tiles. */
qpat_status qpat_set_tiles(qpat_plan plan, int32_t rows, int32_t cols, int32_t row_threads,
                           int32_t col_threads);
qpat_status qpat_get_tiles(qpat_plan plan, int32_t* rows, int32_t* cols, int32_t* row_threads,
                           int32_t* col_threads);
qpat_status qpat_tune(qpat_plan plan, int32_t batch, qpat_stream stream);

/* Diagnostic timing of one pass kind on the plan's work buffers: the
 * kernel of one phase of an iterate, launched `reps` times back-to-back on
 * `stream` between two HIP events (after one warm-up launch), at iterate n = 1.
 * Returns the mean duration per launch in milliseconds and synchronises the
 * stream; the plan's work buffers are overwritten.  Pass ids:
 *   forward  0 column d/dx^+, d/dy^+ of p      1 row: velocity update (eq num-vel)
 *            2 column d/dx^-, d/dy^- of v      3 row: density update (eq num-rho)
 *            4 column Y_dis, Y_abs             5 row: pressure (eq num-p), sensors
 *   adjoint  6 row: M^T r, c^2 p*              7 column Y_dis, Y_abs
 *            8 row: transposed density update  9 column d/dx^+, d/dy^+
 *           10 row: transposed velocity update 11 column sum of d/dr_i^-
 * Passes 4, 5, 7, 8 exist only for lossy plans (QPAT_E_INVALID otherwise). */
qpat_status qpat_time_pass(qpat_plan plan, int32_t pass, int32_t batch, int32_t reps,
                           qpat_stream stream, float* ms_per_launch);

/* Diagnostic probe of the persistent-launch alternative: the mean time of
 * one exchange step of `nblocks` blocks of `threads` threads, each block
 * writing `words` floats to its slot of a device buffer and then reading the
 * slot of the next block (as float4 vectors, all of a thread's loads in
 * flight together), with the blocks synchronised in between by
 *   design 0  a device-wide barrier in a cooperative launch (one arrival counter),
 *   design 1  a hierarchical barrier in a cooperative launch (an arrival
 *             counter per XCD group, then a global counter and a generation
 *             word polled by one lane per block with back-off),
 *   design 2  kernel boundaries: one launch per step, replayed from a hipGraph.
 * Steps are timed with HIP events on `stream` (which is synchronised) as the
 * difference of runs of `iters` and iters/10 steps, so launch costs cancel.
 * Every wait is bounded: *timed_out is set when a block gave up waiting (the
 * kernel then ends early and *us_per_step is meaningless).  Cooperative
 * designs need every block resident (QPAT_E_UNSUPPORTED otherwise).  Limits:
 * threads 64..1024 (multiple of 64), nblocks 1..4096, iters 2..100000, words
 * 0..2^20 and a multiple of 4.  The probe allocates and frees its own buffers. */
qpat_status qpat_probe_barrier(int32_t design, int32_t nblocks, int32_t threads, int32_t iters, int32_t words,
                               qpat_stream stream, float* us_per_step, int32_t* timed_out);

/* hipGraph mode: when enabled, the kernel sequence of a forward / adjoint /
 * jtjv call is captured into a hipGraph on first use and replayed on later
 * calls with the same operation, batch and buffer addresses. */
qpat_status qpat_set_graph(qpat_plan plan, int32_t enable);

/* Uneven-grid batch: plans of different sizes (and numbers of time steps)
 * advanced together, one launch per phase for all of them.  All plans must be
 * lossy or all lossless (else QPAT_E_UNSUPPORTED).  The batch keeps references
 * to the plans, which must outlive it.  Pointer arrays are host arrays of `count` device
 * pointers laid out as for the single-plan calls with B = 1. */
qpat_status qpat_batch_create(const qpat_plan* plans, int32_t count, qpat_batch* out);
void qpat_batch_destroy(qpat_batch batch);
qpat_status qpat_batch_forward(qpat_batch batch, const float* const* p0, float* const* data,
                               qpat_stream stream);
qpat_status qpat_batch_adjoint(qpat_batch batch, const float* const* res, float* const* grad,
                               qpat_stream stream);
qpat_status qpat_batch_jtjv(qpat_batch batch, const float* const* v, float* const* out,
                            qpat_stream stream);
qpat_status qpat_batch_set_graph(qpat_batch batch, int32_t enable);
/* Schedule of a batch.  0: one launch per pass covers every problem (a
 * launch runs with the largest LDS and thread count of its problems).  1: one
 * launch sequence per grid size (nx, ny), each with the launch shape of its
 * plans, the sequences running side by side on streams of the batch forked
 * from and joined back into the caller's stream (inside the captured graph
 * in graph mode).  Setting a schedule rebuilds the batch's launch state from
 * the plans' current launch shapes (synchronising the device).  Results do
 * not depend on the schedule. */
qpat_status qpat_batch_set_schedule(qpat_batch batch, int32_t schedule);
qpat_status qpat_batch_get_schedule(qpat_batch batch, int32_t* schedule);
/* Autotune a batch: for every grid size, qpat_tune on its first plan for the
 * number of problems of that size (in the batch's graph mode), that shape
 * given to every plan of the size (the plans' launch shapes change); then
 * both schedules timed on full forward + adjoint sweeps of the batch and the
 * faster kept.  Synchronises `stream`; overwrites the batch's work buffers. */
qpat_status qpat_batch_tune(qpat_batch batch, qpat_stream stream);

/* Inner product with FP64 accumulation of two device float vectors of length
 * n; the result is written to *out (device double).  Deterministic: a fixed
 * block partition reduced in a fixed order (wavefront shuffles, then LDS).
 * The partial sums live in a library buffer per (device, stream), allocated
 * on the first call on that pair: calls on different streams do not share
 * one, calls on one stream are ordered by it. */
qpat_status qpat_dot(const float* a, const float* b, int64_t n, double* out, qpat_stream stream);

/* qpat_dot for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and result bits, with the partial sums in a static device
 * array of 512 doubles (4 KB) that the library holds on every device it runs
 * on until the process ends.  The call allocates nothing; the first call on
 * a device looks up the array's address there.  Lengths 0 .. 2^40 (the
 * array holds one partial per block, at most 512 blocks, whatever n);
 * QPAT_E_INVALID beyond.  Every call on one device shares that device's
 * array: calls that overlap on one device (on different streams, or from
 * different threads) race and must be ordered by the caller. */
qpat_status qpat_dot_noalloc(const float* a, const float* b, int64_t n, double* out, qpat_stream stream);

/* ---- Lagged-diffusivity TV priorconditioner of the inexact-Newton driver
 * (Section 5.2: the TV functional of eq tvm with D of eq dd, its gradient
 * M[x] x of eqs jm, m, m1, and M_gamma = M + gamma I of eq pre), for fields on
 * an nx x ny grid (row-major [ny][nx], device floats, caller-owned).  D takes
 * the differences across the internal edges between horizontally and
 * vertically adjacent nodes, every edge of length 1 (the grid's edges all have
 * one length, which only rescales beta and gamma); C[x] = diag((|D x|^2 +
 * beta)^(-1/2)).  A qpat_tv holds the edge weights C and the FP64 work space
 * of its solver for up to `batch` fields; calls are asynchronous on `stream`
 * unless they say otherwise, and one qpat_tv must not be used from two streams
 * at once. */
typedef struct qpat_tv_s* qpat_tv;
/* nx, ny >= 2 with nx*ny <= 2^24; batch in [1, 64]. */
qpat_status qpat_tv_create(int32_t nx, int32_t ny, int32_t batch, qpat_tv* out);
void qpat_tv_destroy(qpat_tv tv);
/* C from fields x [batch][ny][nx] (beta > 0): the lagged weights of eq m1. */
qpat_status qpat_tv_set_weights(qpat_tv tv, const float* x, double beta, int32_t batch, qpat_stream stream);
/* y = M_gamma x for [batch][ny][nx] fields with the current weights (gamma >= 0). */
qpat_status qpat_tv_apply(qpat_tv tv, double gamma, const float* x, float* y, int32_t batch,
                          qpat_stream stream);
/* z = M_gamma^-1 r (gamma > 0), the preconditioner solve of Algorithm 4, per
 * field: conjugate gradients in FP64, each iteration preconditioned by one
 * multigrid V-cycle (2 x 2 aggregation down to a single node, Galerkin coarse
 * operators, one damped Jacobi sweep before and after each coarse
 * correction), until ||r - M_gamma z|| <= tol ||r|| (0 < tol < 1) or max_iter
 * iterations; *iters (may be NULL) receives the iterations run.  Synchronises
 * the stream (the convergence test reads residual norms every 8 iterations). */
qpat_status qpat_tv_solve(qpat_tv tv, double gamma, const float* r, float* z, int32_t batch, double tol,
                          int32_t max_iter, int32_t* iters, qpat_stream stream);
/* Smoothed TV value sum_l sqrt((D x)_l^2 + beta) per field into out[batch]
 * (host doubles).  Synchronises the stream. */
qpat_status qpat_tv_value(qpat_tv tv, const float* x, double beta, int32_t batch, double* out,
                          qpat_stream stream);
/* y = a x + b y over n device floats (the vector updates of Algorithm 4). */
qpat_status qpat_axpby(int64_t n, float a, const float* x, float b, float* y, qpat_stream stream);

/* ---- Inexact-Newton reconstruction of p0 from acoustic data (Section 5.2.1:
 * Algorithm 5, the lagged-diffusivity outer loop with step length 1, around
 * Algorithm 4, PCG on the Gauss-Newton system J^T J d = -grad of eq apj with
 * the TV priorconditioner M_gamma[X^k] of eq pre), for `batch` data sets of
 * one plan solved side by side.  The unknown is p0 itself (J = H_a), the
 * misfit eps = 0.5 |H_a X - data|^2, its gradient H_a^*(H_a X - data)
 * (eq gr).  Every J^T J d is one batched qpat_jtjv_data call; the PCG scalars
 * (r.z, d.J^T J d, alpha, beta) and the stopping ratio stay on the device as
 * FP64 values; the host reads one flag per data set per PCG iteration (which
 * data sets go on) and the misfits once per outer step.  Because H_a is
 * linear, the residual at X^{k+1} = X^k + sum_i alpha_i d_i is formed as
 * r^k + sum_i alpha_i (H_a d_i) from the data of the PCG's own products, so
 * an outer step costs its PCG products plus one adjoint solve (the gradient
 * for the next step) and no forward solve; the first step skips the forward
 * solve too when every initial image is zero (H_a 0 = 0).
 *  beta, gamma   TV smoothing and preconditioner shift (> 0).
 *  i_max, i_m, tol_in   PCG runs while i < i_max and (i < i_m or
 *                1 - r_i.z_i / r_{i-i_m}.z_{i-i_m} > tol_in), as printed in Algorithm 4.
 *  outer_max, tol_out   outer steps while k = 0 or 1 - eps^k / eps^{k-1} > tol_out,
 *                at most outer_max (Algorithm 5; per data set).
 *  solve_tol, solve_max_iter   the M_gamma solves (as qpat_tv_solve). */
typedef struct {
  double beta, gamma;
  int32_t i_max, i_m;
  double tol_in;
  int32_t outer_max;
  double tol_out;
  double solve_tol;
  int32_t solve_max_iter;
} qpat_ld_params;
typedef struct qpat_ld_s* qpat_ld;
/* Work space (TV weights and solver, PCG vectors, FP64 scalars) for `batch`
 * data sets of `plan` (batch in [1, 64]); the plan must outlive it. */
qpat_status qpat_ld_create(qpat_plan plan, int32_t batch, qpat_ld* out);
void qpat_ld_destroy(qpat_ld ld);
/* data [batch][nt][ns] (device); x [batch][ny][nx] (device): the initial
 * images on entry, the reconstructions on return.  eps_hist: host
 * [batch][outer_max + 1] misfits eps^0 .. (entries past the last step repeat
 * the last value); pcg_iters: host [batch][outer_max] PCG iterations of each
 * outer step (-1 where a data set had already stopped); *outer_steps (may be
 * NULL): outer steps run; *solve_iters (may be NULL): M_gamma solver
 * iterations in all.  The gradient at the last iterate is not formed (no
 * step uses it).  Synchronises `stream`. */
qpat_status qpat_ld_run(qpat_ld ld, const float* data, float* x, const qpat_ld_params* p, double* eps_hist,
                        int32_t* pcg_iters, int32_t* outer_steps, int32_t* solve_iters, qpat_stream stream);

/* ---- 3-D solver (Section 3.2.3 with d = 3: velocity and density with three
 * components each, so the stacked state z_n of Section 3.2.4 holds 7N values,
 * and the source of eq s1 puts p0 / (6 c0^2) into each density component at
 * n = -1 and 0).  Conventions follow the 2-D solver axis by axis: fields are
 * [nz][ny][nx] (x fastest), node (k, j, i) at ((i - nx/2) dx, (j - ny/2) dy,
 * (k - nz/2) dz); the PML lies inside the grid on all six faces; the
 * measurement M interpolates trilinearly from the 8 surrounding nodes.
 *  nx, ny, nz  axis lengths in [4, 128]; every prime factor of 11 or more is
 *              transformed by a direct DFT stage (e.g. 33, 37, 49, 53 are
 *              supported); ny * nz <= 4096.
 *  dz          spacing along z [m]; sensor_xyz host [ns][3] positions [m].
 *  Other fields as in qpat_params.
 * Work is in FP32 with the medium tables built in FP64 and rounded once.
 * The 3-D plan has its own entry points; `batch` vectors run in one set of
 * launches, in [1, 4096]. */
typedef struct {
  int32_t nx, ny, nz;
  double dx, dy, dz, dt;
  int32_t nt;
  double c_ref;
  int32_t pml_size;
  double pml_alpha;
  double alpha0_db;
  double y;
  int32_t ns;
  const double* sensor_xyz;
} qpat_params3d;
typedef struct qpat_plan3d_s* qpat_plan3d;

/* Host-only parameter check (sizes, values, sensors inside the grid). */
qpat_status qpat3d_validate(const qpat_params3d* prm);
/* c0, rho0: host [nz][ny][nx], finite and > 0.  QPAT_E_UNSTABLE when dt
 * exceeds 2 asin(c_ref / max c0) / (c_ref |k|_max) with c_ref < max c0. */
qpat_status qpat3d_plan_create(const qpat_params3d* prm, const double* c0, const double* rho0,
                               qpat_plan3d* out);
void qpat3d_plan_destroy(qpat_plan3d plan);
/* H_a: p0 [B][nz][ny][nx] -> data [B][nt][ns]. */
qpat_status qpat3d_forward(qpat_plan3d plan, const float* p0, float* data, int32_t batch, qpat_stream stream);
/* H_a^*: residual [B][nt][ns] -> gradient [B][nz][ny][nx] (reverse mode of the forward). */
qpat_status qpat3d_adjoint(qpat_plan3d plan, const float* res, float* grad, int32_t batch,
                           qpat_stream stream);
/* J^T J v = H_a^* H_a v: v [B][nz][ny][nx] -> out [B][nz][ny][nx]. */
qpat_status qpat3d_jtjv(qpat_plan3d plan, const float* v, float* out, int32_t batch, qpat_stream stream);
/* One spectral operator on B fields: op 0..7 = d/dx^+, d/dx^-, d/dy^+, d/dy^-,
 * d/dz^+, d/dz^-, Y_dis, Y_abs (symbols as in qpat_op, with the 3-D |k|). */
qpat_status qpat3d_apply(qpat_plan3d plan, int32_t op, const float* in, float* out, int32_t batch,
                         qpat_stream stream);
/* Launch shape: x-lines per row block (even, >= 2, at most 64), spectrum
 * columns per plane block (>= 1), threads per row block (64..512) and per
 * plane block (64..1024, powers of two); both blocks must fit the 160 KB of
 * LDS.  Results do not depend on the shape.  A new plan picks the rows and
 * both thread counts per batch size (fewer lines and more plane threads for
 * batches that leave CUs idle); qpat3d_set_tiles fixes all four, and
 * qpat3d_get_tiles reports the fixed shape, or the automatic one for a single
 * vector.  row_threads / plane_threads may be NULL in qpat3d_get_tiles. */
qpat_status qpat3d_set_tiles(qpat_plan3d plan, int32_t rows, int32_t cols, int32_t row_threads,
                             int32_t plane_threads);
qpat_status qpat3d_get_tiles(qpat_plan3d plan, int32_t* rows, int32_t* cols, int32_t* row_threads,
                             int32_t* plane_threads);
/* hipGraph capture and replay of whole 3-D solves (as qpat_set_graph). */
qpat_status qpat3d_set_graph(qpat_plan3d plan, int32_t enable);

/* ---- Optical operators (Section 3.1, 2-D): the diffusion approximation with
 * its Robin condition (eq DA) discretised by P1 Galerkin FEM (eqs var_fo,
 * system_forward2), the heating map H = mu o I Phi (eq forward_out), its
 * Frechet derivative J_o (eq dh_des) and adjoint J_o^* (eqs system_adjoint,
 * system_adjoint1, prodtproj).  The mesh is matched to an nx x ny acoustic
 * grid of spacing dx: every grid node is the centre of a square pixel, the
 * FEM nodes are the (nx + 1) x (ny + 1) pixel corners, and pixel (j, i) holds
 * element 2 (j nx + i) (corners (j,i), (j,i+1), (j+1,i+1)) and element
 * 2 (j nx + i) + 1 (corners (j,i), (j+1,i+1), (j+1,i)).  Coefficients and
 * heating are elemental, [batch][2 nx ny] device floats; the work is FP64.
 * Systems are solved by conjugate gradients, each iteration preconditioned
 * by one multigrid V-cycle on the node grid (2 x 2 aggregation down to one
 * node, Galerkin coarse stencils, one damped Jacobi sweep before and after
 * each coarse correction), to ||rhs - A x|| <= tol ||rhs||, checked every 8
 * iterations (the calls synchronise the stream); *iters (may be NULL)
 * receives the iterations run.  An optical handle holds the coefficients and
 * Phi of its last forward call for J_o and J_o^*; one handle must not be used
 * from two streams at once.
 *  create      nx, ny >= 1, (nx + 1)(ny + 1) <= 2^26, dx > 0, batch in [1, 64].
 *  forward     kappa, mu > 0 elemental; currents host [batch][4] doubles, the
 *              inward current I_s on the bottom (j = 0), top, left (i = 0) and
 *              right sides; gamma_2 = 1/pi.  H = mu o I Phi.
 *  jv          dH = J_o [dkappa, dmu] at the last forward state.
 *  jtv         (gkappa, gmu) = J_o^* H.
 *  pixels      transpose = 0: p [batch][ny][nx] = mean of each pixel's two
 *              elements of H (initial pressure on the acoustic grid,
 *              Gruneisen 1); transpose = 1: H = half of p to each element. */
typedef struct qpat_optical_s* qpat_optical;
qpat_status qpat_optical_create(int32_t nx, int32_t ny, double dx, int32_t batch, qpat_optical* out);
void qpat_optical_destroy(qpat_optical optical);
qpat_status qpat_optical_forward(qpat_optical optical, const float* kappa, const float* mu, const double* currents,
                                 float* H, int32_t batch, double tol, int32_t max_iter, int32_t* iters,
                                 qpat_stream stream);
qpat_status qpat_optical_jv(qpat_optical optical, const float* dkappa, const float* dmu, float* dH, int32_t batch,
                            double tol, int32_t max_iter, int32_t* iters, qpat_stream stream);
qpat_status qpat_optical_jtv(qpat_optical optical, const float* H, float* gkappa, float* gmu, int32_t batch,
                             double tol, int32_t max_iter, int32_t* iters, qpat_stream stream);
qpat_status qpat_optical_pixels(qpat_optical optical, const float* in, float* out, int32_t transpose,
                                int32_t batch, qpat_stream stream);

/* Failure detection (opt-in).  With the check enabled, every qpat_forward /
 * qpat_jv call also scans its sensor data, and every qpat_adjoint / qpat_jtjv
 * call its gradient, for NaN or Inf values with one small kernel on the same
 * stream after the solve (a plan-owned device flag, no host synchronisation).
 * qpat_check synchronises `stream`, reads the flag and clears it: it returns
 * QPAT_E_NONFINITE if any checked output since the last qpat_check held a
 * non-finite value (an unstable medium or time step, or non-finite inputs),
 * QPAT_OK otherwise.  Enabling allocates the 4-byte flag once. */
qpat_status qpat_set_check(qpat_plan plan, int32_t enable);
qpat_status qpat_check(qpat_plan plan, qpat_stream stream);

/* Plan introspection: sizes and the device bytes the plan holds. */
qpat_status qpat_plan_info(qpat_plan plan, int32_t* nx, int32_t* ny, int32_t* nt, int32_t* ns,
                           size_t* device_bytes);

const char* qpat_status_string(qpat_status status);
const char* qpat_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* QPAT_H */
