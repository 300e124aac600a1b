// Internal structures shared by the HIP kernels (kernels.hip) and the host
// runtime (plan.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace qpat {

constexpr int kBlock = 256;   // threads per block of the helper kernels (default for the passes)
constexpr int kMaxThreads = 512;  // maximum threads per block of a row / column pass
constexpr size_t kMaxLds = 163840;  // gfx950: LDS bytes available to one work-group
constexpr int kMaxPer = 8;    // pointwise elements per thread held in registers
constexpr int kColPer = 4;    // spectrum elements of one field per thread in a column pass
constexpr int kConRegs = 4;   // adjoint scatter: contributions of a node held inline in its record
constexpr int kTapCap = 64;   // sensor taps of one row tile staged in LDS
constexpr int kXcds = 8;      // MI355X: 8 XCDs, work-groups dispatched round-robin

// One bilinear sensor tap pair on one grid row: the sensor's contribution from
// row y is wl * f[y][ixl] + wr * f[y][ixr]; `slot` (0/1) says whether y is the
// sensor's lower or upper row; entries are sorted by row y.
struct alignas(16) Tap {
  int s, slot, y, ixl, ixr;
  float wl, wr;
  int pad;
};

// Per-plan device data (medium diagonals, multipliers, twiddles, taps).
struct Medium {
  int nx, ny, nxh, nt, ns, lossy;
  float dt;
  float ypow;             // power-law exponent y of the absorption
  int rt, ct;             // rows per row-pass tile, spectrum columns per column-pass tile
  int lrt, lct;           // log2(rt), log2(ct)
  int srt, lsrt;          // spectra are stored in srt x ct tiles (srt a multiple of rt); log2(srt)
  int rthr, cthr;         // threads per block of the row / column passes
  uint32_t radx, rady;    // radix plans (max radix 8), 4 bits per stage, first stage lowest
  int nstx, nsty;
  const float *c2, *c2eta, *c2tau, *rho0, *bx, *by;   // [ny][nx]; bx = dt/rho_x, by = dt/rho_y
  const float *avx, *arx, *avy, *ary;                 // PML diagonals: [nx] / [ny]
  const float2 *dxp, *dxm;                            // [nxh+1] i kx e^{+-i kx dx/2}
  const float2 *dyp, *dym;                            // [ny]
  const float *kap, *ldis, *labs;                     // [nxh+1][ny] (column-major), divided by nx*ny
  const float2 *twx, *twy;                            // per-stage FFT twiddles [nx] / [ny]
  const float2* twyr;                                 // the same for the reversed ny plan
  const int* tap_off;                                 // [ny+1] CSR offsets into taps
  const Tap* taps;
  // Adjoint scatter M^T r as a gather per grid node: node_off [ny+1] CSR
  // offsets (in records) into nodes, two int4 per node: (y, x, c0, c1) and the
  // first kConRegs of its contributions scon[c0..c1) (tap index << 1 | right
  // weight, in increasing tap index; zero-padded).
  const int* node_off;
  const int4* nodes;
  const int* scon;
};

// Per-vector work buffers (owned by the plan).
struct Work {
  float *f0, *f1, *f2, *f3;   // forward: v_x v_y rho_x rho_y;  adjoint: their adjoints
  float* q;                   // forward: p snapshot (checkpoints); adjoint: q = c^2 p*
  float2 *s0, *s1;            // half spectra, ny x nx/2 in srt x ct tiles (DC / Nyquist packed in column 0)
  float* part;                // forward: sensor partials [nt][ns][2]; adjoint: residual in tap order [nt][2 ns]
};

// Per-call input / output pointers of one vector.
struct IO {
  const float* in;   // forward: p0 [ny][nx] (read at iterates -1, 0); adjoint: residual [nt][ns]; apply: field
  float* out;        // forward: data [nt][ns] (sensor-data combine); adjoint: gradient [ny][nx] (written at
                     // iterates 0 and -1); apply: field
  float* sens;       // sound-speed sensitivities dp^m/dc, [slots][ny][nx] (RM_X passes only)
  double* gc;        // adjoint: correlation sum_m p*^m dp^m/dc [ny][nx] (RM_X passes only)
};

struct Item {
  Medium m;
  Work w;
};

// Kernel argument block of the row / column passes.  Uniform launches use m,
// w0 and wstride (item i's work buffers are w0 shifted by i * wstride bytes);
// table launches use map and items.  io holds the per-call pointers.
struct Launch {
  Medium m;
  Work w0;
  long long wstride;
  int nitems;
  const int2* map;
  const Item* items;
  const IO* io;
};

// Column-pass multiplier codes: out_o = sum_i M[o][i] * in_i, code per entry.
enum MultCode : int {
  MC_NONE = 0, MC_DXP = 1, MC_DXM = 2, MC_DYP = 3, MC_DYM = 4, MC_LDIS = 5, MC_LABS = 6
};
constexpr int mpack(int m00, int m01, int m10, int m11) {
  return m00 | (m01 << 4) | (m10 << 8) | (m11 << 12);
}

// Column-pass kinds (see kColCode in the kernels).
enum ColMode : int { CM_GRADP1 = 0, CM_GRADM2 = 1, CM_FRAC = 2, CM_GRADP2 = 3, CM_DIVM = 4, CM_APPLY = 5 };
constexpr int kColModes = 6;

// Row-pass kernels.
enum RowMode : int {
  RM_F1 = 0,   // forward: grad p -> v update -> spectra of (v_x, v_y)
  RM_F2 = 1,   // forward: div v -> rho update (+ source) -> spectra of (S, u)   [lossy]
  RM_F2L = 2,  // forward lossless: div v -> rho update -> p, sensors, spectrum of p
  RM_F3 = 3,   // forward lossy: Y S, Y u -> p, sensors, spectrum of p
  RM_A1 = 4,   // adjoint lossy: p* -> + M^T r -> q, spectra of (eta q, tau q)
  RM_A1L = 5,  // adjoint lossless: p* -> + M^T r -> rho* update -> spectra of e*
  RM_A2 = 6,   // adjoint lossy: Y ops -> rho* update -> spectra of e*
  RM_A3 = 7,   // adjoint: grad e* -> v* update -> spectra of g*
  RM_FWD1 = 8, // single real field (row pairs) -> spectrum s0
  RM_INV1 = 9, // spectrum s0 -> single real field (row pairs)
  // Modifier of RM_F2L / RM_F3 / RM_A1 / RM_A1L: the forward passes also store
  // the sensitivity dp/dc of the new pressure into IO::sens at the slot held in
  // the flags; the adjoint passes add p* times that sensitivity into IO::gc.
  RM_X = 16,
  // Modifier of RM_F2 / RM_A2 at iterates n >= 1: the instance holds only the
  // path with the two FFTs' boundary stage fused (compile-time lengths whose
  // plan allows it; see kernels_row_fused).
  RM_FZ = 32
};

// Per-launch flags.
enum Flags : int {
  FL_STORE_P = 1,     // forward: also store p into Work::q
  FL_NO_SENSORS = 2,  // forward: skip the sensor partials (replay)
};
constexpr int kSlotShift = 8;  // RM_X passes: flags >> kSlotShift is the sensitivity slot

// roctx range for the lifetime of the object (plan.cpp).
struct TraceRange {
  explicit TraceRange(const char* name);
  ~TraceRange();
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

// Launch helpers implemented in kernels.hip.
// `len`: for table launches (uniform false), the row (column) length every
// item shares, or 0 when the items' lengths differ.  `tg`: uniform launches
// only, FFT twiddles read from global memory (the LDS size then excludes the
// twiddle tables, see row_lds_bytes / col_lds_bytes); the line length must be
// one of kernels_have_length's.
hipError_t launch_row(int mode, const Launch& L, bool uniform, int len, bool tg, int ntile, int chunk, int nblocks,
                      int threads, size_t lds, int n, int flags, hipStream_t st);
hipError_t launch_col(int cm, int mcode, const Launch& L, bool uniform, int len, bool tg, int ntile, int chunk,
                      int nblocks, int threads, size_t lds, int n, hipStream_t st);
// Row lengths whose RM_FZ instances exist (uniform launches, and table
// launches of that length), for launches reading global twiddles (tg) or not.
bool kernels_row_fused(int n, bool tg);
// Row (col false) or column lengths with compile-time kernel instances.
bool kernels_have_length(int n, bool col);
hipError_t launch_combine(const Item* items, const IO* io, int nitems, int max_count,
                          hipStream_t st);
hipError_t kernels_allow_lds(size_t bytes);
hipError_t launch_tap_order(const Item* items, const IO* io, int nitems, int max_count, hipStream_t st);
hipError_t launch_grad_c(const float* c2, const float* p0, const float* g0, const double* gc, long long n,
                         int batch, long long gc_stride, float* out, hipStream_t st);
hipError_t launch_dot(const float* a, const float* b, int64_t n, double* partial, int nblk,
                      double* out, hipStream_t st);
// Sets *flag (device int) to 1 if any of the n floats at x is NaN or infinite.
hipError_t launch_finite(const float* x, int64_t n, int* flag, hipStream_t st);
// Blocks (and partial sums) of the inner product of length n: at most kDotBlocks.
constexpr int kDotBlocks = 512;
// Device address, on the current device, of the static partial-sum array of
// qpat_dot_noalloc (kDotBlocks doubles), looked up once per device.
hipError_t dot_scratch(double** ptr);
// Largest length qpat_dot_noalloc accepts.
constexpr int64_t kDotNoallocMaxN = int64_t(1) << 40;
inline int dot_blocks(int64_t n) {
  const int64_t b = (n + kBlock - 1) / kBlock;
  return int(b < 1 ? 1 : (b > kDotBlocks ? kDotBlocks : b));
}

// LDS line layout: element e of a line sits at px(e) = e + e/8.  The pad slot
// after every 8 elements spreads the strided writes of the early Stockham
// stages over the banks.  Column lines get one more slot (the transposed
// loads of a multi-column tile would otherwise hit one bank).
__host__ __device__ constexpr int px(int e) { return e + (e >> 3); }
__host__ __device__ constexpr int lstride(int n) { return n + (n >> 3); }
__host__ __device__ constexpr int col_lstride(int ny) { return lstride(ny) + 1; }

// LDS bytes of one block of each pass: ping-pong line buffers (one buffer
// for lines transformed in place, ip), the twiddle tables unless they are read
// from global memory (tg; columns: the plan and its reverse), and (rows) the
// staged sensor taps.
inline size_t row_lds_bytes(int nx, int rt, bool tg = false, bool ip = false) {
  return size_t((ip ? 1 : 2) * rt * lstride(nx) + (tg ? 0 : nx)) * sizeof(float2) +
         kTapCap * (sizeof(Tap) + sizeof(float));
}
inline size_t col_lds_bytes(int ny, int ct, bool tg = false, bool ip = false) {
  return (size_t(ip ? 1 : 2) * 2 * ct * col_lstride(ny) + (tg ? 0 : 2 * size_t(ny))) * sizeof(float2);
}

}  // namespace qpat
