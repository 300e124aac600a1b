// Internal structures of the 3-D solver shared by its kernels (k3d.hip) and
// its host runtime (plan3d.cpp).  Not part of the public ABI.
//
// Layout: fields are [nz][ny][nx] (x fastest); "lines" are the nz*ny x-lines,
// line l = z*ny + y.  A field's half spectrum along x has nxh1 = nx/2 + 1
// columns and is stored in column tiles of ct columns: element (c, l) sits at
// (c / ct) * (nlines * ct) + l * ct + c % ct, so a y-z plane pass reads one
// contiguous chunk per tile and a row pass writes runs of ct elements.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace qpat3 {

constexpr int kBlock = 256;          // threads per block of the helper kernels
constexpr int kRowMax = 512;         // most threads of a row block
constexpr int kPlaneMax = 1024;      // most threads of a plane block
constexpr int kMaxN = 128;           // longest axis
constexpr int kMaxStages = 8;        // FFT stages per axis
constexpr size_t kMaxLds = 163840;   // gfx950 LDS per work-group
constexpr int kXcds = 8;
constexpr int kCus = 256;            // MI355X compute units

// FFT plan of one axis: the radices in stage order (2, 3, 4, 5, 7, 8 have
// their own butterflies; any other prime runs as a direct DFT stage).
struct AxisPlan {
  int n, nst;
  int r[kMaxStages];
};

// One trilinear tap line of a sensor: the sensor's contribution from line
// `line` is wl * f[line][ixl] + wr * f[line][ixr]; slot 0..3 names which of
// the sensor's four lines it is.  Sorted by line.
struct Tap3 {
  int s, slot, line, ixl, ixr;
  float wl, wr;
  int pad;
};

// One grid node that receives the transposed measurement M^T r: the sum of
// w * r[s] over its entries [e0, e1) of the scatter list; sorted by (line, ix).
struct ScatterNode {
  int line, ix, e0, e1;
};
struct ScatterEntry {
  int s;
  float w;
};

struct Medium3 {
  int nx, ny, nz, nxh1, nlines, nt, ns, lossy;
  float dt;
  int rt, ct, ctiles;                 // lines per row tile, columns per plane tile, column tiles
  int rthr, pthr;                     // threads per row / plane block
  AxisPlan px, py, pz;
  const float *c2, *c2eta, *c2tau, *rho0;      // [N]
  const float *bx, *by, *bz;                   // dt / rho0 at the staggered positions [N]
  const float *avx, *arx, *avy, *ary, *avz, *arz;  // PML diagonals [nx] / [ny] / [nz]
  const float2 *dxp, *dxm, *dyp, *dym, *dzp, *dzm;  // 1-D symbols i k e^{+-i k d/2}: [nxh1] / [ny] / [nz]
  const float *kap, *ldis, *labs;              // [nxh1][nz][ny] (a column's lines contiguous), each / N
  const float2 *twx, *twy, *twz;               // e^{-2 pi i m / n}, m < n
  const int* tap_off;                          // [nlines + 1]
  const Tap3* taps;
  const int* node_off;                         // [nlines + 1] into nodes
  const ScatterNode* nodes;
  const ScatterEntry* entries;
};

// Per-vector work buffers.
struct Work3 {
  float* f;       // 7 fields of N: forward v_x v_y v_z rho_x rho_y rho_z p; adjoint their adjoints, q
  float2* s;      // 4 half spectra, each ctiles * ct * nlines (3: the pressure of the forward)
  float* part;    // forward: sensor partials [nt][ns][4]
};

struct IO3 {
  const float* in;   // forward: p0 [N]; adjoint: residual [nt][ns]; apply: field
  float* out;        // forward: data [nt][ns]; adjoint: gradient [N]; apply: field
};

struct Launch3 {
  Medium3 m;
  Work3 w0;
  long long wstride;   // bytes between the work buffers of consecutive items
  int nitems;
  const IO3* io;
};

enum Row3 : int {
  R3_F1 = 0,    // forward: d_i^+ p -> velocity update -> spectra of v_x, v_y, v_z
  R3_F2 = 1,    // forward lossy: d_i^- v_i -> density update (+ source) -> spectra of S, u
  R3_F2L = 2,   // forward lossless: density update -> p, sensors, spectrum of p
  R3_F3 = 3,    // forward lossy: Y_dis S, Y_abs u -> p, sensors, spectrum of p
  R3_A1 = 4,    // adjoint lossy: p* + M^T r -> q, spectra of eta q, tau q
  R3_A1L = 5,   // adjoint lossless: p* + M^T r -> transposed density update -> spectra of e*_i
  R3_A2 = 6,    // adjoint lossy: Y terms -> transposed density update -> spectra of e*_i
  R3_A3 = 7,    // adjoint: transposed velocity update -> spectra of g*_i
  R3_FWD1 = 8,  // field -> spectrum 0
  R3_INV1 = 9   // spectrum 0 -> field
};

enum Plane3 : int {
  P3_GRADP1 = 0,  // 1 -> 3: d_x^+, d_y^+, d_z^+ of spectrum 3 into spectra 0..2
  P3_GRADM2 = 1,  // 3 -> 3: d_i^- of field i
  P3_FRAC = 2,    // 2 -> 2: Y_dis of field 0, Y_abs of field 1
  P3_GRADP2 = 3,  // 3 -> 3: d_i^+ of field i
  P3_APPLY = 5    // 1 -> 1: one operator (code in the launch)
};

enum OpCode3 : int { OP_DXP = 0, OP_DXM, OP_DYP, OP_DYM, OP_DZP, OP_DZM, OP_LDIS, OP_LABS };

// LDS bytes of a row block (two buffers of 3 x rt/2 lines + twiddles) and of
// a plane block (twiddles + two buffers of ct columns x nlines: a block
// transforms one field).
inline size_t row3_lds(int nx, int rt) { return (size_t(2) * 3 * (rt / 2) * nx + nx) * sizeof(float2); }
inline size_t plane3_lds(int ny, int nz, int ct) { return (size_t(2) * ct * ny * nz + ny + nz) * sizeof(float2); }

hipError_t launch_row3(int mode, const Launch3& L, int ntile, int chunk, int n, hipStream_t st);
// blocks per column tile of a plane pass: one per field of the diagonal
// passes and one per output of the gradient (one-field blocks are small
// enough in LDS that several share a CU and hide each other's barrier waits)
__host__ __device__ constexpr int plane3_split(int mode) {
  return (mode == P3_GRADM2 || mode == P3_GRADP2 || mode == P3_GRADP1) ? 3 : mode == P3_FRAC ? 2 : 1;
}
hipError_t launch_plane3(int mode, int code, const Launch3& L, int ntile, int chunk, int n, hipStream_t st);
hipError_t launch_combine3(const Launch3& L, hipStream_t st);
hipError_t k3d_allow_lds(size_t bytes);

}  // namespace qpat3
