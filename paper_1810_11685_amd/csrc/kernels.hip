// HIP kernels of the k-space acoustic operator for gfx950 (MI355X).
//
// Every spectral operator F^-1 diag(m) F of Section 3.2.2 (staggered
// gradients of eq grr, fractional Laplacians Y_dis and Y_abs) is split into
//   row pass  : inverse row FFTs of the previous spectra, the pointwise update
//               of eqs num-vel / num-rho / num-p (or their transposes), and the
//               forward row FFTs of the next fields, all on rows held in LDS;
//   column pass: forward column FFT, multiplier(s), inverse column FFT, on a
//               tile of spectrum columns held in LDS.
// Two real fields share one complex row FFT (z = a + i b); spectra are stored
// as half spectra [ny][nx/2] with the (real) DC and Nyquist columns packed as
// the real and imaginary parts of column 0.  FFTs are radix-2/3/4/8 Stockham
// passes between two LDS buffers; inverse transforms use conj(FFT(conj(.))).
// The 1/(nx ny) normalisation is folded into the multiplier tables.
//
// A launch covers any number of problems ("items", possibly of different
// sizes): block b reads (item, tile) from a block map built on the host, which
// places consecutive tiles of one item on the same XCD.
#include "qpat_internal.hpp"

#include <map>
#include <mutex>

namespace qpat {

// ---------------------------------------------------------------- complex
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
// Complex product with its two fused multiply-adds written out: left to the
// compiler, which product of each part it fuses depends on the surrounding
// code, so two inlined copies of one FFT stage could round differently.
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(__builtin_fmaf(a.x, b.x, -(a.y * b.y)), __builtin_fmaf(a.y, b.x, a.x * b.y));
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }  // -i * a

// ---------------------------------------------------------------- butterflies (forward DFT)
template <int R> __device__ __forceinline__ void bfly(float2* v);

template <> __device__ __forceinline__ void bfly<2>(float2* v) {
  const float2 a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}

template <> __device__ __forceinline__ void bfly<3>(float2* v) {
  const float s = 0.86602540378443864676f;  // sin(pi/3)
  const float2 t1 = cadd(v[1], v[2]);
  const float2 t2 = make_float2(v[0].x - 0.5f * t1.x, v[0].y - 0.5f * t1.y);
  const float2 t3 = mul_mi(cscale(csub(v[1], v[2]), s));
  v[0] = cadd(v[0], t1);
  v[1] = cadd(t2, t3);
  v[2] = csub(t2, t3);
}

template <> __device__ __forceinline__ void bfly<4>(float2* v) {
  const float2 t0 = cadd(v[0], v[2]), t1 = csub(v[0], v[2]);
  const float2 t2 = cadd(v[1], v[3]), t3 = mul_mi(csub(v[1], v[3]));
  v[0] = cadd(t0, t2);
  v[2] = csub(t0, t2);
  v[1] = cadd(t1, t3);
  v[3] = csub(t1, t3);
}

template <> __device__ __forceinline__ void bfly<8>(float2* v) {
  const float c = 0.70710678118654752440f;
  float2 e[4] = {v[0], v[2], v[4], v[6]};
  float2 o[4] = {v[1], v[3], v[5], v[7]};
  bfly<4>(e);
  bfly<4>(o);
  // W8^1 o1 = c (s1 + i d1) and W8^3 o3 = c (d3 - i s3), each scaling fused
  // into the adds and subtracts that use it (written out, as in cmul)
  const float s1 = o[1].x + o[1].y, d1 = o[1].y - o[1].x;
  const float s3 = o[3].x + o[3].y, d3 = o[3].y - o[3].x;
  const float2 o2 = mul_mi(o[2]);  // W8^2
  v[0] = cadd(e[0], o[0]);
  v[4] = csub(e[0], o[0]);
  v[1] = make_float2(__builtin_fmaf(c, s1, e[1].x), __builtin_fmaf(c, d1, e[1].y));
  v[5] = make_float2(__builtin_fmaf(-c, s1, e[1].x), __builtin_fmaf(-c, d1, e[1].y));
  v[2] = cadd(e[2], o2);
  v[6] = csub(e[2], o2);
  v[3] = make_float2(__builtin_fmaf(c, d3, e[3].x), __builtin_fmaf(-c, s3, e[3].y));
  v[7] = make_float2(__builtin_fmaf(-c, d3, e[3].x), __builtin_fmaf(c, s3, e[3].y));
}

// 24-bit unsigned product (full-rate multiply); every grid and spectrum
// index of a pass is below 2^24.
__device__ __forceinline__ unsigned mul24(unsigned a, unsigned b) { return __umul24(a, b); }

// Quotient a / d for 0 <= a < 2^22 without an integer divide: a float
// reciprocal estimate and one exact correction step.
__device__ __forceinline__ int fdiv(int a, int d, float rcp) {
  int q = static_cast<int>(static_cast<float>(a) * rcp);
  const int r = a - q * d;
  q += (r >= d) - (r < 0);
  return q;
}

// column index of element ix of spectrum tile column tx
__device__ __forceinline__ int k_of(int tx, int ix, int lct) { return (tx << lct) + ix; }

// One Stockham stage for butterfly j: reads src[j + r nb], twiddles by
// W_{Ns R}^{k r} (k = j mod Ns, Ns a power of two), writes dst[(j - k) R + k + r Ns].
// Twiddles are stored per stage as [r - 1][k] (the stage's block starts at
// Ns - R0, R0 the first radix), so the lanes of a wave read consecutive
// entries.
template <int R>
__device__ __forceinline__ void stockham(const float2* src, float2* dst, int j, int nb, int Ns,
                                         int off, const float2* tw) {
  float2 v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = src[px(j + r * nb)];
  const int k = j & (Ns - 1);
  if (Ns > 1) {
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[off + (r - 1) * Ns + k]);
  }
  bfly<R>(v);
  const int base = (j - k) * R + k;
#pragma unroll
  for (int r = 0; r < R; ++r) dst[px(base + r * Ns)] = v[r];
}

// Forward FFT of `nlines` lines of length n (line stride ls) held in LDS
// buffer a, using b as the ping-pong partner and the twiddle table tw (LDS).
// The radix plan puts the radix-3 stage (if any) last so that Ns is a power of
// two in every stage.  All threads of the block take part; returns the buffer
// that holds the result.  The caller must have synchronised after writing the
// input; the routine ends synchronised.
__device__ float2* fft_lines(float2* a, float2* b, int nlines, int n, int ls, uint32_t rad, int nst,
                             const float2* tw) {
  int Ns = 1;
  const int R0 = rad & 15;
  for (int s = 0; s < nst; ++s) {
    const int R = (rad >> (4 * s)) & 15;
    const int nb = n / R;
    const float rnb = 1.0f / static_cast<float>(nb);
    const int off = Ns - R0;
    const int total = nlines * nb;
    for (int it = threadIdx.x; it < total; it += blockDim.x) {
      const int line = fdiv(it, nb, rnb);
      const int j = it - line * nb;
      const float2* src = a + line * ls;
      float2* dst = b + line * ls;
      if (R == 8)
        stockham<8>(src, dst, j, nb, Ns, off, tw);
      else if (R == 4)
        stockham<4>(src, dst, j, nb, Ns, off, tw);
      else if (R == 2)
        stockham<2>(src, dst, j, nb, Ns, off, tw);
      else
        stockham<3>(src, dst, j, nb, Ns, off, tw);
    }
    __syncthreads();
    float2* t = a;
    a = b;
    b = t;
    Ns *= R;
  }
  return a;
}

// Compile-time versions of the same radix plans (see plan_radix) for the
// common line lengths: every stage's radix, stride and twiddle step is a
// constant, so index arithmetic folds into shifts and LDS immediate offsets.
__host__ __device__ constexpr int ilog2c(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}
__host__ __device__ constexpr int plan_nst(int n) {
  const bool three = n % 3 == 0;
  const int a = ilog2c(three ? n / 3 : n);
  return (a % 3 ? 1 : 0) + a / 3 + (three ? 1 : 0);
}
// Power-of-two part 2^a: radix 8 stages, with the remainder as two radix-4
// stages at both ends (a = 3q + 1: 4 8..8 4) or one radix-4 second stage
// (a = 3q + 2: 8 4 8..8), so that a plan of two or more stages starts and
// ends with the same radix where it can (the row passes fuse the boundary
// stage of two FFTs); then the radix-3 stage, if any.
__host__ __device__ constexpr int plan_radix(int n, int s) {
  const bool three = n % 3 == 0;
  const int a = ilog2c(three ? n / 3 : n);
  const int rem = a % 3, q = a / 3;
  const int np2 = (rem ? 1 : 0) + q;  // power-of-two stages
  if (s >= np2) return 3;
  if (rem == 0) return 8;
  if (rem == 1) return q == 0 ? 2 : ((s == 0 || s == np2 - 1) ? 4 : 8);
  return q == 0 ? 4 : (s == 1 ? 4 : 8);
}

// Padded offset of a displacement d from a base position b when b + d stays
// in b's run of 8 or d is a multiple of 8: px(b + d) = px(b) + pxd(d).
__host__ __device__ constexpr int pxd(int d) { return d + (d >> 3); }

// The stage shapes of the compile-time plans keep every butterfly access in
// that form: reads j + r NB with NB a multiple of 8; writes base + r NS with
// NS a multiple of 8, or base = (j - k) R + k whose residue mod 8 (k, or a
// multiple of R when NS = 1) leaves room for r NS mod 8.
__host__ __device__ constexpr bool stage_folds(int R, int NS, int NB) {
  return NB % 8 == 0 &&
         (NS % 8 == 0 || (R != 3 && 8 % NS == 0 && (NS == 1 ? 8 % R == 0 : (NS * R) % 8 == 0)));
}

// The three parts of a compile-time stage for butterfly j: gather its inputs
// from an LDS line, twiddle and transform in registers, scatter its outputs.
template <int R, int NB>
__device__ __forceinline__ void stage_load(float2* v, const float2* src, unsigned j) {
  const float2* s = src + px(int(j));
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = s[pxd(r * NB)];
}
template <int R, int NS, int OFF>
__device__ __forceinline__ void stage_regs(float2* v, unsigned j, const float2* tw) {
  if constexpr (NS > 1) {
    const float2* t = tw + OFF + (j & (NS - 1));
#pragma unroll
    for (int r = 1; r < R; ++r) v[r] = cmul(v[r], t[(r - 1) * NS]);
  }
  bfly<R>(v);
}
template <int R, int NS>
__device__ __forceinline__ void stage_store(const float2* v, float2* dst, unsigned j) {
  const unsigned k = j & (NS - 1);
  float2* d = dst + px(int((j - k) * R + k));
#pragma unroll
  for (int r = 0; r < R; ++r) d[pxd(r * NS)] = v[r];
}

template <int R, int NS, int NB, int OFF>
__device__ __forceinline__ void stockham_c(const float2* src, float2* dst, unsigned j, const float2* tw) {
  static_assert(stage_folds(R, NS, NB), "stage offsets do not fold");
  float2 v[R];
  stage_load<R, NB>(v, src, j);
  stage_regs<R, NS, OFF>(v, j, tw);
  stage_store<R, NS>(v, dst, j);
}

// LS: line stride (a compile-time constant, so line offsets fold too).
template <int N, int LS, int S, int NS>
__device__ __forceinline__ float2* fft_c(float2* a, float2* b, int nlines, const float2* tw) {
  if constexpr (S == plan_nst(N)) {
    return a;
  } else {
    constexpr int R = plan_radix(N, S), NB = N / R, OFF = NS - plan_radix(N, 0);
    const unsigned total = unsigned(nlines) * NB;
    for (unsigned it = threadIdx.x; it < total; it += blockDim.x) {
      const unsigned line = it / NB, j = it % NB;
      stockham_c<R, NS, NB, OFF>(a + line * LS, b + line * LS, j, tw);
    }
    __syncthreads();
    return fft_c<N, LS, S + 1, NS * R>(b, a, nlines, tw);
  }
}

// In-place version: every thread gathers and transforms all its butterflies
// of a stage, the block synchronises, then every thread scatters its outputs
// into the same buffer.  A thread holds at most kMaxPer values per stage
// (the host bounds a tile to kMaxPer elements per thread).
template <int N, int LS, int S, int NS>
__device__ __forceinline__ float2* fft_c_ip(float2* a, int nlines, const float2* tw) {
  if constexpr (S == plan_nst(N)) {
    return a;
  } else {
    constexpr int R = plan_radix(N, S), NB = N / R, OFF = NS - plan_radix(N, 0);
    constexpr int MB = (kMaxPer + R - 1) / R;
    const unsigned total = unsigned(nlines) * NB;
    float2 v[MB][R];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
      const unsigned it = threadIdx.x + i * blockDim.x;
      if (it < total) {
        const unsigned line = it / NB, j = it % NB;
        static_assert(stage_folds(R, NS, NB), "stage offsets do not fold");
        stage_load<R, NB>(v[i], a + line * LS, j);
        stage_regs<R, NS, OFF>(v[i], j, tw);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MB; ++i) {
      const unsigned it = threadIdx.x + i * blockDim.x;
      if (it < total) {
        const unsigned line = it / NB, j = it % NB;
        stage_store<R, NS>(v[i], a + line * LS, j);
      }
    }
    __syncthreads();
    return fft_c_ip<N, LS, S + 1, NS * R>(a, nlines, tw);
  }
}

// Radix of stage s of the compile-time plan of length N, or of that plan in
// reverse order (REV).  A power-of-two plan reversed still has power-of-two
// Ns in every stage; its per-stage twiddles form their own table.
template <int N, bool REV>
__host__ __device__ constexpr int radix_of(int s) {
  return REV ? plan_radix(N, plan_nst(N) - 1 - s) : plan_radix(N, s);
}

// Stages S .. S1-1 of the plan (direction REV) on `nlines` LDS lines of
// stride LS, ping-ponging from a; NS = product of the radices before S.
// Returns the buffer holding the result; ends synchronised.
template <int N, bool REV, int LS, int S, int S1, int NS>
__device__ __forceinline__ float2* fft_stages(float2* a, float2* b, int nlines, const float2* tw) {
  if constexpr (S == S1) {
    return a;
  } else {
    constexpr int R = radix_of<N, REV>(S), NB = N / R, OFF = NS - radix_of<N, REV>(0);
    const unsigned total = unsigned(nlines) * NB;
    for (unsigned it = threadIdx.x; it < total; it += blockDim.x) {
      const unsigned line = it / NB, j = it % NB;
      stockham_c<R, NS, NB, OFF>(a + line * LS, b + line * LS, j, tw);
    }
    __syncthreads();
    return fft_stages<N, REV, LS, S + 1, S1, NS * R>(b, a, nlines, tw);
  }
}

// Stages S .. S1-1 of the plan of length N (REV: the plan in reverse order)
// in place (see fft_c_ip).
template <int N, int LS, int S, int S1, int NS, bool REV = false>
__device__ __forceinline__ float2* fft_range_ip(float2* a, int nlines, const float2* tw) {
  if constexpr (S == S1) {
    return a;
  } else {
    constexpr int R = radix_of<N, REV>(S), NB = N / R, OFF = NS - radix_of<N, REV>(0);
    constexpr int MB = (kMaxPer + R - 1) / R;
    const unsigned total = unsigned(nlines) * NB;
    float2 v[MB][R];
#pragma unroll
    for (int i = 0; i < MB; ++i) {
      const unsigned it = threadIdx.x + i * blockDim.x;
      if (it < total) {
        const unsigned line = it / NB, j = it % NB;
        stage_load<R, NB>(v[i], a + line * LS, j);
        stage_regs<R, NS, OFF>(v[i], j, tw);
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MB; ++i) {
      const unsigned it = threadIdx.x + i * blockDim.x;
      if (it < total) {
        const unsigned line = it / NB, j = it % NB;
        stage_store<R, NS>(v[i], a + line * LS, j);
      }
    }
    __syncthreads();
    return fft_range_ip<N, LS, S + 1, S1, NS * R, REV>(a, nlines, tw);
  }
}

// Row lines whose plan starts and ends with the same radix (512 = 8 8 8):
// the two FFTs of a row pass around a pointwise update share their boundary
// stage in registers.  The last stage of the first FFT leaves butterfly jj of
// a line with the values at jj + r N/R, exactly the inputs of butterfly jj in
// the first stage of the second FFT, so one thread per (line, jj) runs that
// last stage, the update `pw(line, jj, v)` on its R values, and that first
// stage, skipping an LDS round trip and a barrier on each side of the
// update.  The arithmetic is the unfused sequence's.  Ends synchronised with
// the second FFT's result in the returned buffer.
template <int N>
__host__ __device__ constexpr bool row_fusable() {
  return N > 0 && (N & (N - 1)) == 0 && plan_radix(N, 0) == plan_radix(N, plan_nst(N) - 1) && plan_nst(N) >= 2;
}
template <int N>
__host__ __device__ constexpr int fused_slots() { return (kMaxPer + plan_radix(N, 0) - 1) / plan_radix(N, 0); }
// pw(i, line, jj, v): the update of butterfly slot i (0 <= i < fused_slots)
// of this thread, (line, jj), on its R values v.  A thread has at most
// fused_slots butterflies (the host bounds a tile to kMaxPer elements per
// thread), slot i being butterfly threadIdx.x + i blockDim.x.
template <int N, bool IP, class PW>
__device__ __forceinline__ float2* fft_fused(float2* a, float2* b, int nlines, const float2* tw, PW pw) {
  constexpr int LS = lstride(N), NST = plan_nst(N), R = plan_radix(N, 0), NB = N / R, MB = fused_slots<N>();
  constexpr int OFFL = NB - R;  // twiddles of the last stage (Ns = N / R)
  float2* r;
  if constexpr (IP) r = fft_range_ip<N, LS, 0, NST - 1, 1>(a, nlines, tw);
  else r = fft_stages<N, false, LS, 0, NST - 1, 1>(a, b, nlines, tw);
  float2* o = IP ? r : (r == a ? b : a);
  const unsigned total = unsigned(nlines) * NB;
  float2 v[MB][R];
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const unsigned it = threadIdx.x + i * blockDim.x;
    if (it < total) {
      const unsigned line = it / NB, jj = it % NB;
      stage_load<R, NB>(v[i], r + line * LS, jj);
      stage_regs<R, NB, OFFL>(v[i], jj, tw);
    }
  }
  if constexpr (IP) __syncthreads();
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const unsigned it = threadIdx.x + i * blockDim.x;
    if (it < total) {
      const unsigned line = it / NB, jj = it % NB;
      // The values pass an LDS store and load in the unfused sequence; the
      // empty asm statements keep them opaque here too, so no multiply of
      // one side is contracted with an add of the other (same rounding).
#pragma unroll
      for (int q = 0; q < R; ++q) asm volatile("" : "+v"(v[i][q].x), "+v"(v[i][q].y));
      pw(i, int(line), int(jj), v[i]);
#pragma unroll
      for (int q = 0; q < R; ++q) asm volatile("" : "+v"(v[i][q].x), "+v"(v[i][q].y));
      stage_regs<R, 1, 0>(v[i], jj, tw);
      stage_store<R, 1>(v[i], o + line * LS, jj);
    }
  }
  __syncthreads();
  if constexpr (IP) return fft_range_ip<N, LS, 1, NST, R>(o, nlines, tw);
  else return fft_stages<N, false, LS, 1, NST, R>(o, r, nlines, tw);
}

// The same fusion for updates that read two lines and write two lines per
// position (rows 2l and 2l+1 packed as one complex line on one side of the
// update, each row its own line on the other): work item (l, jj) runs the
// last stage on lines inl(l, 0) and inl(l, 1), `pw(i, l, jj, va, vb)` on their
// values, and the first stage on lines outl(l, 0) and outl(l, 1).
template <int N>
__host__ __device__ constexpr int fused2_slots() { return (kMaxPer / 2 + plan_radix(N, 0) - 1) / plan_radix(N, 0); }
template <int N, bool IP, class IL, class OL, class PW>
__device__ __forceinline__ float2* fft_fused2(float2* a, float2* b, int nlines, const float2* tw, IL inl, OL outl,
                                              PW pw) {
  constexpr int LS = lstride(N), NST = plan_nst(N), R = plan_radix(N, 0), NB = N / R, MB = fused2_slots<N>();
  constexpr int OFFL = NB - R;
  float2* r;
  if constexpr (IP) r = fft_range_ip<N, LS, 0, NST - 1, 1>(a, nlines, tw);
  else r = fft_stages<N, false, LS, 0, NST - 1, 1>(a, b, nlines, tw);
  float2* o = IP ? r : (r == a ? b : a);
  const unsigned total = unsigned(nlines / 2) * NB;
  float2 va[MB][R], vb[MB][R];
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const unsigned it = threadIdx.x + i * blockDim.x;
    if (it < total) {
      const int l = int(it / NB);
      const unsigned jj = it % NB;
      stage_load<R, NB>(va[i], r + inl(l, 0) * LS, jj);
      stage_regs<R, NB, OFFL>(va[i], jj, tw);
      stage_load<R, NB>(vb[i], r + inl(l, 1) * LS, jj);
      stage_regs<R, NB, OFFL>(vb[i], jj, tw);
    }
  }
  if constexpr (IP) __syncthreads();
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const unsigned it = threadIdx.x + i * blockDim.x;
    if (it < total) {
      const int l = int(it / NB);
      const unsigned jj = it % NB;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        asm volatile("" : "+v"(va[i][q].x), "+v"(va[i][q].y));
        asm volatile("" : "+v"(vb[i][q].x), "+v"(vb[i][q].y));
      }
      pw(i, l, int(jj), va[i], vb[i]);
#pragma unroll
      for (int q = 0; q < R; ++q) {
        asm volatile("" : "+v"(va[i][q].x), "+v"(va[i][q].y));
        asm volatile("" : "+v"(vb[i][q].x), "+v"(vb[i][q].y));
      }
      stage_regs<R, 1, 0>(va[i], jj, tw);
      stage_store<R, 1>(va[i], o + outl(l, 0) * LS, jj);
      stage_regs<R, 1, 0>(vb[i], jj, tw);
      stage_store<R, 1>(vb[i], o + outl(l, 1) * LS, jj);
    }
  }
  __syncthreads();
  if constexpr (IP) return fft_range_ip<N, LS, 1, NST, R>(o, nlines, tw);
  else return fft_stages<N, false, LS, 1, NST, R>(o, r, nlines, tw);
}

// First thread index of this thread's wavefront as a scalar, so that tests on
// it compile to scalar branches: a wave whose lanes have no work item skips a
// fused section (and its operand loads) as a whole, while the lanes of a wave
// with work stay together for the lane exchanges.
__device__ __forceinline__ unsigned wave_base() { return __builtin_amdgcn_readfirstlane(threadIdx.x) & ~63u; }

// The value x of the adjacent lane (lane ^ 1): a DPP quad permutation
// [1, 0, 3, 2], a VALU move (no LDS round trip).  Both lanes of a pair must
// be active.
__device__ __forceinline__ float lane_pair_swap(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));
}

// The same fusion for updates that pair rows 2l and 2l+1 as one complex line
// on one side of the update and keep each row its own line on the other.
// Work item (l, sd, jj) runs the last stage on line inl(l, sd), the update
// `pw(i, l, sd, jj, v, active)` of row 2l + sd, and the first stage on line
// outl(l, sd).  Consecutive work items hold the two rows of a pair, so the
// two lanes of a pair trade the half of a packed line each needs with one
// lane shuffle per value inside pw; pw therefore runs on every lane (lanes
// without a work item hold zeros and `active` false).
template <int N, bool IP, class IL, class OL, class PW>
__device__ __forceinline__ float2* fft_fused_pairs(float2* a, float2* b, int nlines, const float2* tw, IL inl,
                                                   OL outl, PW pw) {
  constexpr int LS = lstride(N), NST = plan_nst(N), R = plan_radix(N, 0), NB = N / R, MB = fused_slots<N>();
  constexpr int OFFL = NB - R;
  float2* r;
  if constexpr (IP) r = fft_range_ip<N, LS, 0, NST - 1, 1>(a, nlines, tw);
  else r = fft_stages<N, false, LS, 0, NST - 1, 1>(a, b, nlines, tw);
  float2* o = IP ? r : (r == a ? b : a);
  const unsigned total = unsigned(nlines) * NB;  // even: pairs are both in range or both out
  float2 v[MB][R];
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const unsigned it = threadIdx.x + i * blockDim.x;
    const unsigned p = it >> 1, sd = it & 1u, l = p / NB, jj = p % NB;
    if (it < total) {
      stage_load<R, NB>(v[i], r + inl(int(l), int(sd)) * LS, jj);
      stage_regs<R, NB, OFFL>(v[i], jj, tw);
    } else {
#pragma unroll
      for (int q = 0; q < R; ++q) v[i][q] = make_float2(0.f, 0.f);
    }
  }
  if constexpr (IP) __syncthreads();
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    if (wave_base() + i * blockDim.x < total) {  // wave-uniform: the exchanges see whole waves
      const unsigned it = threadIdx.x + i * blockDim.x;
      const unsigned p = it >> 1, sd = it & 1u, l = p / NB, jj = p % NB;
      const bool active = it < total;
#pragma unroll
      for (int q = 0; q < R; ++q) asm volatile("" : "+v"(v[i][q].x), "+v"(v[i][q].y));
      pw(i, int(l), int(sd), int(jj), v[i], active);
#pragma unroll
      for (int q = 0; q < R; ++q) asm volatile("" : "+v"(v[i][q].x), "+v"(v[i][q].y));
      if (active) {
        stage_regs<R, 1, 0>(v[i], jj, tw);
        stage_store<R, 1>(v[i], o + outl(int(l), int(sd)) * LS, jj);
      }
    }
  }
  __syncthreads();
  if constexpr (IP) return fft_range_ip<N, LS, 1, NST, R>(o, nlines, tw);
  else return fft_stages<N, false, LS, 1, NST, R>(o, r, nlines, tw);
}

// FFT of `nlines` lines: compile-time plan for the common lengths, the
// runtime plan otherwise.  Same contract as fft_lines; row lines have stride
// lstride(n), column lines (COL) col_lstride(n).  IP (instances with a
// compile-time length only, n == NF): the stages run in place in a (b unused).
// NF != 0: a kernel instance for lines of length NF carries that compile-time
// plan only (and the runtime plan as a fallback), so the other lengths'
// unrolled code does not weigh on it.
template <bool COL, int NF = 0, bool IP = false>
__device__ __forceinline__ float2* fft_any(float2* a, float2* b, int nlines, int n, int ls, uint32_t rad,
                                           int nst, const float2* tw) {
  if constexpr (NF != 0) {
    if constexpr (IP) return fft_c_ip<NF, COL ? col_lstride(NF) : lstride(NF), 0, 1>(a, nlines, tw);
    if (n == NF) return fft_c<NF, COL ? col_lstride(NF) : lstride(NF), 0, 1>(a, b, nlines, tw);
    return fft_lines(a, b, nlines, n, ls, rad, nst, tw);
  } else {
#define QPAT_FFT_CASE(N) \
  case N: return fft_c<N, COL ? col_lstride(N) : lstride(N), 0, 1>(a, b, nlines, tw);
    switch (n) {
      QPAT_FFT_CASE(128)
      QPAT_FFT_CASE(256)
      QPAT_FFT_CASE(384)
      QPAT_FFT_CASE(512)
      QPAT_FFT_CASE(1024)
      default: return fft_lines(a, b, nlines, n, ls, rad, nst, tw);
    }
#undef QPAT_FFT_CASE
  }
}

// ---------------------------------------------------------------- packing
// Conjugated inverse-FFT input of the pair (A, B) of packed half-spectrum
// rows: Z = A + iB with Hermitian completion; writes Z[k] and Z[n-k].
__device__ __forceinline__ void build_inv(float2* L, float2 A, float2 B, int k, int nx, int nxh) {
  if (k == 0) {
    L[0] = make_float2(A.x, -B.x);
    L[px(nxh)] = make_float2(A.y, -B.y);
  } else {
    L[px(k)] = make_float2(A.x - B.y, -(A.y + B.x));
    L[px(nx - k)] = make_float2(A.x + B.y, -(B.x - A.y));
  }
}

// Split the FFT Z of a + i b into the packed half spectra A (of a), B (of b).
__device__ __forceinline__ void unpack(const float2* L, int k, int nx, int nxh, float2& A, float2& B) {
  if (k == 0) {
    const float2 z0 = L[0], zn = L[px(nxh)];
    A = make_float2(z0.x, zn.x);
    B = make_float2(z0.y, zn.y);
  } else {
    const float2 zk = L[px(k)], zm = L[px(nx - k)];
    A = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
    B = make_float2(0.5f * (zk.y + zm.y), 0.5f * (zm.x - zk.x));
  }
}

__device__ __forceinline__ float2* other(float2* r, float2* a, float2* b) { return r == a ? b : a; }

// Half spectra are stored in tiles of rt rows x ct columns (the row- and
// column-pass tile sizes): element (ky, kx) sits at
//   ((ky / rt) (nxh / ct) + kx / ct) rt ct + (ky mod rt) ct + kx mod ct,
// so the rt rows of one row tile form one contiguous run and a column tile is
// a sequence of runs of rt*ct elements.  All loops below walk memory order.

// The load phase of a block issues every global load before its first LDS
// write: fetch_* gathers into registers, put_* scatters into LDS, so the phase
// costs one memory round trip rather than one per loop iteration.  Bounds
// (enforced on the host): a row tile holds rt*nx <= kMaxPer*B reals, hence at
// most kPairIt complex pairs per thread; a line length is at most kMaxPer*B.
constexpr int kPairIt = kMaxPer / 2;
constexpr int kRowPairIt = kMaxPer / 4;

struct PairRegs {
  float2 a[kPairIt], b[kPairIt];
};
struct RowPairRegs {
  float2 a[kRowPairIt], b[kRowPairIt];
};
template <int K>
struct TwRegsK {
  float2 t[K];
};
using TwRegs = TwRegsK<kMaxPer>;

// Row length of a row-pass instance: the compile-time length NF when the
// instance carries one (it is launched only for rows of that length), else
// the plan's.  nxh = nx / 2 (half-spectrum columns).
template <int NF>
__device__ __forceinline__ int row_len(const Medium& M) { return NF > 0 ? NF : M.nx; }
template <int NF>
__device__ __forceinline__ int row_half(const Medium& M) { return NF > 0 ? NF / 2 : M.nxh; }

// Spectra are stored in tiles of srt rows x ct columns (row tiles of srt
// rows one after another, the column tiles of one row tile one after another,
// each tile row-major).  A row block's rt rows (srt a multiple of rt) are rows
// r0 .. r0 + rt - 1 of one storage row tile.  The block enumerates its
// elements p in the order of an rt x ct tiling (column tile major); element p
// sits at spec_row_base + spec_row_off(p).  With srt = rt that is base + p.
template <int NF>
__device__ __forceinline__ unsigned spec_row_base(const Medium& M, int tile) {
  const unsigned y0 = unsigned(tile) << M.lrt;
  return mul24(y0 >> M.lsrt, unsigned(M.srt * row_half<NF>(M))) + ((y0 & unsigned(M.srt - 1)) << M.lct);
}
__device__ __forceinline__ unsigned spec_row_off(const Medium& M, unsigned p) {
  const int s = M.lrt + M.lct;
  return ((p >> s) << (M.lsrt + M.lct)) + (p & ((1u << s) - 1u));
}

// line j <- rows j of the row tile (s0, s1)
template <int NF>
__device__ __forceinline__ void fetch_pair(PairRegs& R, const Medium& M, const float2* __restrict__ s0,
                                           const float2* __restrict__ s1, int tile) {
  const int tot = M.rt * row_half<NF>(M);
  const unsigned base = spec_row_base<NF>(M, tile);
#pragma unroll
  for (int k = 0; k < kPairIt; ++k) {
    const int p = threadIdx.x + k * blockDim.x;
    if (p < tot) {
      const unsigned o = base + spec_row_off(M, p);
      R.a[k] = s0[o];
      R.b[k] = s1[o];
    }
  }
}
template <int NF>
__device__ __forceinline__ void put_pair(const PairRegs& R, float2* buf, const Medium& M) {
  const int nx = row_len<NF>(M), nxh = row_half<NF>(M), LS = lstride(nx), rc = M.rt * M.ct, tot = M.rt * nxh;
#pragma unroll
  for (int k = 0; k < kPairIt; ++k) {
    const int p = threadIdx.x + k * blockDim.x;
    if (p < tot) {
      const int w = p & (rc - 1);
      const int j = w >> M.lct, kx = ((p >> (M.lrt + M.lct)) << M.lct) + (w & (M.ct - 1));
      build_inv(buf + j * LS, R.a[k], R.b[k], kx, nx, nxh);
    }
  }
}

// line l <- rows (2l, 2l+1) of the row tile of s0
template <int NF>
__device__ __forceinline__ void fetch_rowpair(RowPairRegs& R, const Medium& M, const float2* __restrict__ s0,
                                              int tile) {
  const int nxh = row_half<NF>(M), hc = (M.rt >> 1) * M.ct, tot = (M.rt >> 1) * nxh;
  const unsigned base = spec_row_base<NF>(M, tile);
#pragma unroll
  for (int k = 0; k < kRowPairIt; ++k) {
    const int q = threadIdx.x + k * blockDim.x;
    if (q < tot) {
      const int tx = q >> (M.lrt - 1 + M.lct), w2 = q & (hc - 1);
      const int l = w2 >> M.lct, ix = w2 & (M.ct - 1);
      const unsigned off = base + (unsigned(tx) << (M.lsrt + M.lct)) + (2 * l) * M.ct + ix;
      R.a[k] = s0[off];
      R.b[k] = s0[off + M.ct];
    }
  }
}
template <int NF>
__device__ __forceinline__ void put_rowpair(const RowPairRegs& R, float2* buf, const Medium& M) {
  const int nx = row_len<NF>(M), nxh = row_half<NF>(M), LS = lstride(nx), hc = (M.rt >> 1) * M.ct,
            tot = (M.rt >> 1) * nxh;
#pragma unroll
  for (int k = 0; k < kRowPairIt; ++k) {
    const int q = threadIdx.x + k * blockDim.x;
    if (q < tot) {
      const int tx = q >> (M.lrt - 1 + M.lct), w2 = q & (hc - 1);
      const int l = w2 >> M.lct, ix = w2 & (M.ct - 1);
      build_inv(buf + l * LS, R.a[k], R.b[k], k_of(tx, ix, M.lct), nx, nxh);
    }
  }
}

template <int K>
__device__ __forceinline__ void fetch_tw(TwRegsK<K>& R, const float2* __restrict__ tw, int n) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = threadIdx.x + k * blockDim.x;
    if (i < n) R.t[k] = tw[i];
  }
}
template <int K>
__device__ __forceinline__ void put_tw(const TwRegsK<K>& R, float2* dst, int n) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = threadIdx.x + k * blockDim.x;
    if (i < n) dst[i] = R.t[k];
  }
}

// Spectrum store; NT (launches of about one block per CU): non-temporal, so
// the kernel's end has fewer dirty L2 lines to write back before the next
// pass, on other XCDs, reads them.  With many blocks per CU the plain store is
// the faster one (measured: one 512^2 vector 154.0 -> 152.0 ms non-temporal,
// 1024^2 x 8 pass sum 554 -> 661 us).
typedef float f2v_t __attribute__((ext_vector_type(2)));
template <bool NT>
__device__ __forceinline__ void st_spec(float2* p, float2 v) {
  if constexpr (NT) {
    f2v_t x;
    x.x = v.x;
    x.y = v.y;
    __builtin_nontemporal_store(x, reinterpret_cast<f2v_t*>(p));
  } else {
    *p = v;
  }
}

// (the store loops are unrolled so that the LDS reads of several iterations
// are in flight together: the global stores in between cannot alias LDS)
template <int NF, bool NT = false>
__device__ __forceinline__ void store_pair_spectra(const float2* buf, const Medium& M, float2* __restrict__ s0,
                                                   float2* __restrict__ s1, int tile) {
  const int nx = row_len<NF>(M), nxh = row_half<NF>(M), LS = lstride(nx), rc = M.rt * M.ct;
  const unsigned base = spec_row_base<NF>(M, tile);
#pragma unroll 4
  for (int p = threadIdx.x; p < M.rt * nxh; p += blockDim.x) {
    const int w = p & (rc - 1);
    const int j = w >> M.lct, k = ((p >> (M.lrt + M.lct)) << M.lct) + (w & (M.ct - 1));
    float2 A, B;
    unpack(buf + j * LS, k, nx, nxh, A, B);
    const unsigned o = base + spec_row_off(M, p);
    st_spec<NT>(s0 + o, A);
    st_spec<NT>(s1 + o, B);
  }
}

template <int NF, bool NT = false>
__device__ __forceinline__ void store_rowpair_spectra(const float2* buf, const Medium& M, float2* __restrict__ s0,
                                                      int tile) {
  const int nx = row_len<NF>(M), nxh = row_half<NF>(M), LS = lstride(nx), hc = (M.rt >> 1) * M.ct;
  const unsigned base = spec_row_base<NF>(M, tile);
#pragma unroll 4
  for (int q = threadIdx.x; q < (M.rt >> 1) * nxh; q += blockDim.x) {
    const int tx = q >> (M.lrt - 1 + M.lct), w2 = q & (hc - 1);
    const int l = w2 >> M.lct, ix = w2 & (M.ct - 1);
    const unsigned off = base + (unsigned(tx) << (M.lsrt + M.lct)) + (2 * l) * M.ct + ix;
    float2 A, B;
    unpack(buf + l * LS, k_of(tx, ix, M.lct), nx, nxh, A, B);
    st_spec<NT>(s0 + off, A);
    st_spec<NT>(s0 + off + M.ct, B);
  }
}

// Row-pair LDS layout: row y0+j lives in component (j & 1) of line j >> 1.
__device__ __forceinline__ float& pcomp(float2* buf, int j, int x, int nx) {
  float2* e = buf + (j >> 1) * lstride(nx) + px(x);
  return (j & 1) ? e->y : e->x;
}

// Value of row y0+j after an inverse FFT of row-pair lines (conj trick undone).
__device__ __forceinline__ float rowpair_val(const float2* buf, int j, int x, int nx) {
  const float2 e = buf[(j >> 1) * lstride(nx) + px(x)];
  return (j & 1) ? -e.y : e.x;
}

// Sensor taps of the tile's rows (and, in the adjoint, the residual samples
// they need, in tap order) are staged in LDS; entries beyond the LDS capacity
// are read from global memory.  The tap range is read with the first loads of
// a block; the taps themselves are fetched after the first barrier (thread i
// holds tap e0 + i, blockDim.x >= kTapCap) and written to LDS only where the
// sensors are used, so their latency hides behind the first FFT.

struct TapStage {
  Tap* tl;     // [kTapCap]
  float* rv;   // [kTapCap]
  int e0, e1;  // CSR range of the tile
  int w[8];    // this thread's tap, word by word
  float r;     // and its residual sample
  int n0, n1;  // adjoint: CSR range of the tile's scatter nodes
  int4 nd;     // this thread's node (y, x, c0, c1)
  int con[kConRegs];  // and its first contributions
};

__device__ __forceinline__ void taps_range(TapStage& T, const Medium& M, void* base, int y0, int rt,
                                           bool nodes = false) {
  T.tl = reinterpret_cast<Tap*>(base);
  T.rv = reinterpret_cast<float*>(T.tl + kTapCap);
  T.e0 = M.tap_off[y0];
  T.e1 = M.tap_off[y0 + rt];
  if (nodes) {
    T.n0 = M.node_off[y0];
    T.n1 = M.node_off[y0 + rt];
  }
}

// Adjoint: this thread's scatter node and its first contributions, one record
// (issued early, consumed after the inverse FFT).
__device__ __forceinline__ void nodes_fetch(TapStage& T, const Medium& M) {
  const int i = threadIdx.x;
  if (i < T.n1 - T.n0) {
    const int4* rec = M.nodes + 2 * (T.n0 + i);
    T.nd = rec[0];
    const int4 c = rec[1];
    T.con[0] = c.x;
    T.con[1] = c.y;
    T.con[2] = c.z;
    T.con[3] = c.w;
  }
}

// rtap: residual samples in tap order for sample m ([nt][ntap]), or null
__device__ __forceinline__ void taps_fetch(TapStage& T, const Medium& M, const float* __restrict__ rtap, int m) {
  const int i = threadIdx.x;
  if (i < min(T.e1 - T.e0, kTapCap)) {
    const int4* src = reinterpret_cast<const int4*>(M.taps + T.e0 + i);
    const int4 lo = src[0], hi = src[1];
    T.w[0] = lo.x, T.w[1] = lo.y, T.w[2] = lo.z, T.w[3] = lo.w;
    T.w[4] = hi.x, T.w[5] = hi.y, T.w[6] = hi.z, T.w[7] = hi.w;
    if (rtap) T.r = rtap[unsigned(m) * unsigned(2 * M.ns) + T.e0 + i];
  }
}

__device__ __forceinline__ void taps_put(const TapStage& T, bool with_res) {
  const int i = threadIdx.x;
  if (i < min(T.e1 - T.e0, kTapCap)) {
    int4* dst = reinterpret_cast<int4*>(T.tl + i);
    dst[0] = make_int4(T.w[0], T.w[1], T.w[2], T.w[3]);
    dst[1] = make_int4(T.w[4], T.w[5], T.w[6], T.w[7]);
    if (with_res) T.rv[i] = T.r;
  }
}

__device__ __forceinline__ Tap tap_at(const Medium& M, const TapStage& T, int e) {
  const Tap* src = (e - T.e0 < kTapCap) ? T.tl + (e - T.e0) : M.taps + e;
  Tap t;
  t.s = src->s;
  t.slot = src->slot;
  t.y = src->y;
  t.ixl = src->ixl;
  t.ixr = src->ixr;
  t.wl = src->wl;
  t.wr = src->wr;
  t.pad = 0;
  return t;
}

// Forward sensor partials for rows y0 .. y0+rt-1 (bilinear taps, eq num-m).
__device__ __forceinline__ void sensor_partials(const Medium& M, const TapStage& T, float2* buf, int y0,
                                                float* __restrict__ part, int m) {
  for (int e = T.e0 + threadIdx.x; e < T.e1; e += blockDim.x) {
    const Tap t = tap_at(M, T, e);
    const int j = t.y - y0;
    const float v = t.wl * pcomp(buf, j, t.ixl, M.nx) + t.wr * pcomp(buf, j, t.ixr, M.nx);
    part[(unsigned(m) * unsigned(M.ns) + t.s) * 2 + t.slot] = v;
  }
}

// Adjoint sensor scatter M^T r for rows y0 .. y0+rt-1 as a gather: one thread
// per grid node a tap touches adds that node's contributions in increasing
// tap index, the order of a serial scatter over the row's taps, so the result
// does not depend on the thread count.
__device__ __forceinline__ float scatter_term(const Medium& M, const TapStage& T, const float* __restrict__ rtap,
                                              int m, float acc, int code) {
  const int e = code >> 1;
  const bool staged = e - T.e0 < kTapCap;
  const Tap* src = staged ? T.tl + (e - T.e0) : M.taps + e;
  const float w = (code & 1) ? src->wr : src->wl;
  const float rv = staged ? T.rv[e - T.e0] : rtap[unsigned(m) * unsigned(2 * M.ns) + e];
  return acc + w * rv;
}

__device__ __forceinline__ void sensor_scatter(const Medium& M, const TapStage& T, float2* buf, int y0,
                                               const float* __restrict__ rtap, int m) {
  const int nn = T.n1 - T.n0;
  for (int i = threadIdx.x; i < nn; i += blockDim.x) {
    const bool pre = i == int(threadIdx.x);  // the first round's node was fetched early
    const int4 nd = pre ? T.nd : M.nodes[2 * (T.n0 + i)];
    float& v = pcomp(buf, nd.x - y0, nd.y, M.nx);
    float acc = v;
#pragma unroll
    for (int k = 0; k < kConRegs; ++k)
      if (nd.z + k < nd.w) acc = scatter_term(M, T, rtap, m, acc, pre ? T.con[k] : M.scon[nd.z + k]);
    for (int c = nd.z + kConRegs; c < nd.w; ++c) acc = scatter_term(M, T, rtap, m, acc, M.scon[c]);
    v = acc;
  }
}

// ---------------------------------------------------------------- block -> (item, tile)
// Uniform launches (all items are vectors of one plan) carry the medium in
// the kernel arguments and find their work buffers by a fixed stride, so the
// first global loads of a block are its data; other launches read (item,
// tile) from a block map and the item descriptors from device memory.
// Either way consecutive tiles of one item are placed on one XCD.
template <bool U>
__device__ __forceinline__ bool locate(const Launch& L, int ntile, int chunk, int& item, int& tile) {
  if constexpr (U) {
    const int b = blockIdx.x;
    const int i = (b & (kXcds - 1)) * chunk + (b / kXcds);
    if (i >= L.nitems * ntile) return false;
    item = i / ntile;
    tile = i - item * ntile;
    return true;
  } else {
    const int2 bm = L.map[blockIdx.x];
    item = bm.x;
    tile = bm.y;
    return bm.x >= 0;
  }
}

template <bool U>
__device__ __forceinline__ const Medium& medium_of(const Launch& L, int item) {
  if constexpr (U)
    return L.m;
  else
    return L.items[item].m;
}

__device__ __forceinline__ Work shift_work(const Work& w, long long off) {
  Work r;
  r.f0 = reinterpret_cast<float*>(reinterpret_cast<char*>(w.f0) + off);
  r.f1 = reinterpret_cast<float*>(reinterpret_cast<char*>(w.f1) + off);
  r.f2 = reinterpret_cast<float*>(reinterpret_cast<char*>(w.f2) + off);
  r.f3 = reinterpret_cast<float*>(reinterpret_cast<char*>(w.f3) + off);
  r.q = reinterpret_cast<float*>(reinterpret_cast<char*>(w.q) + off);
  r.s0 = reinterpret_cast<float2*>(reinterpret_cast<char*>(w.s0) + off);
  r.s1 = reinterpret_cast<float2*>(reinterpret_cast<char*>(w.s1) + off);
  r.part = reinterpret_cast<float*>(reinterpret_cast<char*>(w.part) + off);
  return r;
}

// ---------------------------------------------------------------- kernel arguments
// The scalar cache is cold when a kernel starts, so every kernel-argument
// load is a memory round trip.  The compiler issues loads where their values
// are first needed: behind the early-exit branches of the prologue that makes
// two or three dependent round trips before a block's first data load.  These
// empty asm statements take the fields the prologue and the load phase of a
// uniform launch need (and the block size, an implicit argument) as SGPR
// operands, so their loads issue as one batch at the top of the kernel.  (Table launches read their medium from the item
// table in global memory after locating the item.)
template <int BM>
__device__ __forceinline__ void row_args_batch(const Launch& L, int ntile, int chunk, int n, int flags) {
  const Medium& m = L.m;
  const Work& w = L.w0;
  asm volatile("" ::"s"(ntile), "s"(chunk), "s"(n), "s"(flags), "s"(L.nitems), "s"(L.wstride), "s"(m.nx),
               "s"(m.nxh), "s"(m.nt), "s"(m.rt), "s"(m.ct), "s"(m.lrt), "s"(m.lct), "s"(m.twx), "s"(blockDim.x));
  asm volatile("" ::"s"(m.srt), "s"(m.lsrt));
  if constexpr (BM == RM_F1 || BM == RM_A3) {
    asm volatile("" ::"s"(w.s0), "s"(w.s1), "s"(w.f0), "s"(w.f1), "s"(m.bx), "s"(m.by), "s"(m.avx), "s"(m.avy));
  } else if constexpr (BM == RM_F2 || BM == RM_F2L) {
    asm volatile("" ::"s"(w.s0), "s"(w.s1), "s"(w.f2), "s"(w.f3), "s"(m.rho0), "s"(m.arx), "s"(m.ary), "s"(m.c2),
                 "s"(m.tap_off));
  } else if constexpr (BM == RM_F3) {
    asm volatile("" ::"s"(w.s0), "s"(w.s1), "s"(w.f2), "s"(w.f3), "s"(m.c2), "s"(m.c2eta), "s"(m.c2tau),
                 "s"(m.tap_off));
  } else if constexpr (BM == RM_A1) {
    asm volatile("" ::"s"(w.s0), "s"(w.part), "s"(m.c2), "s"(m.c2eta), "s"(m.c2tau), "s"(m.tap_off),
                 "s"(m.taps), "s"(m.ny), "s"(m.ns), "s"(m.node_off), "s"(m.nodes), "s"(m.scon));
  } else if constexpr (BM == RM_A1L) {
    asm volatile("" ::"s"(w.s0), "s"(w.f2), "s"(w.f3), "s"(m.c2), "s"(m.rho0), "s"(m.arx), "s"(m.ary),
                 "s"(m.tap_off), "s"(m.node_off), "s"(m.nodes));
  } else if constexpr (BM == RM_A2) {
    asm volatile("" ::"s"(w.s0), "s"(w.s1), "s"(w.q), "s"(w.f2), "s"(w.f3), "s"(m.rho0), "s"(m.arx), "s"(m.ary));
  } else {
    asm volatile("" ::"s"(w.s0));
  }
}

template <int CM>
__device__ __forceinline__ void col_args_batch(const Launch& L, int ntile, int chunk, int n) {
  const Medium& m = L.m;
  asm volatile("" ::"s"(ntile), "s"(chunk), "s"(n), "s"(L.nitems), "s"(L.wstride), "s"(m.ny), "s"(m.nxh),
               "s"(m.nt), "s"(m.srt), "s"(m.ct), "s"(m.lsrt), "s"(m.lct), "s"(L.w0.s0), "s"(L.w0.s1), "s"(m.twy),
               "s"(m.twyr), "s"(blockDim.x));
  if constexpr (CM == CM_FRAC) {
    asm volatile("" ::"s"(m.ldis), "s"(m.labs));
  } else if constexpr (CM == CM_GRADP1 || CM == CM_GRADP2) {
    asm volatile("" ::"s"(m.kap), "s"(m.dxp), "s"(m.dyp));
  } else if constexpr (CM == CM_GRADM2 || CM == CM_DIVM) {
    asm volatile("" ::"s"(m.kap), "s"(m.dxm), "s"(m.dym));
  }
}

// ---------------------------------------------------------------- row pass
// Every global load of a pass is issued in one phase at the start: spectra and
// twiddles into LDS, pointwise operands into registers (at most kMaxPer
// elements per thread); the FFT stages then run out of LDS only.
#define FOR_K _Pragma("unroll") for (int k = 0; k < kMaxPer; ++k)
// Load loops skip whole iterations on a block-uniform test and clamp the
// ragged last one (its extra lanes re-read the last element): no per-lane
// branch, so the loads of all iterations issue back to back.
#define FOR_K_LD _Pragma("unroll") for (int k = 0; k < kMaxPer; ++k) if (k * B < tot)

// TG: the FFT stages read their twiddles from the plan's table in global
// memory (L1/L2 resident) instead of a copy staged in LDS.  That takes the
// table load and its LDS writes off a block's critical path, which pays when
// a launch has about one block per CU; with several blocks per CU the LDS
// copy (and the occupancy it costs) is the better trade.
template <int MODE, bool U, int NF, bool TG = false>
__global__ void __launch_bounds__(kMaxThreads)
row_kernel(const Launch L, int ntile, int chunk, int n, int flags) {
  constexpr int BM = MODE & ~(RM_X | RM_FZ);
  constexpr bool FZ = (MODE & RM_FZ) != 0;
  constexpr bool XS = (MODE & RM_X) != 0;
  extern __shared__ float2 lds[];
  if constexpr (U) row_args_batch<BM>(L, ntile, chunk, n, flags);
  int item, tile;
  if (!locate<U>(L, ntile, chunk, item, tile)) return;
  const Medium& M = medium_of<U>(L, item);
  const Work W = U ? shift_work(L.w0, item * L.wstride) : L.items[item].w;
  const IO& X = L.io[item];
  if (n > M.nt - 2) return;  // this problem has finished (uneven batches)
  const int nx = row_len<NF>(M), nxh = row_half<NF>(M), rt = M.rt;
  const int y0 = tile * rt;
  const int B = blockDim.x;
  const int LS = lstride(nx);
  // IP: instances with a compile-time length run their FFT stages in place in
  // one LDS buffer unless they read global twiddles (TG, launches of about
  // one block per CU, where the extra barriers would cost): the freed LDS lets
  // more blocks share a CU.
  constexpr bool IP = NF > 0 && !TG;
  constexpr int NBUF = IP ? 1 : 2;
  float2* bufA = lds;
  float2* bufB = IP ? lds : lds + rt * LS;
  float2* const twl = lds + NBUF * rt * LS;
  const float2* const tw = TG ? static_cast<const float2*>(M.twx) : twl;
  void* tap_base = lds + NBUF * rt * LS + (TG ? 0 : nx);
  const int tot = rt * nx;
  const float dt = M.dt;
  const float rnx = 1.0f / static_cast<float>(nx);
  // row j of element it of the tile, and the offset of grid row y (integer
  // shifts / a constant divide when the instance has a compile-time length)
  auto rowdiv = [&](int it) -> int {
    if constexpr (NF > 0) return int(unsigned(it) / unsigned(NF));
    else return fdiv(it, nx, rnx);
  };
  auto rowoff = [&](int y) -> unsigned {
    if constexpr (NF > 0) return unsigned(y) * unsigned(NF);
    else return mul24(y, nx);
  };
  // RM_X variants: this iterate's slot of the sound-speed sensitivities
  float* const sens = XS ? X.sens + size_t(unsigned(flags) >> kSlotShift) * unsigned(nx * M.ny) : nullptr;

  if constexpr ((BM == RM_F1 || BM == RM_A3) && row_fusable<NF>()) {
    // eq num-vel (RM_F1: v_i = A_i (A_i v_i - dt/rho_i d/dr_i^+ p)) and its
    // transpose (RM_A3) with the update between the two FFTs in registers:
    // butterfly (row j, jj) of the boundary stage holds the row's values at
    // x = jj + q N/R
    constexpr int R = plan_radix(NF, 0), NB = NF / R, MB = fused_slots<NF>();
    const bool first = BM == RM_F1 ? (n == 0) : (n == M.nt - 2);  // the state starts at zero
    float v0x[MB][R], v0y[MB][R], bx[MB][R], by[MB][R], ax[MB][R], ay[MB];
    PairRegs S;
    TwRegs TW;
    fetch_pair<NF>(S, M, W.s0, W.s1, tile);
    if constexpr (!TG) fetch_tw(TW, M.twx, nx);
#pragma unroll
    for (int i = 0; i < MB; ++i) {
      if (wave_base() + i * B < rt * NB) {
        const unsigned it = min(unsigned(threadIdx.x + i * B), unsigned(rt * NB) - 1u);
        const int j = int(it / NB), jj = int(it % NB), y = y0 + j;
        const unsigned base = rowoff(y) + jj;
#pragma unroll
        for (int q = 0; q < R; ++q) {
          v0x[i][q] = W.f0[base + q * NB];
          v0y[i][q] = W.f1[base + q * NB];
          bx[i][q] = M.bx[base + q * NB];
          by[i][q] = M.by[base + q * NB];
          ax[i][q] = M.avx[jj + q * NB];
        }
        ay[i] = M.avy[y];
      }
    }
    put_pair<NF>(S, bufA, M);
    if constexpr (!TG) put_tw(TW, twl, nx);
    __syncthreads();
    auto pw = [&](int i, int j, int jj, float2* v) {
#pragma clang fp contract(off)  // the same rounding fused or not (no cross-path contraction choices)
      const unsigned base = rowoff(y0 + j) + jj;
#pragma unroll
      for (int q = 0; q < R; ++q) {
        const float2 z = v[q];
        if constexpr (BM == RM_F1) {
          const float vx = ax[i][q] * (ax[i][q] * (first ? 0.f : v0x[i][q]) - bx[i][q] * z.x);
          const float vy = ay[i] * (ay[i] * (first ? 0.f : v0y[i][q]) + by[i][q] * z.y);
          W.f0[base + q * NB] = vx;
          W.f1[base + q * NB] = vy;
          v[q] = make_float2(vx, vy);
        } else {
          const float vbx = (first ? 0.f : v0x[i][q]) - z.x;
          const float vby = (first ? 0.f : v0y[i][q]) + z.y;
          W.f0[base + q * NB] = ax[i][q] * ax[i][q] * vbx;
          W.f1[base + q * NB] = ay[i] * ay[i] * vby;
          v[q] = make_float2(-ax[i][q] * bx[i][q] * vbx, -ay[i] * by[i][q] * vby);
        }
      }
    };
    float2* r = fft_fused<NF, IP>(bufA, bufB, rt, tw, pw);
    store_pair_spectra<NF, TG>(r, M, W.s0, W.s1, tile);
  } else if constexpr (BM == RM_F1) {
    // eq num-vel: v_i = A_i (A_i v_i - dt/rho_i d/dr_i^+ p)
    const bool first = (n == 0);  // v^{-1/2} = 0
    float vxo[kMaxPer], vyo[kMaxPer], bx[kMaxPer], by[kMaxPer], ax[kMaxPer], ay[kMaxPer];
    PairRegs S;
    TwRegs TW;
    fetch_pair<NF>(S, M, W.s0, W.s1, tile);
    if constexpr (!TG) fetch_tw(TW, M.twx, nx);
    FOR_K_LD {
      const int it = min(int(threadIdx.x) + k * B, tot - 1);
      {
        const int j = rowdiv(it), x = it - j * nx, y = y0 + j;
        const unsigned idx = rowoff(y) + x;
        vxo[k] = W.f0[idx];
        vyo[k] = W.f1[idx];
        bx[k] = M.bx[idx];
        by[k] = M.by[idx];
        ax[k] = M.avx[x];
        ay[k] = M.avy[y];
      }
    }
    put_pair<NF>(S, bufA, M);
    if constexpr (!TG) put_tw(TW, twl, nx);
    __syncthreads();
    float2* r = fft_any<false, NF, IP>(bufA, bufB, rt, nx, LS, M.radx, M.nstx, tw);
    float2* o = other(r, bufA, bufB);
    // all LDS reads of the loop first: its LDS writes go to the other buffer,
    // which the compiler cannot tell, so an interleaved loop waits per element
    float2 zr[kMaxPer];
    FOR_K {
      const int it = threadIdx.x + k * B;
      if (it < tot) {
        const int j = rowdiv(it), x = it - j * nx;
        zr[k] = r[j * LS + px(x)];
      }
    }
    if constexpr (IP) __syncthreads();  // the loop below writes the buffer just read
    FOR_K {
      const int it = threadIdx.x + k * B;
      if (it < tot) {
#pragma clang fp contract(off)  // the same rounding fused or not (no cross-path contraction choices)
        const int j = rowdiv(it), x = it - j * nx;
        const unsigned idx = rowoff(y0 + j) + x;
        const float2 z = zr[k];
        const float vx = ax[k] * (ax[k] * (first ? 0.f : vxo[k]) - bx[k] * z.x);
        const float vy = ay[k] * (ay[k] * (first ? 0.f : vyo[k]) + by[k] * z.y);
        W.f0[idx] = vx;
        W.f1[idx] = vy;
        o[j * LS + px(x)] = make_float2(vx, vy);
      }
    }
    __syncthreads();
    r = fft_any<false, NF, IP>(o, other(o, bufA, bufB), rt, nx, LS, M.radx, M.nstx, tw);
    store_pair_spectra<NF, TG>(r, M, W.s0, W.s1, tile);
  } else if constexpr (FZ) {
    // RM_FZ instances of the lossy density passes (forward eq num-rho and its
    // transpose) at iterates n >= 1, past the source and the zero initial
    // state: only the fused path is compiled, so the first iterates' code does
    // not set these kernels' register count.  The host launches them only for
    // compile-time lengths whose plan fuses (kernels_row_fused).  Plans whose
    // boundary stage has radix 8 (256, 512) hold one row per work item, the
    // rows 2l and 2l+1 of a pair in adjacent lanes (fft_fused_pairs); radix-4
    // ones (128, 1024) two rows per work item (fft_fused2), which is faster
    // there, and only where the twiddles sit in LDS.
    constexpr bool PAIRS = plan_radix(NF > 0 ? NF : 8, 0) > 4;
    if constexpr (BM == RM_F2 && row_fusable<NF>() && PAIRS) {
      // each row's inverse line in, S and u lines (rows 2l, 2l+1 packed) out
      constexpr int R = plan_radix(NF, 0), NB = NF / R, MB = fused_slots<NF>();
      const int half = rt / 2;
      float rxo[MB][R], ryo[MB][R], r0[MB][R], ax[MB][R], ay[MB];
      PairRegs S;
      TwRegs TW;
      fetch_pair<NF>(S, M, W.s0, W.s1, tile);
      if constexpr (!TG) fetch_tw(TW, M.twx, nx);
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        if (wave_base() + i * B < rt * NB) {
          const unsigned it = min(unsigned(threadIdx.x + i * B), unsigned(rt * NB) - 1u);
          const unsigned p = it >> 1, l = p / NB, jj = p % NB;
          const int y = y0 + 2 * int(l) + int(it & 1u);
          const unsigned base = rowoff(y) + jj;
#pragma unroll
          for (int q = 0; q < R; ++q) {
            rxo[i][q] = W.f2[base + q * NB];
            ryo[i][q] = W.f3[base + q * NB];
            r0[i][q] = M.rho0[base + q * NB];
            ax[i][q] = M.arx[jj + q * NB];
          }
          ay[i] = M.ary[y];
        }
      }
      put_pair<NF>(S, bufA, M);
      if constexpr (!TG) put_tw(TW, twl, nx);
      __syncthreads();
      auto inl = [&](int l, int sd) { return 2 * l + sd; };
      auto outl = [&](int l, int sd) { return sd * half + l; };
      auto pw = [&](int i, int l, int sd, int jj, float2* v, bool active) {
#pragma clang fp contract(off)  // the same rounding fused or not (no cross-path contraction choices)
        const unsigned base = rowoff(y0 + 2 * l + sd) + jj;
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const float ex = v[q].x, ey = -v[q].y;
          const float s = 0.f;
          const float rx = ax[i][q] * (ax[i][q] * rxo[i][q] - dt * r0[i][q] * ex) + s;
          const float ry = ay[i] * (ay[i] * ryo[i][q] - dt * r0[i][q] * ey) + s;
          if (active) {
            W.f2[base + q * NB] = rx;
            W.f3[base + q * NB] = ry;
          }
          const float sum = rx + ry, u = r0[i][q] * (ax[i][q] * ex + ay[i] * ey);
          // row 2l keeps S and sends u; row 2l+1 keeps u and sends S
          const float got = lane_pair_swap(sd ? sum : u);
          v[q] = sd ? make_float2(got, u) : make_float2(sum, got);
        }
      };
      float2* r = fft_fused_pairs<NF, IP>(bufA, bufB, rt, tw, inl, outl, pw);
      store_rowpair_spectra<NF, TG>(r, M, W.s0, tile);
      store_rowpair_spectra<NF, TG>(r + half * LS, M, W.s1, tile);
    } else if constexpr (BM == RM_F2 && row_fusable<NF>() && !TG) {
      // iterates past the source: the update between the two FFTs in
      // registers, rows 2l and 2l+1 of each position together (their S and
      // u values share one complex line each on the output side)
      constexpr int R = plan_radix(NF, 0), NB = NF / R, MB = fused2_slots<NF>();
      const int half = rt / 2;
      float rxa[MB][R], rya[MB][R], r0a[MB][R], rxb[MB][R], ryb[MB][R], r0b[MB][R], ax[MB][R];
      float aya[MB], ayb[MB];
      PairRegs S;
      TwRegs TW;
      fetch_pair<NF>(S, M, W.s0, W.s1, tile);
      if constexpr (!TG) fetch_tw(TW, M.twx, nx);
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        if (wave_base() + i * B < half * NB) {
          const unsigned it = min(unsigned(threadIdx.x + i * B), unsigned(half * NB) - 1u);
          const int l = int(it / NB), jj = int(it % NB), ya = y0 + 2 * l;
          const unsigned ba = rowoff(ya) + jj, bb = ba + nx;
#pragma unroll
          for (int q = 0; q < R; ++q) {
            rxa[i][q] = W.f2[ba + q * NB];
            rya[i][q] = W.f3[ba + q * NB];
            r0a[i][q] = M.rho0[ba + q * NB];
            rxb[i][q] = W.f2[bb + q * NB];
            ryb[i][q] = W.f3[bb + q * NB];
            r0b[i][q] = M.rho0[bb + q * NB];
            ax[i][q] = M.arx[jj + q * NB];
          }
          aya[i] = M.ary[ya];
          ayb[i] = M.ary[ya + 1];
        }
      }
      put_pair<NF>(S, bufA, M);
      if constexpr (!TG) put_tw(TW, twl, nx);
      __syncthreads();
      auto inl = [&](int l, int sd) { return 2 * l + sd; };
      auto outl = [&](int l, int sd) { return sd * half + l; };
      auto pw = [&](int i, int l, int jj, float2* va, float2* vb) {
#pragma clang fp contract(off)  // the same rounding fused or not (no cross-path contraction choices)
        const unsigned ba = rowoff(y0 + 2 * l) + jj, bb = ba + nx;
        const float s = 0.f;
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const float exa = va[q].x, eya = -va[q].y, exb = vb[q].x, eyb = -vb[q].y;
          const float rxA = ax[i][q] * (ax[i][q] * rxa[i][q] - dt * r0a[i][q] * exa) + s;
          const float ryA = aya[i] * (aya[i] * rya[i][q] - dt * r0a[i][q] * eya) + s;
          const float rxB = ax[i][q] * (ax[i][q] * rxb[i][q] - dt * r0b[i][q] * exb) + s;
          const float ryB = ayb[i] * (ayb[i] * ryb[i][q] - dt * r0b[i][q] * eyb) + s;
          W.f2[ba + q * NB] = rxA;
          W.f3[ba + q * NB] = ryA;
          W.f2[bb + q * NB] = rxB;
          W.f3[bb + q * NB] = ryB;
          va[q] = make_float2(rxA + ryA, rxB + ryB);
          vb[q] = make_float2(r0a[i][q] * (ax[i][q] * exa + aya[i] * eya), r0b[i][q] * (ax[i][q] * exb + ayb[i] * eyb));
        }
      };
      float2* r = fft_fused2<NF, IP>(bufA, bufB, rt, tw, inl, outl, pw);
      store_rowpair_spectra<NF, TG>(r, M, W.s0, tile);
      store_rowpair_spectra<NF, TG>(r + half * LS, M, W.s1, tile);
    } else if constexpr (BM == RM_A2 && row_fusable<NF>() && PAIRS) {
      // the eta / tau lines (rows 2l, 2l+1 packed) in, each row's line out
      const bool first = (n == M.nt - 2);
      constexpr int R = plan_radix(NF, 0), NB = NF / R, MB = fused_slots<NF>();
      const int half = rt / 2;
      float qv[MB][R], x0[MB][R], y0v[MB][R], r0[MB][R], ax[MB][R], ay[MB];
      RowPairRegs S0, S1;
      TwRegs TW;
      fetch_rowpair<NF>(S0, M, W.s0, tile);
      fetch_rowpair<NF>(S1, M, W.s1, tile);
      if constexpr (!TG) fetch_tw(TW, M.twx, nx);
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        if (wave_base() + i * B < rt * NB) {
          const unsigned it = min(unsigned(threadIdx.x + i * B), unsigned(rt * NB) - 1u);
          const unsigned p = it >> 1, l = p / NB, jj = p % NB;
          const int y = y0 + 2 * int(l) + int(it & 1u);
          const unsigned base = rowoff(y) + jj;
#pragma unroll
          for (int q = 0; q < R; ++q) {
            qv[i][q] = W.q[base + q * NB];
            x0[i][q] = W.f2[base + q * NB];
            y0v[i][q] = W.f3[base + q * NB];
            r0[i][q] = M.rho0[base + q * NB];
            ax[i][q] = M.arx[jj + q * NB];
          }
          ay[i] = M.ary[y];
        }
      }
      put_rowpair<NF>(S0, bufA, M);
      put_rowpair<NF>(S1, bufA + half * LS, M);
      if constexpr (!TG) put_tw(TW, twl, nx);
      __syncthreads();
      auto inl = [&](int l, int sd) { return sd * half + l; };
      auto outl = [&](int l, int sd) { return 2 * l + sd; };
      auto pw = [&](int i, int l, int sd, int jj, float2* v, bool active) {
#pragma clang fp contract(off)  // the same rounding fused or not (no cross-path contraction choices)
        const unsigned base = rowoff(y0 + 2 * l + sd) + jj;
#pragma unroll
        for (int q = 0; q < R; ++q) {
          // row 2l holds the eta line (yd of rows 2l, 2l+1), row 2l+1 the tau
          // line (ya of rows 2l, 2l+1): each sends the value the other's row needs
          const float got = lane_pair_swap(sd ? v[q].x : -v[q].y);
          const float yd = sd ? got : v[q].x, ya = sd ? -v[q].y : got;
          const float sb = qv[i][q] - yd;
          const float rbx = (first ? 0.f : x0[i][q]) + sb, rby = (first ? 0.f : y0v[i][q]) + sb;
          v[q] = make_float2(r0[i][q] * ax[i][q] * (ya - dt * rbx), r0[i][q] * ay[i] * (ya - dt * rby));
          if (active) {
            W.f2[base + q * NB] = ax[i][q] * ax[i][q] * rbx;
            W.f3[base + q * NB] = ay[i] * ay[i] * rby;
          }
        }
      };
      float2* r = fft_fused_pairs<NF, IP>(bufA, bufB, rt, tw, inl, outl, pw);
      store_pair_spectra<NF, TG>(r, M, W.s0, W.s1, tile);
    } else if constexpr (BM == RM_A2 && row_fusable<NF>() && !TG) {
      const bool first = (n == M.nt - 2);
      // the update between the two FFTs in registers: rows 2l and 2l+1 of
      // each position together (they share the input lines)
      constexpr int R = plan_radix(NF, 0), NB = NF / R, MB = fused2_slots<NF>();
      const int half = rt / 2;
      float qa[MB][R], xa[MB][R], ya0[MB][R], r0a[MB][R], qb[MB][R], xb[MB][R], yb0[MB][R], r0b[MB][R];
      float ax[MB][R], aya[MB], ayb[MB];
      RowPairRegs S0, S1;
      TwRegs TW;
      fetch_rowpair<NF>(S0, M, W.s0, tile);
      fetch_rowpair<NF>(S1, M, W.s1, tile);
      if constexpr (!TG) fetch_tw(TW, M.twx, nx);
#pragma unroll
      for (int i = 0; i < MB; ++i) {
        if (wave_base() + i * B < half * NB) {
          const unsigned it = min(unsigned(threadIdx.x + i * B), unsigned(half * NB) - 1u);
          const int l = int(it / NB), jj = int(it % NB), y = y0 + 2 * l;
          const unsigned ba = rowoff(y) + jj, bb = ba + nx;
#pragma unroll
          for (int q = 0; q < R; ++q) {
            qa[i][q] = W.q[ba + q * NB];
            xa[i][q] = W.f2[ba + q * NB];
            ya0[i][q] = W.f3[ba + q * NB];
            r0a[i][q] = M.rho0[ba + q * NB];
            qb[i][q] = W.q[bb + q * NB];
            xb[i][q] = W.f2[bb + q * NB];
            yb0[i][q] = W.f3[bb + q * NB];
            r0b[i][q] = M.rho0[bb + q * NB];
            ax[i][q] = M.arx[jj + q * NB];
          }
          aya[i] = M.ary[y];
          ayb[i] = M.ary[y + 1];
        }
      }
      put_rowpair<NF>(S0, bufA, M);
      put_rowpair<NF>(S1, bufA + half * LS, M);
      if constexpr (!TG) put_tw(TW, twl, nx);
      __syncthreads();
      auto inl = [&](int l, int sd) { return sd * half + l; };
      auto outl = [&](int l, int sd) { return 2 * l + sd; };
      auto pw = [&](int i, int l, int jj, float2* va, float2* vb) {
#pragma clang fp contract(off)  // the same rounding fused or not (no cross-path contraction choices)
        const unsigned ba = rowoff(y0 + 2 * l) + jj, bb = ba + nx;
#pragma unroll
        for (int q = 0; q < R; ++q) {
          // rows 2l and 2l+1 of the (conjugated) inverse transforms
          const float yda = va[q].x, ydb = -va[q].y, yaa = vb[q].x, yab = -vb[q].y;
          const float sba = qa[i][q] - yda, sbb = qb[i][q] - ydb;
          const float rbxa = (first ? 0.f : xa[i][q]) + sba, rbya = (first ? 0.f : ya0[i][q]) + sba;
          const float rbxb = (first ? 0.f : xb[i][q]) + sbb, rbyb = (first ? 0.f : yb0[i][q]) + sbb;
          va[q] = make_float2(r0a[i][q] * ax[i][q] * (yaa - dt * rbxa), r0a[i][q] * aya[i] * (yaa - dt * rbya));
          vb[q] = make_float2(r0b[i][q] * ax[i][q] * (yab - dt * rbxb), r0b[i][q] * ayb[i] * (yab - dt * rbyb));
          W.f2[ba + q * NB] = ax[i][q] * ax[i][q] * rbxa;
          W.f3[ba + q * NB] = aya[i] * aya[i] * rbya;
          W.f2[bb + q * NB] = ax[i][q] * ax[i][q] * rbxb;
          W.f3[bb + q * NB] = ayb[i] * ayb[i] * rbyb;
        }
      };
      float2* r = fft_fused2<NF, IP>(bufA, bufB, rt, tw, inl, outl, pw);
      store_pair_spectra<NF, TG>(r, M, W.s0, W.s1, tile);
    }
  } else if constexpr (BM == RM_F2 || BM == RM_F2L) {
    // eq num-rho with the additive source of eq s1 (dt s = p0 / (2 d c^2), d = 2)
    const bool skip = (n == -1);  // v^{-1/2} = 0 and rho^{-1} = 0
    const bool inject = (n <= 0);
    float rxo[kMaxPer], ryo[kMaxPer], r0[kMaxPer], ax[kMaxPer], ay[kMaxPer], src[kMaxPer], c2[kMaxPer];
    PairRegs S;
    TwRegs TW;
    TapStage T{};
    if constexpr (BM == RM_F2L) taps_range(T, M, tap_base, y0, rt);
    if (!skip) fetch_pair<NF>(S, M, W.s0, W.s1, tile);
    if constexpr (!TG) fetch_tw(TW, M.twx, nx);
    FOR_K_LD {
      const int it = min(int(threadIdx.x) + k * B, tot - 1);
      {
        const int j = rowdiv(it), x = it - j * nx, y = y0 + j;
        const unsigned idx = rowoff(y) + x;
        rxo[k] = W.f2[idx];
        ryo[k] = W.f3[idx];
        r0[k] = M.rho0[idx];
        ax[k] = M.arx[x];
        ay[k] = M.ary[y];
        if constexpr (BM == RM_F2L) c2[k] = M.c2[idx];
      }
    }
    if (inject) {  // first two iterates only (kept apart so the loads above issue back to back)
      FOR_K_LD {
        const int it = min(int(threadIdx.x) + k * B, tot - 1);
        {
          const int j = rowdiv(it), x = it - j * nx;
          const unsigned idx = rowoff(y0 + j) + x;
          if constexpr (BM != RM_F2L) c2[k] = M.c2[idx];
          src[k] = X.in[idx];
        }
      }
    }
    if (!skip) put_pair<NF>(S, bufA, M);
    if constexpr (!TG) put_tw(TW, twl, nx);
    __syncthreads();
    if constexpr (BM == RM_F2L) taps_fetch(T, M, nullptr, 0);
    float2* r = nullptr;
    float2* o = bufA;
    if (!skip) {
      r = fft_any<false, NF, IP>(bufA, bufB, rt, nx, LS, M.radx, M.nstx, tw);
      o = other(r, bufA, bufB);
    }
    float2 zr[kMaxPer];
    if (!skip) {
      FOR_K {
        const int it = threadIdx.x + k * B;
        if (it < tot) {
          const int j = rowdiv(it), x = it - j * nx;
          zr[k] = r[j * LS + px(x)];
        }
      }
    }
    if constexpr (IP) __syncthreads();  // the loop below writes the buffer just read
    FOR_K {
      const int it = threadIdx.x + k * B;
      if (it < tot) {
#pragma clang fp contract(off)  // the same rounding fused or not (no cross-path contraction choices)
        const int j = rowdiv(it), x = it - j * nx;
        const unsigned idx = rowoff(y0 + j) + x;
        float ex = 0.f, ey = 0.f;
        if (!skip) {
          const float2 z = zr[k];
          ex = z.x;
          ey = -z.y;
        } else {
          W.f0[idx] = 0.f;  // the state z_0 holds v^{-1/2} = 0
          W.f1[idx] = 0.f;
        }
        const float s = inject ? src[k] * (0.25f / c2[k]) : 0.f;
        const float rx = ax[k] * (ax[k] * (skip ? 0.f : rxo[k]) - dt * r0[k] * ex) + s;
        const float ry = ay[k] * (ay[k] * (skip ? 0.f : ryo[k]) - dt * r0[k] * ey) + s;
        W.f2[idx] = rx;
        W.f3[idx] = ry;
        if constexpr (BM == RM_F2) {
          // S = sum_i rho_i and u = rho0 sum_i A_i d/dr_i^- v_i feed eq num-p.
          // Each is transformed with its own rows paired (S and u differ by
          // orders of magnitude, so they must not share one complex FFT).
          pcomp(o, j, x, nx) = rx + ry;
          pcomp(o + (rt / 2) * LS, j, x, nx) = r0[k] * (ax[k] * ex + ay[k] * ey);
        } else {
          const float p = c2[k] * (rx + ry);
          pcomp(o, j, x, nx) = p;
          if (flags & FL_STORE_P) W.q[idx] = p;
          if constexpr (XS) sens[idx] = 2.f * p * rsqrtf(c2[k]);  // d(c^2 S)/dc
        }
      }
    }
    if constexpr (BM == RM_F2L) taps_put(T, false);
    __syncthreads();
    if constexpr (BM == RM_F2) {
      r = fft_any<false, NF, IP>(o, other(o, bufA, bufB), rt, nx, LS, M.radx, M.nstx, tw);
      store_rowpair_spectra<NF, TG>(r, M, W.s0, tile);
      store_rowpair_spectra<NF, TG>(r + (rt / 2) * LS, M, W.s1, tile);
    } else {
      if (!(flags & FL_NO_SENSORS)) sensor_partials(M, T, o, y0, W.part, n + 1);
      r = fft_any<false, NF, IP>(o, other(o, bufA, bufB), rt / 2, nx, LS, M.radx, M.nstx, tw);
      store_rowpair_spectra<NF, TG>(r, M, W.s0, tile);
    }
  } else if constexpr (BM == RM_F3) {
    // eq num-p: p = c^2 (S - eta Y_dis S + tau Y_abs u)
    float rxo[kMaxPer], ryo[kMaxPer], c2[kMaxPer], ce[kMaxPer], ctau[kMaxPer];
    TapStage T;
    taps_range(T, M, tap_base, y0, rt);
    RowPairRegs S0, S1;
    TwRegs TW;
    fetch_rowpair<NF>(S0, M, W.s0, tile);
    fetch_rowpair<NF>(S1, M, W.s1, tile);
    if constexpr (!TG) fetch_tw(TW, M.twx, nx);
    FOR_K_LD {
      const int it = min(int(threadIdx.x) + k * B, tot - 1);
      {
        const int j = rowdiv(it), x = it - j * nx;
        const unsigned idx = rowoff(y0 + j) + x;
        rxo[k] = W.f2[idx];
        ryo[k] = W.f3[idx];
        c2[k] = M.c2[idx];
        ce[k] = M.c2eta[idx];
        ctau[k] = M.c2tau[idx];
      }
    }
    put_rowpair<NF>(S0, bufA, M);
    put_rowpair<NF>(S1, bufA + (rt / 2) * LS, M);
    if constexpr (!TG) put_tw(TW, twl, nx);
    __syncthreads();
    taps_fetch(T, M, nullptr, 0);
    float2* r = fft_any<false, NF, IP>(bufA, bufB, rt, nx, LS, M.radx, M.nstx, tw);
    float2* o = other(r, bufA, bufB);
    float ysr[kMaxPer], yur[kMaxPer];
    FOR_K {
      const int it = threadIdx.x + k * B;
      if (it < tot) {
        const int j = rowdiv(it), x = it - j * nx;
        ysr[k] = rowpair_val(r, j, x, nx);
        yur[k] = rowpair_val(r + (rt / 2) * LS, j, x, nx);
      }
    }
    if constexpr (IP) __syncthreads();  // the loop below writes the buffer just read
    FOR_K {
      const int it = threadIdx.x + k * B;
      if (it < tot) {
        const int j = rowdiv(it), x = it - j * nx;
        const float ys = ysr[k], yu = yur[k];
        const float p = c2[k] * (rxo[k] + ryo[k]) - ce[k] * ys + ctau[k] * yu;
        pcomp(o, j, x, nx) = p;
        const unsigned idx = rowoff(y0 + j) + x;
        if (flags & FL_STORE_P) W.q[idx] = p;
        if constexpr (XS) {
          // eq Twelve: c^2 eta ~ c^(y+2) and c^2 tau ~ c^(y+1), so each term of
          // eq num-p differentiates to its power over c
          const float S = rxo[k] + ryo[k];
          sens[idx] = (2.f * c2[k] * S - (M.ypow + 2.f) * ce[k] * ys + (M.ypow + 1.f) * ctau[k] * yu) * rsqrtf(c2[k]);
        }
      }
    }
    taps_put(T, false);
    __syncthreads();
    if (!(flags & FL_NO_SENSORS)) sensor_partials(M, T, o, y0, W.part, n + 1);
    r = fft_any<false, NF, IP>(o, other(o, bufA, bufB), rt / 2, nx, LS, M.radx, M.nstx, tw);
    store_rowpair_spectra<NF, TG>(r, M, W.s0, tile);
  } else if constexpr (BM == RM_A1 || BM == RM_A1L) {
    // transpose of eqs num-m and num-p: p* += M^T r_{n+1}; q = c^2 p*
    const bool first = (n == M.nt - 2);
    const int half = rt / 2;
    float c2[kMaxPer], ce[kMaxPer], ctau[kMaxPer], rbx0[kMaxPer], rby0[kMaxPer], r0[kMaxPer];
    float ax[kMaxPer], ay[kMaxPer], gacc[kMaxPer];
    TapStage T;
    taps_range(T, M, tap_base, y0, rt, true);
    RowPairRegs S0;
    TwRegs TW;
    if (!first) fetch_rowpair<NF>(S0, M, W.s0, tile);
    if constexpr (!TG) fetch_tw(TW, M.twx, nx);
    FOR_K_LD {
      const int it = min(int(threadIdx.x) + k * B, tot - 1);
      {
        const int j = rowdiv(it), x = it - j * nx, y = y0 + j;
        const unsigned idx = rowoff(y) + x;
        c2[k] = M.c2[idx];
        if constexpr (BM == RM_A1) {
          ce[k] = M.c2eta[idx];
          ctau[k] = M.c2tau[idx];
        } else {
          rbx0[k] = W.f2[idx];
          rby0[k] = W.f3[idx];
          r0[k] = M.rho0[idx];
          ax[k] = M.arx[x];
          ay[k] = M.ary[y];
        }
      }
    }
    float sv[kMaxPer];
    double gprev[kMaxPer];
    if constexpr (XS) {
      FOR_K_LD {
        const int it = min(int(threadIdx.x) + k * B, tot - 1);
        {
          const int j = rowdiv(it), x = it - j * nx;
          const unsigned idx = rowoff(y0 + j) + x;
          sv[k] = sens[idx];
          gprev[k] = first ? 0.0 : X.gc[idx];
        }
      }
    }
    if constexpr (BM == RM_A1L) {
      if (n == -1 && M.nt >= 2) {  // the gradient accumulated at n = 0
        FOR_K_LD {
          const int it = min(int(threadIdx.x) + k * B, tot - 1);
          {
            const int j = rowdiv(it), x = it - j * nx;
            gacc[k] = X.out[rowoff(y0 + j) + x];
          }
        }
      }
    }
    if (!first) put_rowpair<NF>(S0, bufA, M);
    if constexpr (!TG) put_tw(TW, twl, nx);
    __syncthreads();
    taps_fetch(T, M, W.part, n + 1);
    nodes_fetch(T, M);
    float2* r = bufA;
    if (!first) {
      r = fft_any<false, NF, IP>(bufA, bufB, half, nx, LS, M.radx, M.nstx, tw);
      // p* = -(grad_x^- g_x + grad_y^- g_y): negate the (conjugated) inverse
#pragma unroll 4
      for (int it = threadIdx.x; it < half * LS; it += B) {
        const float2 z = r[it];
        r[it] = make_float2(-z.x, z.y);
      }
    } else {
      for (int it = threadIdx.x; it < half * LS; it += B) r[it] = make_float2(0.f, 0.f);
    }
    taps_put(T, true);
    __syncthreads();
    sensor_scatter(M, T, r, y0, W.part, n + 1);
    __syncthreads();
    float2* o = other(r, bufA, bufB);
    float pbr[kMaxPer];
    FOR_K {
      const int it = threadIdx.x + k * B;
      if (it < tot) {
        const int j = rowdiv(it), x = it - j * nx;
        pbr[k] = pcomp(r, j, x, nx);
      }
    }
    if constexpr (IP) __syncthreads();  // the loop below writes the buffer just read
    FOR_K {
      const int it = threadIdx.x + k * B;
      if (it < tot) {
        const int j = rowdiv(it), x = it - j * nx;
        const unsigned idx = rowoff(y0 + j) + x;
        const float pb = pbr[k];
        if constexpr (XS) X.gc[idx] = gprev[k] + double(pb) * double(sv[k]);
        if constexpr (BM == RM_A1) {
          // eta q and tau q, each with its own rows paired (see RM_F2)
          W.q[idx] = c2[k] * pb;
          pcomp(o, j, x, nx) = ce[k] * pb;
          pcomp(o + half * LS, j, x, nx) = ctau[k] * pb;
        } else {
          // lossless: S* = q, u* = 0, then the transposed mass update
          const float q = c2[k] * pb;
          const float rbx = (first ? 0.f : rbx0[k]) + q, rby = (first ? 0.f : rby0[k]) + q;
          if (n == 0) X.out[idx] = rbx + rby;
          if (n == -1) {
            X.out[idx] = (rbx + rby + (M.nt >= 2 ? gacc[k] : 0.f)) * (0.25f / c2[k]);
          } else {
            o[j * LS + px(x)] = make_float2(-dt * r0[k] * ax[k] * rbx, -dt * r0[k] * ay[k] * rby);
            W.f2[idx] = ax[k] * ax[k] * rbx;
            W.f3[idx] = ay[k] * ay[k] * rby;
          }
        }
      }
    }
    __syncthreads();
    if constexpr (BM == RM_A1) {
      r = fft_any<false, NF, IP>(o, other(o, bufA, bufB), rt, nx, LS, M.radx, M.nstx, tw);
      store_rowpair_spectra<NF, TG>(r, M, W.s0, tile);
      store_rowpair_spectra<NF, TG>(r + half * LS, M, W.s1, tile);
    } else if (n != -1) {
      r = fft_any<false, NF, IP>(o, other(o, bufA, bufB), rt, nx, LS, M.radx, M.nstx, tw);
      store_pair_spectra<NF, TG>(r, M, W.s0, W.s1, tile);
    }
  } else if constexpr (BM == RM_A2) {
    // transpose of the mass update and of the Y terms of eq num-p
    const bool first = (n == M.nt - 2);
    float qv[kMaxPer], rbx0[kMaxPer], rby0[kMaxPer], r0[kMaxPer], ax[kMaxPer], ay[kMaxPer];
    float c2[kMaxPer], gacc[kMaxPer];
    RowPairRegs S0, S1;
    TwRegs TW;
    fetch_rowpair<NF>(S0, M, W.s0, tile);
    fetch_rowpair<NF>(S1, M, W.s1, tile);
    if constexpr (!TG) fetch_tw(TW, M.twx, nx);
    FOR_K_LD {
      const int it = min(int(threadIdx.x) + k * B, tot - 1);
      {
        const int j = rowdiv(it), x = it - j * nx, y = y0 + j;
        const unsigned idx = rowoff(y) + x;
        qv[k] = W.q[idx];
        rbx0[k] = W.f2[idx];
        rby0[k] = W.f3[idx];
        r0[k] = M.rho0[idx];
        ax[k] = M.arx[x];
        ay[k] = M.ary[y];
      }
    }
    if (n == -1) {  // the last iterate: gradient scaling and the sum accumulated at n = 0
      FOR_K_LD {
        const int it = min(int(threadIdx.x) + k * B, tot - 1);
        {
          const int j = rowdiv(it), x = it - j * nx;
          const unsigned idx = rowoff(y0 + j) + x;
          c2[k] = M.c2[idx];
          gacc[k] = M.nt >= 2 ? X.out[idx] : 0.f;
        }
      }
    }
    put_rowpair<NF>(S0, bufA, M);
    put_rowpair<NF>(S1, bufA + (rt / 2) * LS, M);
    if constexpr (!TG) put_tw(TW, twl, nx);
    __syncthreads();
    float2* r = fft_any<false, NF, IP>(bufA, bufB, rt, nx, LS, M.radx, M.nstx, tw);
    float2* o = other(r, bufA, bufB);
    float ydr[kMaxPer], yar[kMaxPer];
    FOR_K {
      const int it = threadIdx.x + k * B;
      if (it < tot) {
        const int j = rowdiv(it), x = it - j * nx;
        ydr[k] = rowpair_val(r, j, x, nx);
        yar[k] = rowpair_val(r + (rt / 2) * LS, j, x, nx);
      }
    }
    if constexpr (IP) __syncthreads();  // the loop below writes the buffer just read
    FOR_K {
      const int it = threadIdx.x + k * B;
      if (it < tot) {
#pragma clang fp contract(off)  // the same rounding fused or not (no cross-path contraction choices)
        const int j = rowdiv(it), x = it - j * nx;
        const unsigned idx = rowoff(y0 + j) + x;
        const float yd = ydr[k], ya = yar[k];
        const float sb = qv[k] - yd;
        const float rbx = (first ? 0.f : rbx0[k]) + sb, rby = (first ? 0.f : rby0[k]) + sb;
        if (n == 0) X.out[idx] = rbx + rby;
        if (n == -1) {
          X.out[idx] = (rbx + rby + gacc[k]) * (0.25f / c2[k]);
        } else {
          o[j * LS + px(x)] = make_float2(r0[k] * ax[k] * (ya - dt * rbx), r0[k] * ay[k] * (ya - dt * rby));
          W.f2[idx] = ax[k] * ax[k] * rbx;
          W.f3[idx] = ay[k] * ay[k] * rby;
        }
      }
    }
    __syncthreads();
    if (n != -1) {
      r = fft_any<false, NF, IP>(o, other(o, bufA, bufB), rt, nx, LS, M.radx, M.nstx, tw);
      store_pair_spectra<NF, TG>(r, M, W.s0, W.s1, tile);
    }
  } else if constexpr (BM == RM_A3) {
    // transpose of eq num-vel
    const bool first = (n == M.nt - 2);
    float vbx0[kMaxPer], vby0[kMaxPer], bx[kMaxPer], by[kMaxPer], ax[kMaxPer], ay[kMaxPer];
    PairRegs S;
    TwRegs TW;
    fetch_pair<NF>(S, M, W.s0, W.s1, tile);
    if constexpr (!TG) fetch_tw(TW, M.twx, nx);
    FOR_K_LD {
      const int it = min(int(threadIdx.x) + k * B, tot - 1);
      {
        const int j = rowdiv(it), x = it - j * nx, y = y0 + j;
        const unsigned idx = rowoff(y) + x;
        vbx0[k] = W.f0[idx];
        vby0[k] = W.f1[idx];
        bx[k] = M.bx[idx];
        by[k] = M.by[idx];
        ax[k] = M.avx[x];
        ay[k] = M.avy[y];
      }
    }
    put_pair<NF>(S, bufA, M);
    if constexpr (!TG) put_tw(TW, twl, nx);
    __syncthreads();
    float2* r = fft_any<false, NF, IP>(bufA, bufB, rt, nx, LS, M.radx, M.nstx, tw);
    float2* o = other(r, bufA, bufB);
    float2 zr[kMaxPer];
    FOR_K {
      const int it = threadIdx.x + k * B;
      if (it < tot) {
        const int j = rowdiv(it), x = it - j * nx;
        zr[k] = r[j * LS + px(x)];
      }
    }
    if constexpr (IP) __syncthreads();  // the loop below writes the buffer just read
    FOR_K {
      const int it = threadIdx.x + k * B;
      if (it < tot) {
#pragma clang fp contract(off)  // the same rounding fused or not (no cross-path contraction choices)
        const int j = rowdiv(it), x = it - j * nx;
        const unsigned idx = rowoff(y0 + j) + x;
        const float2 z = zr[k];
        const float vbx = (first ? 0.f : vbx0[k]) - z.x;
        const float vby = (first ? 0.f : vby0[k]) + z.y;
        o[j * LS + px(x)] = make_float2(-ax[k] * bx[k] * vbx, -ay[k] * by[k] * vby);
        W.f0[idx] = ax[k] * ax[k] * vbx;
        W.f1[idx] = ay[k] * ay[k] * vby;
      }
    }
    __syncthreads();
    r = fft_any<false, NF, IP>(o, other(o, bufA, bufB), rt, nx, LS, M.radx, M.nstx, tw);
    store_pair_spectra<NF, TG>(r, M, W.s0, W.s1, tile);
  } else if constexpr (BM == RM_FWD1) {
    const float* src = X.in;
    TwRegs TW;
    float v[kMaxPer];
    if constexpr (!TG) fetch_tw(TW, M.twx, nx);
    FOR_K_LD {
      const int it = min(int(threadIdx.x) + k * B, tot - 1);
      {
        const int j = rowdiv(it), x = it - j * nx;
        v[k] = src[rowoff(y0 + j) + x];
      }
    }
    FOR_K {
      const int it = threadIdx.x + k * B;
      if (it < tot) {
        const int j = rowdiv(it), x = it - j * nx;
        pcomp(bufA, j, x, nx) = v[k];
      }
    }
    if constexpr (!TG) put_tw(TW, twl, nx);
    __syncthreads();
    float2* r = fft_any<false, NF, IP>(bufA, bufB, rt / 2, nx, LS, M.radx, M.nstx, tw);
    store_rowpair_spectra<NF, TG>(r, M, W.s0, tile);
  } else if constexpr (BM == RM_INV1) {
    RowPairRegs S0;
    TwRegs TW;
    fetch_rowpair<NF>(S0, M, W.s0, tile);
    if constexpr (!TG) fetch_tw(TW, M.twx, nx);
    put_rowpair<NF>(S0, bufA, M);
    if constexpr (!TG) put_tw(TW, twl, nx);
    __syncthreads();
    float2* r = fft_any<false, NF, IP>(bufA, bufB, rt / 2, nx, LS, M.radx, M.nstx, tw);
    float* dst = X.out;
#pragma unroll 4
    for (int it = threadIdx.x; it < tot; it += B) {
      const int j = rowdiv(it), x = it - j * nx;
      dst[rowoff(y0 + j) + x] = rowpair_val(r, j, x, nx);
    }
  }
}

// ---------------------------------------------------------------- column pass
// Multipliers of a launch are either the staggered gradients (kappa times a
// 1-D symbol in x or y) or the fractional-Laplacian tables; the values a
// thread needs are prefetched into registers in the load phase.
struct MultPre {
  float a, b;     // table A / B at (kx, ky): kappa (or Y_dis) and Y_abs
  float an, bn;   // the same at the Nyquist column (packed column 0 only)
  float2 sx, sxn; // x symbol at kx and at the Nyquist column
  float2 sy;      // y symbol at ky
};

__device__ __forceinline__ float2 mult_of(int code, const MultPre& P, bool nyq) {
  switch (code) {
    case MC_DXP:
    case MC_DXM: return cscale(nyq ? P.sxn : P.sx, nyq ? P.an : P.a);
    case MC_DYP:
    case MC_DYM: return cscale(P.sy, nyq ? P.an : P.a);
    case MC_LDIS: return make_float2(nyq ? P.an : P.a, 0.f);
    case MC_LABS: return make_float2(nyq ? P.bn : P.b, 0.f);
    default: return make_float2(0.f, 0.f);
  }
}

// Column-pass kinds: multiplier codes (out_o = sum_i M[o][i] in_i), inputs, outputs.
__device__ constexpr int kColCode[kColModes] = {
    mpack(MC_DXP, 0, MC_DYP, 0),    // CM_GRADP1: d/dx^+ p, d/dy^+ p
    mpack(MC_DXM, 0, 0, MC_DYM),    // CM_GRADM2: d/dx^- v_x, d/dy^- v_y
    mpack(MC_LDIS, 0, 0, MC_LABS),  // CM_FRAC:   Y_dis S, Y_abs u
    mpack(MC_DXP, 0, 0, MC_DYP),    // CM_GRADP2: d/dx^+ e_x, d/dy^+ e_y
    mpack(MC_DXM, MC_DYM, 0, 0),    // CM_DIVM:   d/dx^- g_x + d/dy^- g_y
    0};                             // CM_APPLY:  one operator given at launch
__device__ constexpr int kColIn[kColModes] = {1, 2, 2, 2, 2, 1};
__device__ constexpr int kColOut[kColModes] = {2, 2, 2, 2, 1, 1};

// Column pass for any supported line length (runtime or compile-time FFT
// plan): the tile goes through LDS between every phase.
template <int CM, int NF, bool TG>
__device__ __forceinline__ void col_generic(const Medium& M, const Work& W, int tile, int mcode, float2* lds) {
  constexpr int nin = kColIn[CM], nout = kColOut[CM];
  const int ny = M.ny, nxh = M.nxh, ct = M.ct, ls = col_lstride(ny);
  const int c0 = tile * ct;
  const int B = blockDim.x;
  const int nsl = 2;
  float2* bufA = lds;
  float2* bufB = lds + nsl * ct * ls;
  float2* const twl = lds + 2 * nsl * ct * ls;
  const float2* const tw = TG ? static_cast<const float2*>(M.twy) : twl;
  // which tables this launch uses
  int xcode = 0, ycode = 0;
  bool frac = false, labs = false;
  for (int e = 0; e < 4; ++e) {
    const int c = (mcode >> (4 * e)) & 15;
    if (c == MC_DXP || c == MC_DXM) xcode = c;
    if (c == MC_DYP || c == MC_DYM) ycode = c;
    if (c == MC_LDIS) frac = true;
    if (c == MC_LABS) { frac = true; labs = true; }
  }
  const float* tabA = frac ? M.ldis : M.kap;
  const float2* symx = xcode == MC_DXP ? M.dxp : M.dxm;
  const float2* symy = ycode == MC_DYP ? M.dyp : M.dym;
  // load phase: the tile (transposed into lines), twiddles, multiplier values
  // memory order: field, tile row ty, element (iy, c) of the srt x ct tile
  const float rny = 1.0f / static_cast<float>(ny);
  const int rc = M.srt * ct;
  // (a tile holds nin*ct*ny <= nin*kColPer*B elements: all loads are issued
  // into registers before the first LDS write)
  constexpr int kIt = nin * kColPer;
  const unsigned ncol = unsigned(ct) * ny, ntot = nin * ncol;     // elements per field / tile
  const unsigned rowstep = unsigned(nxh) * M.srt, tbase = unsigned(tile) * rc;  // tile row ty at ty * rowstep
  const int lsh = M.lsrt + M.lct;
  float2 tv[kIt];
#pragma unroll
  for (int k = 0; k < kIt; ++k) {
    const unsigned it = threadIdx.x + k * B;
    if (it < ntot) {
      const bool f = it >= ncol;
      const unsigned rem = f ? it - ncol : it;
      tv[k] = (f ? W.s1 : W.s0)[mul24(rem >> lsh, rowstep) + tbase + (rem & (rc - 1))];
    }
  }
  TwRegsK<kColPer> TW;  // ny <= kColPer * B
  if constexpr (!TG) fetch_tw(TW, M.twy, ny);
  const int tot = ct * ny;
  MultPre P[kColPer];
#pragma unroll
  for (int k = 0; k < kColPer; ++k) {
    const int it = threadIdx.x + k * B;
    if (it < tot) {
      const int c = ct == 1 ? 0 : fdiv(it, ny, rny), ky = it - c * ny, kx = c0 + c;
      const unsigned t = mul24(kx, ny) + ky, tn = mul24(nxh, ny) + ky;   // tables are [kx][ky]
      MultPre& p = P[k];
      p.a = tabA[t];
      p.b = labs ? M.labs[t] : 0.f;
      p.sx = xcode ? symx[kx] : make_float2(0.f, 0.f);
      p.sy = ycode ? symy[ky] : make_float2(0.f, 0.f);
      if (kx == 0) {
        p.an = tabA[tn];
        p.bn = labs ? M.labs[tn] : 0.f;
        p.sxn = xcode ? symx[nxh] : make_float2(0.f, 0.f);
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kIt; ++k) {
    const unsigned it = threadIdx.x + k * B;
    if (it < ntot) {
      const bool f = it >= ncol;
      const unsigned rem = f ? it - ncol : it, w = rem & (rc - 1);
      const unsigned ky = ((rem >> lsh) << M.lsrt) + (w >> M.lct), c = w & (ct - 1);
      bufA[mul24((f ? ct : 0) + c, ls) + px(ky)] = tv[k];
    }
  }
  if constexpr (!TG) put_tw(TW, twl, ny);
  __syncthreads();
  float2* r = fft_any<true, NF>(bufA, bufB, nin * ct, ny, ls, M.rady, M.nsty, tw);
  float2* o = other(r, bufA, bufB);
#pragma unroll
  for (int k = 0; k < kColPer; ++k) {
    const int it = threadIdx.x + k * B;
    if (it < tot) {
      const int c = ct == 1 ? 0 : fdiv(it, ny, rny), ky = it - c * ny;
      const int kx = c0 + c;
      const MultPre& p = P[k];
      // (loops over fields have compile-time bounds so the arrays stay in registers)
      if (kx == 0) {
        // packed column: DC (real part) and Nyquist (imaginary part) columns
        const int km = ky ? ny - ky : 0;
        float2 f0[2], fn[2];
#pragma unroll
        for (int f = 0; f < 2; ++f) {
          if (f < nin) {
            const float2 z = r[mul24(f * ct + c, ls) + px(ky)], zm = cconj(r[mul24(f * ct + c, ls) + px(km)]);
            f0[f] = cscale(cadd(z, zm), 0.5f);
            fn[f] = mul_mi(cscale(csub(z, zm), 0.5f));
          } else {
            f0[f] = fn[f] = make_float2(0.f, 0.f);
          }
        }
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          if (q < nout) {
            float2 g0 = make_float2(0.f, 0.f), gn = make_float2(0.f, 0.f);
#pragma unroll
            for (int f = 0; f < 2; ++f) {
              const int code = (mcode >> (4 * (2 * q + f))) & 15;
              if (code) {
                g0 = cadd(g0, cmul(mult_of(code, p, false), f0[f]));
                gn = cadd(gn, cmul(mult_of(code, p, true), fn[f]));
              }
            }
            // W = G0 + i GN, stored conjugated for the inverse transform
            o[mul24(q * ct + c, ls) + px(ky)] = cconj(make_float2(g0.x - gn.y, g0.y + gn.x));
          }
        }
      } else {
        float2 in[2];
#pragma unroll
        for (int f = 0; f < 2; ++f) in[f] = f < nin ? r[mul24(f * ct + c, ls) + px(ky)] : make_float2(0.f, 0.f);
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          if (q < nout) {
            float2 acc = make_float2(0.f, 0.f);
#pragma unroll
            for (int f = 0; f < 2; ++f) {
              const int code = (mcode >> (4 * (2 * q + f))) & 15;
              if (code) acc = cadd(acc, cmul(mult_of(code, p, false), in[f]));
            }
            o[mul24(q * ct + c, ls) + px(ky)] = cconj(acc);
          }
        }
      }
    }
  }
  __syncthreads();
  r = fft_any<true, NF>(o, other(o, bufA, bufB), nout * ct, ny, ls, M.rady, M.nsty, tw);
  for (unsigned it = threadIdx.x; it < nout * ncol; it += B) {
    const bool f = it >= ncol;
    const unsigned rem = f ? it - ncol : it, w = rem & (rc - 1), ty = rem >> lsh;
    const unsigned ky = (ty << M.lsrt) + (w >> M.lct), c = w & (ct - 1);
    (f ? W.s1 : W.s0)[mul24(ty, rowstep) + tbase + w] = cconj(r[mul24((f ? ct : 0) + c, ls) + px(ky)]);
  }
}

// Value of one multiplier code applied to z at (ky, kx): a = kappa (or Y_dis),
// b = Y_abs, sx / sy the 1-D staggered symbols at kx / ky.
__device__ __forceinline__ float2 mult_apply(int code, float a, float b, float2 sx, float2 sy, float2 z) {
  switch (code) {
    case MC_DXP:
    case MC_DXM: return cmul(cscale(sx, a), z);
    case MC_DYP:
    case MC_DYM: return cmul(cscale(sy, a), z);
    case MC_LDIS: return cscale(z, a);
    case MC_LABS: return cscale(z, b);
    default: return make_float2(0.f, 0.f);
  }
}

// Conjugated products of the packed DC / Nyquist column at row ky: z[f] is
// field f's forward spectrum there, zm[f] the conjugate at the mirror row
// ny - ky; the two real columns are separated, multiplied with their own
// tables (a, b at kx = 0; an, bn at the Nyquist column) and packed again.
template <int CM>
__device__ __forceinline__ void packed_products(int mcode, float a, float b, float an, float bn, float2 sx,
                                                float2 sxn, float2 sy, const float2* z, const float2* zm,
                                                float2* g) {
  constexpr int nin = kColIn[CM], nout = kColOut[CM];
  float2 f0[2], fn[2];
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    if (f < nin) {
      f0[f] = cscale(cadd(z[f], zm[f]), 0.5f);
      fn[f] = mul_mi(cscale(csub(z[f], zm[f]), 0.5f));
    } else {
      f0[f] = fn[f] = make_float2(0.f, 0.f);
    }
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    if (q < nout) {
      float2 g0 = make_float2(0.f, 0.f), gn = make_float2(0.f, 0.f);
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const int code = (mcode >> (4 * (2 * q + f))) & 15;
        if (code) {
          g0 = cadd(g0, mult_apply(code, a, b, sx, sy, f0[f]));
          gn = cadd(gn, mult_apply(code, an, bn, sxn, sy, fn[f]));
        }
      }
      g[q] = cconj(make_float2(g0.x - gn.y, g0.y + gn.x));
    }
  }
}

// Multiply phase through LDS for the first `ncols` columns of the tile
// (including the packed DC / Nyquist column, whose two real columns are
// separated with the mirror element ny - ky): r holds the forward spectra, o
// receives the conjugated products.  Loads its multiplier values itself.
template <int CM>
__device__ __forceinline__ void col_mult_lds(const Medium& M, int tile, int mcode, int ls, int ncols,
                                             const float2* r, float2* o) {
  constexpr int nin = kColIn[CM], nout = kColOut[CM];
  const int ny = M.ny, nxh = M.nxh, ct = M.ct, c0 = tile * ct, B = blockDim.x;
  int xcode = 0, ycode = 0;
  bool frac = false, labs = false;
  for (int e = 0; e < 4; ++e) {
    const int c = (mcode >> (4 * e)) & 15;
    if (c == MC_DXP || c == MC_DXM) xcode = c;
    if (c == MC_DYP || c == MC_DYM) ycode = c;
    if (c == MC_LDIS) frac = true;
    if (c == MC_LABS) { frac = true; labs = true; }
  }
  const float* tabA = frac ? M.ldis : M.kap;
  const float2* symx = xcode == MC_DXP ? M.dxp : M.dxm;
  const float2* symy = ycode == MC_DYP ? M.dyp : M.dym;
  const float rny = 1.0f / static_cast<float>(ny);
  for (int it = threadIdx.x; it < ncols * ny; it += B) {
    const int c = ncols == 1 ? 0 : fdiv(it, ny, rny), ky = it - c * ny, kx = c0 + c;
    const unsigned t = mul24(kx, ny) + ky, tn = mul24(nxh, ny) + ky;   // tables are [kx][ky]
    const float a = tabA[t], b = labs ? M.labs[t] : 0.f;
    const float2 sx = xcode ? symx[kx] : make_float2(0.f, 0.f), sy = ycode ? symy[ky] : make_float2(0.f, 0.f);
    if (kx == 0) {
      const float an = tabA[tn], bn = labs ? M.labs[tn] : 0.f;
      const float2 sxn = xcode ? symx[nxh] : make_float2(0.f, 0.f);
      const int km = ky ? ny - ky : 0;
      float2 z[2], zm[2], g[2];
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        z[f] = f < nin ? r[mul24(f * ct + c, ls) + px(ky)] : make_float2(0.f, 0.f);
        zm[f] = f < nin ? cconj(r[mul24(f * ct + c, ls) + px(km)]) : make_float2(0.f, 0.f);
      }
      packed_products<CM>(mcode, a, b, an, bn, sx, sxn, sy, z, zm, g);
#pragma unroll
      for (int q = 0; q < 2; ++q)
        if (q < nout) o[mul24(q * ct + c, ls) + px(ky)] = g[q];
    } else {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (q < nout) {
          float2 acc = make_float2(0.f, 0.f);
#pragma unroll
          for (int f = 0; f < 2; ++f) {
            const int code = (mcode >> (4 * (2 * q + f))) & 15;
            if (code && f < nin) acc = cadd(acc, mult_apply(code, a, b, sx, sy, r[mul24(f * ct + c, ls) + px(ky)]));
          }
          o[mul24(q * ct + c, ls) + px(ky)] = cconj(acc);
        }
      }
    }
  }
}

// The multiply phase of the packed column (column 0 of tile 0) in place: lines
// f ct hold the forward spectra, lines q ct receive the conjugated products.
// Every thread reads its rows and their mirrors before any is overwritten.
template <int CM>
__device__ __forceinline__ void col_mult_packed_ip(const Medium& M, int mcode, int ls, float2* a) {
  constexpr int nin = kColIn[CM], nout = kColOut[CM];
  const int ny = M.ny, nxh = M.nxh, ct = M.ct, B = blockDim.x, tid = threadIdx.x;
  int xcode = 0, ycode = 0;
  bool frac = false, labs = false;
  for (int e = 0; e < 4; ++e) {
    const int c = (mcode >> (4 * e)) & 15;
    if (c == MC_DXP || c == MC_DXM) xcode = c;
    if (c == MC_DYP || c == MC_DYM) ycode = c;
    if (c == MC_LDIS) frac = true;
    if (c == MC_LABS) { frac = true; labs = true; }
  }
  const float* tabA = frac ? M.ldis : M.kap;
  const float2* symx = xcode == MC_DXP ? M.dxp : M.dxm;
  const float2* symy = ycode == MC_DYP ? M.dyp : M.dym;
  float2 z[kColPer][2], zm[kColPer][2];  // ny <= kColPer * B
#pragma unroll
  for (int k = 0; k < kColPer; ++k) {
    const int ky = tid + k * B;
    if (ky < ny) {
      const int km = ky ? ny - ky : 0;
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        z[k][f] = f < nin ? a[mul24(f * ct, ls) + px(ky)] : make_float2(0.f, 0.f);
        zm[k][f] = f < nin ? cconj(a[mul24(f * ct, ls) + px(km)]) : make_float2(0.f, 0.f);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kColPer; ++k) {
    const int ky = tid + k * B;
    if (ky < ny) {
      const unsigned tn = mul24(nxh, ny) + ky;   // tables are [kx][ky]; kx = 0 here
      const float va = tabA[ky], vb = labs ? M.labs[ky] : 0.f;
      const float an = tabA[tn], bn = labs ? M.labs[tn] : 0.f;
      const float2 sx = xcode ? symx[0] : make_float2(0.f, 0.f), sxn = xcode ? symx[nxh] : make_float2(0.f, 0.f);
      const float2 sy = ycode ? symy[ky] : make_float2(0.f, 0.f);
      float2 g[2];
      packed_products<CM>(mcode, va, vb, an, bn, sx, sxn, sy, z[k], zm[k], g);
#pragma unroll
      for (int q = 0; q < 2; ++q)
        if (q < nout) a[mul24(q * ct, ls) + px(ky)] = g[q];
    }
  }
}

// One Stockham stage in place on `nlines` lines a + l lstep (at most two
// lines of N <= kColPer B points): all butterflies are read and transformed
// in registers, then the block synchronises and writes them back.
template <int R, int NS, int NB, int OFF>
__device__ __forceinline__ void stage_ip(float2* a, int nlines, int lstep, const float2* tw) {
  constexpr int MB = (2 * kColPer + R - 1) / R;
  const unsigned total = unsigned(nlines) * NB;
  float2 v[MB][R];
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const unsigned it = threadIdx.x + i * blockDim.x;
    if (it < total) {
      const unsigned line = it / NB, j = it % NB;
      stage_load<R, NB>(v[i], a + line * lstep, j);
      stage_regs<R, NS, OFF>(v[i], j, tw);
    }
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < MB; ++i) {
    const unsigned it = threadIdx.x + i * blockDim.x;
    if (it < total) {
      const unsigned line = it / NB, j = it % NB;
      stage_store<R, NS>(v[i], a + line * lstep, j);
    }
  }
}

// Column pass for power-of-two line lengths N with a compile-time plan.  The
// forward transform's first stage is computed straight from the global loads
// and the inverse transform (the same plan in reverse order, so that its
// first stage takes the butterfly outputs one thread already holds) writes
// its last stage straight to global memory; in between, the forward
// transform's last stage, the multipliers and the inverse transform's first
// stage stay in registers.  The tile with the packed DC / Nyquist column
// (tile 0) takes its multiply phase through LDS.
// IP: the FFT stages run in place in one LDS line buffer (each exchange
// stage gathers its butterflies into registers, synchronises, scatters), which
// halves the block's LDS and lets more blocks share a CU.
template <int CM, int N, bool TG, bool IP = false>
__device__ __forceinline__ void col_fused(const Medium& M, const Work& W, int tile, int mcode, float2* lds) {
  constexpr int nin = kColIn[CM], nout = kColOut[CM];
  constexpr int NST = plan_nst(N), LS = col_lstride(N);
  constexpr int R1 = radix_of<N, false>(0), NB1 = N / R1;        // first forward = last inverse stage
  constexpr int RS = radix_of<N, false>(NST - 1), NBS = N / RS;  // last forward = first inverse stage
  static_assert(RS == radix_of<N, true>(0) && R1 == radix_of<N, true>(NST - 1), "plan reversal");
  constexpr int OFFS = NBS - R1;  // twiddles of the last forward stage (Ns = NBS)
  constexpr int OFFL = NB1 - RS;  // twiddles of the last inverse stage (Ns = NB1)
  constexpr int kQ = (nin * kColPer + R1 - 1) / R1;  // first-stage butterflies per thread (bound)
  constexpr int kP = (kColPer + RS - 1) / RS;         // middle butterflies per thread (bound)
  const int nxh = M.nxh, ct = M.ct, c0 = tile * ct, B = blockDim.x, lct = M.lct, lsrt = M.lsrt;
  const int tid = threadIdx.x;
  float2* bufA = lds;
  float2* bufB = IP ? lds : lds + 2 * ct * LS;
  float2* const twl = lds + (IP ? 2 : 4) * ct * LS;  // LDS copies: forward-plan twiddles, then reversed-plan ones
  const float2* const tw = TG ? static_cast<const float2*>(M.twy) : twl;
  const float2* const twr = TG ? static_cast<const float2*>(M.twyr) : twl + N;
  int xcode = 0, ycode = 0;
  bool frac = false, labs = false;
  for (int e = 0; e < 4; ++e) {
    const int c = (mcode >> (4 * e)) & 15;
    if (c == MC_DXP || c == MC_DXM) xcode = c;
    if (c == MC_DYP || c == MC_DYM) ycode = c;
    if (c == MC_LDIS) frac = true;
    if (c == MC_LABS) { frac = true; labs = true; }
  }
  const float* tabA = frac ? M.ldis : M.kap;
  const float2* symx = xcode == MC_DXP ? M.dxp : M.dxm;
  const float2* symy = ycode == MC_DYP ? M.dyp : M.dym;
  // element ky of column c of the tile: (ky / srt) rowstep + tbase + (ky mod srt) ct + c;
  // inputs r and r + 1 of a first-stage butterfly are step1 apart (srt divides NB1)
  const unsigned rowstep = unsigned(nxh) * M.srt, tbase = unsigned(tile) * (M.srt * ct);
  const unsigned step1 = mul24(NB1 >> lsrt, rowstep);
  auto elem = [&](unsigned j, unsigned c) { return mul24(j >> lsrt, rowstep) + tbase + ((j & (M.srt - 1)) << lct) + c; };

  // ---- load phase: first-stage inputs, both twiddle tables, middle multipliers
  const unsigned nq = unsigned(nin * ct) * NB1;
  float2 v1[kQ][R1];
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    if (wave_base() + i * B < nq) {
      const unsigned q = min(unsigned(tid + i * B), nq - 1);
      const unsigned l = q / NB1, j = q % NB1, f = l >> lct, c = l & (ct - 1);
      const float2* src = (f ? W.s1 : W.s0) + elem(j, c);
#pragma unroll
      for (int r = 0; r < R1; ++r) v1[i][r] = src[r * step1];
    }
  }
  TwRegsK<kColPer> TW, TWR;  // N <= kColPer * B (ct >= 1)
  if constexpr (!TG) {
    fetch_tw(TW, M.twy, N);
    fetch_tw(TWR, M.twyr, N);
  }
  const unsigned np = unsigned(ct) * NBS;
  const unsigned tstep = unsigned(NBS);   // tables are [kx][ky]: a column's entries are contiguous
  float ma[kP][RS], mb[kP][RS];
  float2 msy[kP][RS], msx[kP];
#pragma unroll
  for (int i = 0; i < kP; ++i) {
    if (wave_base() + i * B < np) {
      const unsigned pp = min(unsigned(tid + i * B), np - 1);
      const unsigned c = pp / NBS, j = pp % NBS, kx = c0 + c;
      const unsigned t0 = mul24(kx, N) + j;
      msx[i] = xcode ? symx[kx] : make_float2(0.f, 0.f);
#pragma unroll
      for (int r = 0; r < RS; ++r) {
        ma[i][r] = tabA[t0 + r * tstep];
        mb[i][r] = labs ? M.labs[t0 + r * tstep] : 0.f;
        msy[i][r] = ycode ? symy[j + r * NBS] : make_float2(0.f, 0.f);
      }
    }
  }
  // ---- forward first stage from registers
#pragma unroll
  for (int i = 0; i < kQ; ++i) {
    const unsigned q = tid + i * B;
    if (q < nq) {
      const unsigned l = q / NB1, j = q % NB1;
      stage_regs<R1, 1, 0>(v1[i], j, tw);
      stage_store<R1, 1>(v1[i], bufA + l * LS, j);
    }
  }
  if constexpr (!TG) {
    put_tw(TW, twl, N);
    put_tw(TWR, twl + N, N);
  }
  __syncthreads();
  // ---- forward stages 2 .. NST-1
  float2* r;
  if constexpr (IP) r = fft_range_ip<N, LS, 1, NST - 1, R1>(bufA, nin * ct, tw);
  else r = fft_stages<N, false, LS, 1, NST - 1, R1>(bufA, bufB, nin * ct, tw);
  float2* o = IP ? r : other(r, bufA, bufB);
  // column 0 of tile 0 holds the packed DC / Nyquist column: its last forward
  // stage goes to LDS (into its own lines of o) for the mirror-element
  // multiply; every other column stays in registers.  A column takes the
  // same path whatever the tile shape, so results do not depend on it.
  const bool packed = c0 == 0;
  if (packed) {
    if constexpr (IP) {
      stage_ip<RS, NBS, NBS, OFFS>(r, nin, ct * LS, tw);  // lines f ct; the loop below reads other lines
    } else {
      for (unsigned it = tid; it < unsigned(nin) * NBS; it += B) {
        const unsigned f = it / NBS, j = it % NBS;
        stockham_c<RS, NBS, NBS, OFFS>(r + f * ct * LS, o + f * ct * LS, j, tw);
      }
    }
  }
  {
    // last forward stage, multipliers, first inverse stage: registers only
    float2 z[kP][nin][RS];
#pragma unroll
    for (int i = 0; i < kP; ++i) {
      const unsigned pp = tid + i * B;
      if (pp < np && !(packed && pp < NBS)) {
        const unsigned c = pp / NBS, j = pp % NBS;
#pragma unroll
        for (int f = 0; f < nin; ++f) {
          stage_load<RS, NBS>(z[i][f], r + (f * ct + c) * LS, j);
          stage_regs<RS, NBS, OFFS>(z[i][f], j, tw);
        }
      }
    }
    if constexpr (IP) __syncthreads();  // the stores below overwrite lines just read
#pragma unroll
    for (int i = 0; i < kP; ++i) {
      const unsigned pp = tid + i * B;
      if (pp < np && !(packed && pp < NBS)) {
        const unsigned c = pp / NBS, j = pp % NBS;
#pragma unroll
        for (int q = 0; q < nout; ++q) {
          float2 w[RS];
#pragma unroll
          for (int rr = 0; rr < RS; ++rr) {
            float2 acc = make_float2(0.f, 0.f);
#pragma unroll
            for (int f = 0; f < nin; ++f) {
              const int code = (mcode >> (4 * (2 * q + f))) & 15;
              if (code) acc = cadd(acc, mult_apply(code, ma[i][rr], mb[i][rr], msx[i], msy[i][rr], z[i][f][rr]));
            }
            w[rr] = cconj(acc);
          }
          stage_regs<RS, 1, 0>(w, j, twr);
          stage_store<RS, 1>(w, o + (q * ct + c) * LS, j);
        }
      }
    }
    __syncthreads();
  }
  if (packed) {
    if constexpr (IP) {
      // column 0 lines, in place: products (q ct), then the first inverse stage
      col_mult_packed_ip<CM>(M, mcode, LS, o);
      __syncthreads();
      stage_ip<RS, 1, NBS, 1 - RS>(o, nout, ct * LS, twr);
    } else {
      // column 0 lines: o (f ct) -> products r (q ct) -> first inverse stage o (q ct)
      col_mult_lds<CM>(M, tile, mcode, LS, 1, o, r);
      __syncthreads();
      for (unsigned it = tid; it < unsigned(nout) * NBS; it += B) {
        const unsigned q = it / NBS, j = it % NBS;
        stockham_c<RS, 1, NBS, 1 - RS>(r + q * ct * LS, o + q * ct * LS, j, twr);
      }
    }
    __syncthreads();
  }
  // ---- inverse stages 2 .. NST-1, then the last one straight to global memory
  float2* r2;
  if constexpr (IP) r2 = fft_range_ip<N, LS, 1, NST - 1, RS, true>(o, nout * ct, twr);
  else r2 = fft_stages<N, true, LS, 1, NST - 1, RS>(o, other(o, bufA, bufB), nout * ct, twr);
  const unsigned nq2 = unsigned(nout * ct) * NB1;
  for (unsigned q = tid; q < nq2; q += B) {
    const unsigned l = q / NB1, j = q % NB1, f = l >> lct, c = l & (ct - 1);
    float2 v[R1];
    stage_load<R1, NB1>(v, r2 + l * LS, j);
    stage_regs<R1, NB1, OFFL>(v, j, twr);
    float2* dst = (f ? W.s1 : W.s0) + elem(j, c);
#pragma unroll
    for (int rr = 0; rr < R1; ++rr) st_spec<TG>(dst + rr * step1, cconj(v[rr]));
  }
}

template <bool U, int CM, int NF, bool TG = false>
__global__ void __launch_bounds__(kMaxThreads)
col_kernel(const Launch L, int ntile, int chunk, int mcode_arg, int n) {
  const int mcode = CM == CM_APPLY ? mcode_arg : kColCode[CM];
  extern __shared__ float2 lds[];
  if constexpr (U) col_args_batch<CM>(L, ntile, chunk, n);
  int item, tile;
  if (!locate<U>(L, ntile, chunk, item, tile)) return;
  const Medium& M = medium_of<U>(L, item);
  const Work W = U ? shift_work(L.w0, item * L.wstride) : L.items[item].w;
  if (n > M.nt - 2) return;  // this problem has finished (uneven batches)
  // fused path: power-of-two lengths whose first-stage stride is a whole number
  // of tile rows.  An instance with a compile-time power-of-two length takes it
  // unconditionally: a row tile of a power-of-two grid of 128+ rows has at most
  // ny / 8 rows (a power of two), and N / R1 >= N / 8, so the condition holds;
  // the generic pass is not compiled into such instances.
  if constexpr (NF == 128 || NF == 256 || NF == 512 || NF == 1024) {
    col_fused<CM, NF, TG, !TG>(M, W, tile, mcode, lds);  // in place unless twiddles are read from global memory
  } else {
#define QPAT_COL_CASE(N)                                                 \
  case N:                                                                \
    if ((N / radix_of<N, false>(0)) % M.srt == 0) {                      \
      col_fused<CM, N, TG>(M, W, tile, mcode, lds);                      \
      return;                                                            \
    }                                                                    \
    break;
    if constexpr (NF == 0) {
      switch (M.ny) {
        QPAT_COL_CASE(128)
        QPAT_COL_CASE(256)
        QPAT_COL_CASE(512)
        QPAT_COL_CASE(1024)
        default: break;
      }
    }
#undef QPAT_COL_CASE
    col_generic<CM, NF, TG>(M, W, tile, mcode, lds);
  }
}

// ---------------------------------------------------------------- sensor data
__global__ void combine_kernel(const Item* __restrict__ items, const IO* __restrict__ io) {
  const Medium& M = items[blockIdx.y].m;
  const float* part = items[blockIdx.y].w.part;
  float* out = io[blockIdx.y].out;
  const int total = M.nt * M.ns;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x)
    out[i] = part[2 * i] + part[2 * i + 1];
}

// Residual samples in sensor-tap order, rtap[m][e] = r[m][s(e)] for the 2 ns
// taps e (the adjoint row passes read one contiguous run per tile).  Written
// into the vector's sensor-partial buffer, which the adjoint does not use.
__global__ void tap_order_kernel(const Item* __restrict__ items, const IO* __restrict__ io) {
  const Medium& M = items[blockIdx.y].m;
  float* dst = items[blockIdx.y].w.part;
  const float* r = io[blockIdx.y].in;
  const int ntap = 2 * M.ns, total = M.nt * ntap;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
    const int m = i / ntap, e = i - m * ntap;
    dst[i] = r[unsigned(m) * unsigned(M.ns) + M.taps[e].s];
  }
}

// ---------------------------------------------------------------- sound-speed gradient
// d<r, H_a p0>/dc = sum_m p*^m dp^m/dc (the equation-of-state part, gc) minus
// (2/c) p0 H_a^* r (the source of eq s1 scales as 1/c^2).
__global__ void __launch_bounds__(kBlock) grad_c_kernel(const float* __restrict__ c2, const float* __restrict__ p0,
                                                        const float* __restrict__ g0, const double* __restrict__ gc,
                                                        long long n, long long gc_stride, float* __restrict__ out) {
  const long long b = blockIdx.y;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double c = sqrt(double(c2[i]));
    out[b * n + i] = float(gc[b * gc_stride + i] - 2.0 * double(p0[b * n + i]) * double(g0[b * n + i]) / c);
  }
}

// ---------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

__global__ void __launch_bounds__(kBlock) dot_partial(const float* __restrict__ a, const float* __restrict__ b,
                                                      int64_t n, double* __restrict__ partial) {
  __shared__ double red[kBlock / 64];
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    acc += double(a[i]) * double(b[i]);
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += red[w];
    partial[blockIdx.x] = s;
  }
}

__global__ void __launch_bounds__(kBlock) dot_final(const double* __restrict__ partial, int nblk,
                                                    double* __restrict__ out) {
  __shared__ double red[kBlock / 64];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblk; i += blockDim.x) acc += partial[i];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < kBlock / 64; ++w) s += red[w];
    *out = s;
  }
}

// ---------------------------------------------------------------- launchers
// Launches pick the kernel instance for their row / column length (lengths
// with a compile-time plan): uniform launches by the plan's length, table
// launches by the length all their items share (`len`, 0 when they differ:
// then the all-length instance).  1024-point columns stay on the all-length
// instance: the dedicated one measured 5-10% slower at 1024^2 x 8.
#define QPAT_FOR_LENGTHS(X) X(128) X(256) X(384) X(512) X(1024)
#define QPAT_FOR_COL_LENGTHS(X) X(128) X(256) X(384) X(512) X(1024)

// Compile-time row lengths whose plan fuses the boundary stage (RM_FZ instances).
#define QPAT_FOR_FUSED_LENGTHS(X) X(128) X(256) X(512) X(1024)

template <int MODE>
static hipError_t launch_row_t(const Launch& L, bool uniform, int len, bool tg, int ntile, int chunk, int nblocks,
                               int threads, size_t lds, int n, int flags, hipStream_t st) {
  const dim3 g(nblocks), t(threads);
  if constexpr ((MODE & RM_FZ) != 0) {
    if (tg && !uniform) return hipErrorInvalidValue;
#define QPAT_ROW_LEN(N)                                                                                        \
  case N:                                                                                                      \
    if (tg) hipLaunchKernelGGL((row_kernel<MODE, true, N, true>), g, t, lds, st, L, ntile, chunk, n, flags);  \
    else if (uniform) hipLaunchKernelGGL((row_kernel<MODE, true, N>), g, t, lds, st, L, ntile, chunk, n, flags); \
    else hipLaunchKernelGGL((row_kernel<MODE, false, N>), g, t, lds, st, L, ntile, chunk, n, flags);            \
    break;
    switch (uniform ? L.m.nx : len) {
      QPAT_FOR_FUSED_LENGTHS(QPAT_ROW_LEN)
      default: return hipErrorInvalidValue;
    }
#undef QPAT_ROW_LEN
    return hipGetLastError();
  } else {
    if (uniform && tg) {
#define QPAT_ROW_LEN(N) \
  case N: hipLaunchKernelGGL((row_kernel<MODE, true, N, true>), g, t, lds, st, L, ntile, chunk, n, flags); break;
      switch (L.m.nx) {
        QPAT_FOR_LENGTHS(QPAT_ROW_LEN)
        default: return hipErrorInvalidValue;  // global-twiddle instances exist for these lengths only
      }
#undef QPAT_ROW_LEN
    } else if (uniform) {
#define QPAT_ROW_LEN(N) \
  case N: hipLaunchKernelGGL((row_kernel<MODE, true, N>), g, t, lds, st, L, ntile, chunk, n, flags); break;
      switch (L.m.nx) {
        QPAT_FOR_LENGTHS(QPAT_ROW_LEN)
        default: hipLaunchKernelGGL((row_kernel<MODE, true, 0>), g, t, lds, st, L, ntile, chunk, n, flags); break;
      }
#undef QPAT_ROW_LEN
    } else {
      if (tg) return hipErrorInvalidValue;
#define QPAT_ROW_LEN(N) \
  case N: hipLaunchKernelGGL((row_kernel<MODE, false, N>), g, t, lds, st, L, ntile, chunk, n, flags); break;
      switch (len) {
        QPAT_FOR_LENGTHS(QPAT_ROW_LEN)
        default: hipLaunchKernelGGL((row_kernel<MODE, false, 0>), g, t, lds, st, L, ntile, chunk, n, flags); break;
      }
#undef QPAT_ROW_LEN
    }
    return hipGetLastError();
  }
}

hipError_t launch_row(int mode, const Launch& L, bool uniform, int len, bool tg, int ntile, int chunk, int nblocks,
                      int threads, size_t lds, int n, int flags, hipStream_t st) {
#define QPAT_ROW_CASE(m) \
  case m: return launch_row_t<m>(L, uniform, len, tg, ntile, chunk, nblocks, threads, lds, n, flags, st);
  switch (mode) {
    QPAT_ROW_CASE(RM_F1)
    QPAT_ROW_CASE(RM_F2)
    QPAT_ROW_CASE(RM_F2L)
    QPAT_ROW_CASE(RM_F3)
    QPAT_ROW_CASE(RM_A1)
    QPAT_ROW_CASE(RM_A1L)
    QPAT_ROW_CASE(RM_A2)
    QPAT_ROW_CASE(RM_A3)
    QPAT_ROW_CASE(RM_FWD1)
    QPAT_ROW_CASE(RM_INV1)
    QPAT_ROW_CASE(RM_F2L | RM_X)
    QPAT_ROW_CASE(RM_F3 | RM_X)
    QPAT_ROW_CASE(RM_A1 | RM_X)
    QPAT_ROW_CASE(RM_A1L | RM_X)
    QPAT_ROW_CASE(RM_F2 | RM_FZ)
    QPAT_ROW_CASE(RM_A2 | RM_FZ)
    default: return hipErrorInvalidValue;
  }
#undef QPAT_ROW_CASE
}

template <int CM>
static hipError_t launch_col_t(int mcode, const Launch& L, bool uniform, int len, bool tg, int ntile, int chunk,
                               int nblocks, int threads, size_t lds, int n, hipStream_t st) {
  const dim3 g(nblocks), t(threads);
  if (uniform && tg) {
#define QPAT_COL_LEN(N) \
  case N: hipLaunchKernelGGL((col_kernel<true, CM, N, true>), g, t, lds, st, L, ntile, chunk, mcode, n); break;
    switch (L.m.ny) {
      QPAT_FOR_COL_LENGTHS(QPAT_COL_LEN)
      default: return hipErrorInvalidValue;
    }
#undef QPAT_COL_LEN
  } else if (uniform) {
#define QPAT_COL_LEN(N) \
  case N: hipLaunchKernelGGL((col_kernel<true, CM, N>), g, t, lds, st, L, ntile, chunk, mcode, n); break;
    switch (L.m.ny) {
      QPAT_FOR_COL_LENGTHS(QPAT_COL_LEN)
      default: hipLaunchKernelGGL((col_kernel<true, CM, 0>), g, t, lds, st, L, ntile, chunk, mcode, n); break;
    }
#undef QPAT_COL_LEN
  } else {
    if (tg) return hipErrorInvalidValue;
#define QPAT_COL_LEN(N) \
  case N: hipLaunchKernelGGL((col_kernel<false, CM, N>), g, t, lds, st, L, ntile, chunk, mcode, n); break;
    switch (len) {
      QPAT_FOR_COL_LENGTHS(QPAT_COL_LEN)
      default: hipLaunchKernelGGL((col_kernel<false, CM, 0>), g, t, lds, st, L, ntile, chunk, mcode, n); break;
    }
#undef QPAT_COL_LEN
  }
  return hipGetLastError();
}

hipError_t launch_col(int cm, int mcode, const Launch& L, bool uniform, int len, bool tg, int ntile, int chunk,
                      int nblocks, int threads, size_t lds, int n, hipStream_t st) {
#define QPAT_COL_CASE(c) \
  case c: return launch_col_t<c>(mcode, L, uniform, len, tg, ntile, chunk, nblocks, threads, lds, n, st);
  switch (cm) {
    QPAT_COL_CASE(CM_GRADP1)
    QPAT_COL_CASE(CM_GRADM2)
    QPAT_COL_CASE(CM_FRAC)
    QPAT_COL_CASE(CM_GRADP2)
    QPAT_COL_CASE(CM_DIVM)
    QPAT_COL_CASE(CM_APPLY)
    default: return hipErrorInvalidValue;
  }
#undef QPAT_COL_CASE
}

bool kernels_row_fused(int n, bool tg) {
#define QPAT_HAVE(N) if (n == N) return row_fusable<N>() && (plan_radix(N, 0) > 4 || !tg);
  QPAT_FOR_FUSED_LENGTHS(QPAT_HAVE)
#undef QPAT_HAVE
  return false;
}

bool kernels_have_length(int n, bool col) {
#define QPAT_HAVE(N) if (n == N) return true;
  if (col) {
    QPAT_FOR_COL_LENGTHS(QPAT_HAVE)
  } else {
    QPAT_FOR_LENGTHS(QPAT_HAVE)
  }
#undef QPAT_HAVE
  return false;
}

// Let every row / column pass kernel use up to `bytes` of dynamic LDS.
template <typename K>
static hipError_t allow_fn(K* k, size_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                             int(bytes));
}
template <int MODE>
static hipError_t allow_row(size_t bytes) {
  hipError_t e = allow_fn(&row_kernel<MODE, false, 0>, bytes);
  if (e == hipSuccess) e = allow_fn(&row_kernel<MODE, true, 0>, bytes);
#define QPAT_ALLOW_ROW(N)                                                       \
  if (e == hipSuccess) e = allow_fn(&row_kernel<MODE, true, N>, bytes);       \
  if (e == hipSuccess) e = allow_fn(&row_kernel<MODE, true, N, true>, bytes); \
  if (e == hipSuccess) e = allow_fn(&row_kernel<MODE, false, N>, bytes);
  QPAT_FOR_LENGTHS(QPAT_ALLOW_ROW)
#undef QPAT_ALLOW_ROW
  return e;
}
template <int MODE>
static hipError_t allow_row_fused(size_t bytes) {
  hipError_t e = hipSuccess;
#define QPAT_ALLOW_ROW(N)                                                       \
  if (e == hipSuccess) e = allow_fn(&row_kernel<MODE, true, N>, bytes);       \
  if (e == hipSuccess) e = allow_fn(&row_kernel<MODE, true, N, true>, bytes); \
  if (e == hipSuccess) e = allow_fn(&row_kernel<MODE, false, N>, bytes);
  QPAT_FOR_FUSED_LENGTHS(QPAT_ALLOW_ROW)
#undef QPAT_ALLOW_ROW
  return e;
}
template <int CM>
static hipError_t allow_col(size_t bytes) {
  hipError_t e = allow_fn(&col_kernel<false, CM, 0>, bytes);
  if (e == hipSuccess) e = allow_fn(&col_kernel<true, CM, 0>, bytes);
#define QPAT_ALLOW_COL(N)                                                     \
  if (e == hipSuccess) e = allow_fn(&col_kernel<true, CM, N>, bytes);       \
  if (e == hipSuccess) e = allow_fn(&col_kernel<true, CM, N, true>, bytes); \
  if (e == hipSuccess) e = allow_fn(&col_kernel<false, CM, N>, bytes);
  QPAT_FOR_COL_LENGTHS(QPAT_ALLOW_COL)
#undef QPAT_ALLOW_COL
  return e;
}

hipError_t kernels_allow_lds(size_t bytes) {
  const hipError_t es[] = {allow_row<RM_F1>(bytes),      allow_row<RM_F2>(bytes),     allow_row<RM_F2L>(bytes),
                           allow_row<RM_F3>(bytes),      allow_row<RM_A1>(bytes),     allow_row<RM_A1L>(bytes),
                           allow_row<RM_A2>(bytes),      allow_row<RM_A3>(bytes),     allow_row<RM_FWD1>(bytes),
                           allow_row<RM_INV1>(bytes),    allow_row<RM_F2L | RM_X>(bytes), allow_row<RM_F3 | RM_X>(bytes),
                           allow_row<RM_A1 | RM_X>(bytes), allow_row<RM_A1L | RM_X>(bytes),
                           allow_row_fused<RM_F2 | RM_FZ>(bytes), allow_row_fused<RM_A2 | RM_FZ>(bytes),
                           allow_col<CM_GRADP1>(bytes), allow_col<CM_GRADM2>(bytes),
                           allow_col<CM_FRAC>(bytes),    allow_col<CM_GRADP2>(bytes), allow_col<CM_DIVM>(bytes),
                           allow_col<CM_APPLY>(bytes)};
  for (hipError_t e : es)
    if (e != hipSuccess) return e;
  return hipSuccess;
}

hipError_t launch_combine(const Item* items, const IO* io, int nitems, int max_count, hipStream_t st) {
  int bx = (max_count + kBlock - 1) / kBlock;
  if (bx > 1024) bx = 1024;
  if (bx < 1) bx = 1;
  hipLaunchKernelGGL(combine_kernel, dim3(bx, nitems), dim3(kBlock), 0, st, items, io);
  return hipGetLastError();
}

hipError_t launch_tap_order(const Item* items, const IO* io, int nitems, int max_count, hipStream_t st) {
  int bx = (max_count + kBlock - 1) / kBlock;
  if (bx > 1024) bx = 1024;
  if (bx < 1) bx = 1;
  hipLaunchKernelGGL(tap_order_kernel, dim3(bx, nitems), dim3(kBlock), 0, st, items, io);
  return hipGetLastError();
}

hipError_t launch_grad_c(const float* c2, const float* p0, const float* g0, const double* gc, long long n,
                         int batch, long long gc_stride, float* out, hipStream_t st) {
  long long bx = (n + kBlock - 1) / kBlock;
  if (bx > 1024) bx = 1024;
  hipLaunchKernelGGL(grad_c_kernel, dim3(unsigned(bx), unsigned(batch)), dim3(kBlock), 0, st, c2, p0, g0, gc, n,
                     gc_stride, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- output check
// flag <- 1 if any of x[0 .. n) is NaN or infinite (every writer stores the
// same value, so no atomics are needed; the host clears the flag).
__global__ void __launch_bounds__(kBlock) finite_kernel(const float* __restrict__ x, int64_t n, int* flag) {
  bool bad = false;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    bad |= !isfinite(x[i]);
  if (bad) *flag = 1;
}

hipError_t launch_finite(const float* x, int64_t n, int* flag, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t want = (n + kBlock - 1) / kBlock;
  const int nblk = int(want < 1024 ? want : 1024);
  hipLaunchKernelGGL(finite_kernel, dim3(nblk), dim3(kBlock), 0, st, x, n, flag);
  return hipGetLastError();
}

// Partial sums of qpat_dot_noalloc: a static array that every device the
// library runs on holds until the process ends, shared by all calls on that
// device.  Host code never passes the array's name to a kernel; it uses the
// device address looked up once per device below.
static __device__ __align__(256) double scratch[kDotBlocks];

hipError_t dot_scratch(double** ptr) {
  static std::mutex mu;
  static std::map<int, double*> addr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> g(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    double* p = nullptr;
    e = hipGetSymbolAddress((void**)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (p == nullptr) return hipErrorInvalidSymbol;
    it = addr.emplace(dev, p).first;
  }
  *ptr = it->second;
  return hipSuccess;
}

hipError_t launch_dot(const float* a, const float* b, int64_t n, double* partial, int nblk, double* out,
                      hipStream_t st) {
  hipLaunchKernelGGL(dot_partial, dim3(nblk), dim3(kBlock), 0, st, a, b, n, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dot_final, dim3(1), dim3(kBlock), 0, st, partial, nblk, out);
  return hipGetLastError();
}

}  // namespace qpat
