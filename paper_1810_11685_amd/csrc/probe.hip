// Grid-barrier probes for the persistent-launch question.
//
// A single solve is a chain of dependent passes, each ending in a global
// exchange (row spectra -> column passes -> row passes).  Inside one
// persistent kernel every exchange would need a device-wide barrier with the
// written data made visible across the XCDs' L2 caches; as separate launches
// the kernel boundary provides both.  These probes time one exchange step
// (every block writes its slot of a buffer, all blocks synchronise, every
// block reads another block's slot) three ways:
//   design 0  cooperative launch, one device-scope arrival counter;
//   design 1  cooperative launch, hierarchical: an arrival counter per XCD
//             group (blocks b with b mod 8 = x), the last arrival of a group
//             arriving at a global counter, the last global arrival bumping
//             a generation word that lane 0 of every block polls with backoff;
//   design 2  no barrier: one kernel per exchange step, captured in a hipGraph
//             (the kernel boundary is the barrier).
// Every wait is bounded: a block that spins longer than `spin_max` polls
// sets a time-out flag and leaves, the other blocks see the flag and leave
// too, and the host reports the time-out.  Cooperative launches are checked
// for co-residency on the host first.
#include <string>

#include "../../include/qpat.h"
#include "qpat_internal.hpp"

namespace qpat {

qpat_status set_error(qpat_status s, const std::string& msg);

namespace {

constexpr int kLine = 32;  // unsigneds per 128-byte line: each counter on its own line

struct BarrierState {
  unsigned xcd[kXcds * kLine];
  unsigned global[kLine];
  unsigned generation[kLine];
  unsigned timeout[kLine];
};

__device__ __forceinline__ unsigned ld_acq(unsigned* p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}

// Barrier k (k = 0, 1, ...) of a grid of nb blocks; counters only grow, so
// barrier k waits for the generation word to reach k + 1.  Returns false
// after a time-out (here or in another block).
__device__ bool grid_barrier(BarrierState* st, int design, unsigned k, int spin_max) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned nb = gridDim.x, b = blockIdx.x;
    __threadfence();  // release this block's writes before arriving
    bool last = false;
    if (design == 0) {
      const unsigned old = __hip_atomic_fetch_add(&st->global[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      last = old == (k + 1) * nb - 1;
    } else {
      const unsigned x = b % kXcds;
      const unsigned nbx = (nb - x + kXcds - 1) / kXcds;  // blocks of group x
      const unsigned ngrp = nb < unsigned(kXcds) ? nb : unsigned(kXcds);
      const unsigned old = __hip_atomic_fetch_add(&st->xcd[x * kLine], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      if (old == (k + 1) * nbx - 1) {
        const unsigned og = __hip_atomic_fetch_add(&st->global[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        last = og == (k + 1) * ngrp - 1;
      }
    }
    bool good = true;
    if (last) {
      __hip_atomic_store(&st->generation[0], k + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      int spins = 0;
      while (ld_acq(&st->generation[0]) < k + 1) {
        if (++spins > spin_max || ld_acq(&st->timeout[0]) != 0u) {
          __hip_atomic_store(&st->timeout[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          good = false;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    __threadfence();  // acquire: other blocks' writes are visible from here on
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}

// One exchange step k: write this block's slot of buffer k & 1, (barrier),
// read the next block's slot of the same buffer.  Slots are float4 vectors
// (words is a multiple of 4) and a thread's loads are unrolled so that they
// are all in flight together, as in the solver's passes.
__device__ __forceinline__ void write_slot(float* buf, int words, int k) {
  float4* dst = reinterpret_cast<float4*>(buf + (size_t(k & 1) * gridDim.x + blockIdx.x) * words);
  const int n4 = words >> 2;
#pragma unroll 4
  for (int i = threadIdx.x; i < n4; i += blockDim.x) dst[i] = make_float4(float(k + i), 0.f, 0.f, 0.f);
}
__device__ __forceinline__ float read_slot(const float* buf, int words, int k) {
  const unsigned nb = gridDim.x;
  const float4* src = reinterpret_cast<const float4*>(buf + (size_t(k & 1) * nb + (blockIdx.x + 1) % nb) * words);
  const int n4 = words >> 2;
  float acc = 0.f;
#pragma unroll 4
  for (int i = threadIdx.x; i < n4; i += blockDim.x) {
    const float4 v = src[i];
    acc += (v.x + v.y) + (v.z + v.w);
  }
  return acc;
}

__global__ void barrier_probe(BarrierState* st, int design, int iters, float* buf, int words, int spin_max,
                              float* sink) {
  float acc = 0.f;
  for (int k = 0; k < iters; ++k) {
    write_slot(buf, words, k);
    if (!grid_barrier(st, design, unsigned(k), spin_max)) break;
    acc += read_slot(buf, words, k);
  }
  if (acc == -1.f) sink[blockIdx.x] = acc;  // keeps the reads
}

// Design 2: one exchange step per launch; step k reads what step k - 1 wrote.
__global__ void exchange_step(float* buf, int words, int k, float* sink) {
  float acc = k > 0 ? read_slot(buf, words, k - 1) : 0.f;
  write_slot(buf, words, k);
  if (acc == -1.f) sink[blockIdx.x] = acc;
}

}  // namespace

qpat_status probe_barrier(int design, int nblocks, int threads, int iters, int words, hipStream_t st,
                          float* us_per_step, int* timed_out) {
  if (design < 0 || design > 2) return set_error(QPAT_E_INVALID, "design must be 0, 1 or 2");
  if (threads < 64 || threads > 1024 || (threads & 63)) return set_error(QPAT_E_INVALID, "threads: 64..1024, multiple of 64");
  if (nblocks < 1 || nblocks > 4096) return set_error(QPAT_E_INVALID, "nblocks must be in [1, 4096]");
  if (iters < 2 || iters > 100000) return set_error(QPAT_E_INVALID, "iters must be in [2, 100000]");
  if (words < 0 || words > (1 << 20) || (words & 3)) return set_error(QPAT_E_INVALID, "words must be a multiple of 4 in [0, 2^20]");
  if (!us_per_step || !timed_out) return set_error(QPAT_E_INVALID, "output pointer is NULL");
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return set_error(QPAT_E_HIP, "device query failed");
  if (design < 2) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, barrier_probe, threads, 0) != hipSuccess)
      return set_error(QPAT_E_HIP, "occupancy query failed");
    if (!prop.cooperativeLaunch || nblocks > per_cu * prop.multiProcessorCount)
      return set_error(QPAT_E_UNSUPPORTED, "the blocks of a cooperative probe must all be resident");
  }
  BarrierState* state = nullptr;
  float *buf = nullptr, *sink = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  qpat_status rc = QPAT_OK;
  std::string what;
  hipError_t e = hipSuccess;
  float ms[2] = {0.f, 0.f};
  const int counts[2] = {iters / 10 > 1 ? iters / 10 : 1, iters};
  const int spin_max = 2000000;
  auto run = [&](int count, float* out_ms) -> hipError_t {
    hipError_t r = hipMemsetAsync(state, 0, sizeof(BarrierState), st);
    if (r != hipSuccess) return r;
    if (design == 2) {
      // capture `count` dependent launches, then time one replay after a warm-up one
      if (ge) (void)hipGraphExecDestroy(ge), ge = nullptr;
      if (g) (void)hipGraphDestroy(g), g = nullptr;
      hipStream_t cs = nullptr;
      r = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
      if (r != hipSuccess) return r;
      r = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      for (int k = 0; k < count && r == hipSuccess; ++k) {
        hipLaunchKernelGGL(exchange_step, dim3(nblocks), dim3(threads), 0, cs, buf, words, k, sink);
        r = hipGetLastError();
      }
      hipError_t r2 = hipStreamEndCapture(cs, &g);
      (void)hipStreamDestroy(cs);
      if (r == hipSuccess) r = r2;
      if (r == hipSuccess) r = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
      if (r == hipSuccess) r = hipGraphLaunch(ge, st);
      if (r == hipSuccess) r = hipEventRecord(a, st);
      if (r == hipSuccess) r = hipGraphLaunch(ge, st);
    } else {
      void* args[] = {&state, &design, &count, &buf, &words, const_cast<int*>(&spin_max), &sink};
      r = hipEventRecord(a, st);
      if (r == hipSuccess)
        r = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(barrier_probe), dim3(nblocks), dim3(threads),
                                       args, 0, st);
    }
    if (r == hipSuccess) r = hipEventRecord(b, st);
    if (r == hipSuccess) r = hipEventSynchronize(b);
    if (r == hipSuccess) r = hipEventElapsedTime(out_ms, a, b);
    return r;
  };
  unsigned to = 0;
  do {
    if ((e = hipMalloc(&state, sizeof(BarrierState))) != hipSuccess) { what = "alloc"; break; }
    if ((e = hipMalloc(&buf, size_t(2) * nblocks * (words > 0 ? words : 1) * sizeof(float))) != hipSuccess) { what = "alloc"; break; }
    if ((e = hipMalloc(&sink, size_t(nblocks) * sizeof(float))) != hipSuccess) { what = "alloc"; break; }
    if ((e = hipEventCreate(&a)) != hipSuccess || (e = hipEventCreate(&b)) != hipSuccess) { what = "event"; break; }
    if ((e = run(counts[0], &ms[0])) != hipSuccess) { what = "probe run"; break; }  // also warms up
    if ((e = run(counts[0], &ms[0])) != hipSuccess) { what = "probe run"; break; }
    if ((e = run(counts[1], &ms[1])) != hipSuccess) { what = "probe run"; break; }
    if ((e = hipMemcpy(&to, state->timeout, sizeof(unsigned), hipMemcpyDeviceToHost)) != hipSuccess) { what = "read"; break; }
  } while (false);
  if (e != hipSuccess) rc = set_error(QPAT_E_HIP, "barrier probe: " + what + ": " + hipGetErrorString(e));
  *timed_out = int(to);
  *us_per_step = counts[1] > counts[0] ? (ms[1] - ms[0]) * 1e3f / float(counts[1] - counts[0]) : 0.f;
  if (ge) (void)hipGraphExecDestroy(ge);
  if (g) (void)hipGraphDestroy(g);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (state) (void)hipFree(state);
  if (buf) (void)hipFree(buf);
  if (sink) (void)hipFree(sink);
  return rc;
}

}  // namespace qpat

extern "C" qpat_status qpat_probe_barrier(int32_t design, int32_t nblocks, int32_t threads, int32_t iters,
                                          int32_t words, qpat_stream stream, float* us_per_step,
                                          int32_t* timed_out) {
  return qpat::probe_barrier(design, nblocks, threads, iters, words, (hipStream_t)stream, us_per_step, timed_out);
}
