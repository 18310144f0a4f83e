// Device helpers shared by the gfx950 kernels: bounded cross-workgroup barrier,
// wave reductions and the FP64 MFMA wrapper.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define RQ_DEV __device__ __forceinline__

namespace rq {

constexpr int kWave = 64;

// Device status word (int64[4]): [0] OR of error bits, [1] spare.
enum : int64_t { kErrTimeout = 1, kErrNonFinite = 2, kErrNoPivot = 4 };

RQ_DEV void raise_status(int64_t* status, int64_t bits) {
  if (status) __hip_atomic_fetch_or(status, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Upper bound on spin iterations of one wait (each iteration sleeps briefly and
// issues one device-coherent load, about 1 us), so a wait that can never finish
// ends in about a second with an error flag instead of hanging the device.
constexpr uint32_t kSpinLimit = 1u << 20;

// Cross-workgroup barrier for persistent kernels whose workgroups are all
// resident.  `counter` starts at 0 for the launch; barrier number `idx`
// (0-based) completes when the counter reaches nwg * (idx + 1).  Every
// workgroup calls it the same number of times with all of its threads.
// The workgroup first synchronizes internally (which orders its threads'
// global writes before thread 0's), then thread 0 alone performs the
// device-scope release, the arrival and the bounded wait, and one device-scope
// acquire before the workgroup proceeds.  With a single workgroup the internal
// synchronization is all that is needed.  Returns false when the wait timed out
// or another workgroup aborted; the caller must then leave the kernel.
RQ_DEV bool grid_barrier(uint32_t* counter, uint32_t* abort_flag, uint32_t nwg, uint32_t idx,
                         int64_t* status) {
  __shared__ int s_ok;
  __syncthreads();
  if (nwg == 1) return true;
  if (threadIdx.x == 0) {
    const uint32_t target = nwg * (idx + 1u);
    __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    uint32_t it = 0;
    while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
        ok = 0;
        break;
      }
      if (++it > kSpinLimit) {
        __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        raise_status(status, kErrTimeout);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    // later loads of data published by other workgroups must not hit stale lines
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// True when an earlier kernel of this handle already timed out: persistent
// kernels then leave at once instead of waiting again.
RQ_DEV bool prior_timeout(const int64_t* status) {
  return status && (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
                    kErrTimeout);
}

RQ_DEV double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// (value, position) maximum: larger value wins, equal values -> lower position.
// NaN values never win (comparisons with NaN are false).
RQ_DEV bool better(double v1, int p1, double v2, int p2) {
  return v1 > v2 || (v1 == v2 && p1 < p2);
}

RQ_DEV void wave_argmax(double& v, int& p, int& who) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    double v2 = __shfl_xor(v, o, kWave);
    int p2 = __shfl_xor(p, o, kWave);
    int w2 = __shfl_xor(who, o, kWave);
    if (better(v2, p2, v, p)) {
      v = v2;
      p = p2;
      who = w2;
    }
  }
}

typedef double dx4 __attribute__((ext_vector_type(4)));

// D(16x16) += A(16x4) * B(4x16), FP64 matrix core.  Lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; it holds D[l / 16 + 4 * i][l % 16]
// in element i of the accumulator (rows strided by 4, unlike the FP32 forms).
RQ_DEV dx4 mfma_f64(double a, double b, dx4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

}  // namespace rq
