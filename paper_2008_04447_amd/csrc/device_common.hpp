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

// Cross-workgroup barrier for kernels whose workgroups are all resident.  Each
// of the nwg workgroups adds one arrival to `counter` and the barrier completes
// when the counter reaches `target`: the caller keeps count of the arrivals of
// earlier barriers on the same counter (zeroed once before the first), so
// consecutive launches need no reset in between.  A single workgroup neither
// arrives nor waits.  Every workgroup calls it with all of its threads.
// The workgroup first synchronizes internally (which orders its threads'
// global writes before thread 0's), then thread 0 alone performs the
// device-scope release, the arrival and the bounded wait, and one device-scope
// acquire before the workgroup proceeds.  With a single workgroup the internal
// synchronization is all that is needed.  Returns false when the wait timed out
// or another workgroup aborted; the caller must then leave the kernel.
RQ_DEV bool grid_barrier(uint32_t* counter, uint32_t* abort_flag, uint32_t nwg, uint32_t target,
                         int64_t* status) {
  __shared__ int s_ok;
  __syncthreads();
  if (nwg == 1) return true;
  if (threadIdx.x == 0) {
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

// ---- published records (persistent-kernel exchange without a barrier) -------
// Each workgroup publishes its per-step record into a slot of its own for that
// step, which holds a sentinel until then (written by a kernel that ran
// before), and readers wait on the record words themselves: one round trip
// through device-coherent memory both synchronizes and delivers the data, and
// as no slot is reused within a launch, no fence or reset is needed.  The
// sentinel is a signalling-NaN bit pattern, which arithmetic never produces
// (it quiets NaNs); kernels canonicalize NaNs they copy from inputs.
constexpr unsigned long long kUnpublished = 0x7FF4DEADBEEF0001ull;

RQ_DEV void publish(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<unsigned long long*>(p),
                     (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}

RQ_DEV unsigned long long peek(const double* p) {
  return __hip_atomic_load(reinterpret_cast<const unsigned long long*>(p), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

RQ_DEV double canonical(double v) { return (v != v) ? __builtin_nan("") : v; }

// 1/sqrt(d) and 1/u for d > 0, u != 0 from the hardware estimates refined by
// one Newton step: a few dependent operations instead of the long IEEE sqrt
// and divide sequences, on the serial chains of the pivot and panel steps.
// Every workgroup runs the same sequence, so all derive the same bits.
RQ_DEV double rsqrt_nr(double d) {
  const double y = __builtin_amdgcn_rsq(d);
  return y * fma(-0.5 * d * y, y, 1.5);
}
RQ_DEV double rcp_nr(double u) {
  const double y = __builtin_amdgcn_rcp(u);
  return y * fma(-u, y, 2.0);
}

// Reflector of a column with leading entry alpha and squared 2-norm s2 > 0
// (Section 2): beta = -sign(alpha) sqrt(s2) with sign(0) = +1, the tail scale
// 1 / (alpha - beta) and tau = (beta - alpha) / beta.
RQ_DEV void reflector_coeffs(double alpha, double s2, double& beta, double& scale, double& tau) {
  const double r = rsqrt_nr(s2);
  const double sn = s2 * r;
  beta = (alpha >= 0.0) ? -sn : sn;
  scale = rcp_nr(alpha - beta);
  tau = (beta - alpha) * ((alpha >= 0.0) ? -r : r);
}

// One bounded wait iteration: false (and the abort flag set) once the wait has
// lasted kSpinLimit polls or another workgroup aborted (checked every 64 polls,
// so the common short wait costs no extra round trip).
RQ_DEV bool keep_waiting(uint32_t& it, uint32_t* abort_flag, int64_t* status) {
  if ((it & 63u) == 63u &&
      __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    return false;
  if (++it > kSpinLimit) {
    __hip_atomic_store(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    raise_status(status, kErrTimeout);
    return false;
  }
  __builtin_amdgcn_s_sleep(1);
  return true;
}

// True when an earlier kernel of this handle already timed out: persistent
// kernels then leave at once instead of waiting again.
RQ_DEV bool prior_timeout(const int64_t* status) {
  return status && (__hip_atomic_load(status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
                    kErrTimeout);
}

// (value, position) maximum: larger value wins, equal values -> lower position.
// NaN values never win (comparisons with NaN are false).
RQ_DEV bool better(double v1, int p1, double v2, int p2) {
  return v1 > v2 || (v1 == v2 && p1 < p2);
}

// ---- cross-lane reductions ----------------------------------------------------
// Built from DPP row moves (quad_perm, row_half_mirror, row_mirror), which read
// a neighbour's register directly instead of going through the LDS crossbar,
// and v_readlane across the four rows of 16 lanes.  Every lane of the group
// combined must be active.  Each stage pairs lanes symmetrically and addition
// is commutative, so every lane of the group ends with bitwise the same value.
constexpr int kDppXor1 = 0xB1;         // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;  // lane i <-> 7 - i within 8 lanes
constexpr int kDppMirror = 0x140;      // lane i <-> 15 - i within 16 lanes

template <int kCtrl>
RQ_DEV int dpp_i32(int v) {
  // every control used here reads a lane of the same row, so no lane keeps an
  // old value and none needs to be supplied
  return __builtin_amdgcn_mov_dpp(v, kCtrl, 0xF, 0xF, true);
}

template <int kCtrl>
RQ_DEV double dpp_f64(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)dpp_i32<kCtrl>((int)(unsigned)b);
  const unsigned hi = (unsigned)dpp_i32<kCtrl>((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

RQ_DEV double readlane_f64(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over the 4 lanes of a quad.
RQ_DEV double quad_sum(double v) {
  v += dpp_f64<kDppXor1>(v);
  v += dpp_f64<kDppXor2>(v);
  return v;
}

// Sum over a row of 16 lanes (lanes 16r .. 16r + 15).
RQ_DEV double row16_sum(double v) {
  v = quad_sum(v);
  v += dpp_f64<kDppHalfMirror>(v);
  v += dpp_f64<kDppMirror>(v);
  return v;
}

// Sum over the wave; the result is wave-uniform.
RQ_DEV double wave_sum(double v) {
  v = row16_sum(v);
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

template <int kCtrl>
RQ_DEV void argmax_step(double& v, int& p, int& who) {
  const double v2 = dpp_f64<kCtrl>(v);
  const int p2 = dpp_i32<kCtrl>(p);
  const int w2 = dpp_i32<kCtrl>(who);
  if (better(v2, p2, v, p)) {
    v = v2;
    p = p2;
    who = w2;
  }
}

// Wave-wide (value, position) maximum with a payload `who`; every lane gets
// the winner.  Positions of real candidates are distinct, so the winner does
// not depend on the order in which candidates meet.  When every aligned group
// of G lanes (G = 1, 2, 4 or 8) already holds one candidate, the DPP stages
// inside a group would compare equal candidates and are left out.
template <int G>
RQ_DEV void group_wave_argmax(double& v, int& p, int& who) {
  static_assert(G == 1 || G == 2 || G == 4 || G == 8, "group of 1, 2, 4 or 8 lanes");
  if (G < 2) argmax_step<kDppXor1>(v, p, who);
  if (G < 4) argmax_step<kDppXor2>(v, p, who);
  if (G < 8) argmax_step<kDppHalfMirror>(v, p, who);
  argmax_step<kDppMirror>(v, p, who);
  double bv = readlane_f64(v, 0);
  int bp = __builtin_amdgcn_readlane(p, 0), bw = __builtin_amdgcn_readlane(who, 0);
#pragma unroll
  for (int r = 16; r < 64; r += 16) {
    const double v2 = readlane_f64(v, r);
    const int p2 = __builtin_amdgcn_readlane(p, r), w2 = __builtin_amdgcn_readlane(who, r);
    if (better(v2, p2, bv, bp)) {
      bv = v2;
      bp = p2;
      bw = w2;
    }
  }
  v = bv;
  p = bp;
  who = bw;
}

RQ_DEV void wave_argmax(double& v, int& p, int& who) { group_wave_argmax<1>(v, p, who); }

// The same maximum when only lanes 0..15 hold candidates: the four stages
// inside the first row of 16 lanes, then lane 0's result to every lane.
RQ_DEV void row0_argmax(double& v, int& p, int& who) {
  argmax_step<kDppXor1>(v, p, who);
  argmax_step<kDppXor2>(v, p, who);
  argmax_step<kDppHalfMirror>(v, p, who);
  argmax_step<kDppMirror>(v, p, who);
  v = readlane_f64(v, 0);
  p = __builtin_amdgcn_readlane(p, 0);
  who = __builtin_amdgcn_readlane(who, 0);
}

typedef double dx4 __attribute__((ext_vector_type(4)));

// D(16x16) += A(16x4) * B(4x16), FP64 matrix core.  Lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; it holds D[l / 16 + 4 * i][l % 16]
// in element i of the accumulator (rows strided by 4, unlike the FP32 forms).
RQ_DEV dx4 mfma_f64(double a, double b, dx4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

}  // namespace rq
