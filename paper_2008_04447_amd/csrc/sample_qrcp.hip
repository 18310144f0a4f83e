// Partial QRCP of the (b+p) x N sample (the pivot block of Algorithms 3-5).
//
// Each of the N sample columns lives in the registers of one lane for the whole
// kernel (ell <= 96 values, padded with zero rows).  A pivot step needs the
// column of largest trailing 2-norm over all workgroups, so every step ends
// with one cross-workgroup exchange: each workgroup publishes its best
// (norm^2, position) and that column's values; after the barrier every
// workgroup picks the same winner, forms the same Householder vector from the
// published column and applies it to its own columns.  Norms of rows j+1.. are
// recomputed from the transformed columns (no downdating).  Ties go to the
// lowest current position; positions follow the transpositions j <-> p_j.
#include "device_common.hpp"
#include "kernels.hpp"

namespace rq {

constexpr int kSqThreads = 256;

template <int LM>
__global__ __launch_bounds__(kSqThreads) void sample_qrcp_kernel(SqArgs a) {
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int wg = blockIdx.x;
  const int c = wg * kSqThreads + t;   // input position of the owned column
  const bool own = c < a.N;
  if (prior_timeout(a.status)) return;

  __shared__ double s_v[LM];
  __shared__ double s_col[LM];
  __shared__ double s_wv[4];
  __shared__ int s_wp[4], s_ww[4];
  __shared__ double s_cv[kSqThreads];
  __shared__ int s_cp[kSqThreads];
  __shared__ double s_tau, s_beta, s_best;
  __shared__ int s_owner, s_bestpos, s_winwg, s_winpos;

  double x[LM];
#pragma unroll
  for (int r = 0; r < LM; ++r) x[r] = (own && r < a.ell) ? a.B[r + (int64_t)c * a.ldb] : 0.0;
  double nu2 = 0.0;
#pragma unroll
  for (int r = 0; r < LM; ++r) nu2 += x[r] * x[r];
  int pos = own ? c : INT_MAX;
  bool active = own;
  bool flagged = false;

  for (int j = 0; j < a.steps; ++j) {
    // ---- local best candidate --------------------------------------------
    double bv = active ? nu2 : -1.0;
    int bp = active ? pos : INT_MAX;
    int who = t;
    if (active && !flagged && !(nu2 <= 1.7976931348623157e308)) {
      raise_status(a.status, kErrNonFinite);
      flagged = true;
    }
    wave_argmax(bv, bp, who);
    if (lane == 0) {
      s_wv[wave] = bv;
      s_wp[wave] = bp;
      s_ww[wave] = who;
    }
    __syncthreads();
    if (t == 0) {
      double v = s_wv[0];
      int p = s_wp[0], w = s_ww[0];
      for (int q = 1; q < 4; ++q)
        if (better(s_wv[q], s_wp[q], v, p)) {
          v = s_wv[q];
          p = s_wp[q];
          w = s_ww[q];
        }
      s_best = v;
      s_bestpos = p;
      s_owner = (p == INT_MAX) ? -1 : w;
    }
    __syncthreads();
    if (t == s_owner) {
#pragma unroll
      for (int r = 0; r < LM; ++r) s_col[r] = x[r];
    }
    __syncthreads();
    double* rec = a.rec + ((int64_t)(j & 1) * a.nwg + wg) * a.rs;
    if (t < LM) rec[2 + t] = (s_owner >= 0) ? s_col[t] : 0.0;
    if (t == 0) {
      rec[0] = s_best;
      rec[1] = (double)s_bestpos;
    }
    // ---- exchange ----------------------------------------------------------
    if (!grid_barrier(a.counter, a.abort_flag, (uint32_t)a.nwg, (uint32_t)j, a.status)) return;
    const double* rj = a.rec + (int64_t)(j & 1) * a.nwg * a.rs;
    if (t < a.nwg) {
      s_cv[t] = rj[(int64_t)t * a.rs];
      s_cp[t] = (int)rj[(int64_t)t * a.rs + 1];
    } else {
      s_cv[t] = -1.0;
      s_cp[t] = INT_MAX;
    }
    __syncthreads();
    if (wave == 0) {
      double v = s_cv[lane];
      int p = s_cp[lane];
      int w = lane;
#pragma unroll
      for (int q = 1; q < kSqThreads / 64; ++q) {
        const int i = lane + 64 * q;
        if (better(s_cv[i], s_cp[i], v, p)) {
          v = s_cv[i];
          p = s_cp[i];
          w = i;
        }
      }
      wave_argmax(v, p, w);
      if (lane == 0) {
        s_winpos = p;
        s_winwg = w;
      }
    }
    __syncthreads();
    const int wpos = s_winpos;
    if (wpos == INT_MAX) {          // every workgroup sees the same: consistent exit
      if (t == 0 && wg == 0) raise_status(a.status, kErrNoPivot);
      return;
    }
    if (t < LM) s_col[t] = rj[(int64_t)s_winwg * a.rs + 2 + t];
    __syncthreads();
    // ---- Householder vector of the winner (wave 0) ----------------------------
    if (wave == 0) {
      double s2 = 0.0;
      if (lane >= j && lane < LM) s2 += s_col[lane] * s_col[lane];
      if (lane + 64 >= j && lane + 64 < LM) s2 += s_col[lane + 64] * s_col[lane + 64];
      s2 = wave_sum(s2);
      const double alpha = s_col[j];
      double beta = 0.0, tau = 0.0, scale = 0.0;
      if (s2 > 0.0) {
        const double sn = sqrt(s2);
        beta = (alpha >= 0.0) ? -sn : sn;
        scale = 1.0 / (alpha - beta);
        tau = (beta - alpha) / beta;
      }
      for (int r = lane; r < LM; r += 64) s_v[r] = (r < j) ? 0.0 : (r == j ? 1.0 : s_col[r] * scale);
      if (lane == 0) {
        s_tau = tau;
        s_beta = beta;
      }
    }
    __syncthreads();
    const double tau = s_tau;
    // ---- positions: j <-> wpos ----------------------------------------------
    if (active) {
      if (pos == wpos) {
        const double beta = s_beta;
        pos = j;
        active = false;
#pragma unroll
        for (int r = 0; r < LM; ++r) x[r] = (r < j) ? x[r] : (r == j ? beta : 0.0);
      } else if (pos == j) {
        pos = wpos;
      }
    }
    // ---- apply the reflection to the remaining columns ---------------------------
    if (active) {
      double d = 0.0;
#pragma unroll
      for (int r = 0; r < LM; ++r) d += s_v[r] * x[r];
      d *= tau;
      // re-read v from LDS rather than keeping a second LM-long register copy
      const volatile double* vv = s_v;
#pragma unroll
      for (int r = 0; r < LM; ++r) x[r] -= d * vv[r];
      nu2 = 0.0;
#pragma unroll
      for (int r = 0; r < LM; ++r) nu2 += (r > j) ? x[r] * x[r] : 0.0;
    }
    __syncthreads();   // s_v / s_col are rewritten in the next step
  }
  // Every workgroup loaded its columns before the first barrier, so the
  // in-place write of the permuted sample cannot overwrite unread input.
  if (own) {
#pragma unroll
    for (int r = 0; r < LM; ++r)
      if (r < a.ell) a.B[r + (int64_t)pos * a.ldb] = x[r];
    if (a.src_top && pos < a.steps) a.src_top[pos] = c;
    if (a.dst_low && c < a.steps) a.dst_low[c] = (pos >= a.steps) ? pos : -1;
    if (a.perm) a.perm[pos] = c;
  }
}

int sq_lm(int ell) {
  if (ell <= 0 || ell > 96) return 0;
  return ((ell + 7) / 8) * 8;
}

int sq_record_stride(int lm) { return ((lm + 2 + 7) / 8) * 8; }

template <int LM>
static hipError_t launch_lm(const SqArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(sample_qrcp_kernel<LM>, dim3(a.nwg), dim3(kSqThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sample_qrcp(const SqArgs& a, int lm, hipStream_t s) {
  switch (lm) {
    case 8: return launch_lm<8>(a, s);
    case 16: return launch_lm<16>(a, s);
    case 24: return launch_lm<24>(a, s);
    case 32: return launch_lm<32>(a, s);
    case 40: return launch_lm<40>(a, s);
    case 48: return launch_lm<48>(a, s);
    case 56: return launch_lm<56>(a, s);
    case 64: return launch_lm<64>(a, s);
    case 72: return launch_lm<72>(a, s);
    case 80: return launch_lm<80>(a, s);
    case 88: return launch_lm<88>(a, s);
    case 96: return launch_lm<96>(a, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rq
