// Partial QRCP of the (b+p) x N sample (the pivot block of Algorithms 3-5).
//
// Each sample column is held in registers by a group of Q lanes (8, or 4 for
// very wide samples) for the whole kernel: lane q of the group keeps rows q,
// q+Q, q+2Q, ... (ell <= 96, padded with zero rows), 1024 / Q columns per
// 1024-thread workgroup.  A pivot step needs
// the column of largest trailing 2-norm over all workgroups, so every step ends
// with one cross-workgroup exchange: each workgroup publishes its best
// (norm^2, position) and that column's values as a record (see the published
// records in device_common.hpp); once all records are in, every workgroup
// picks the same winner, forms the same Householder vector from the
// published column and applies it to its own columns.  Norms of rows j+1.. are
// recomputed from the transformed columns (no downdating).  Ties go to the
// lowest current position; positions follow the transpositions j <-> p_j.
#include "device_common.hpp"
#include "kernels.hpp"

namespace rq {

constexpr int kSqThreads = 1024;
constexpr int kSqWaves = kSqThreads / 64;
constexpr int kSpecCap = 8192;                 // doubles of LDS for the one-round candidate fetch
constexpr int kPoll = kSpecCap / kSqThreads;   // record words polled per thread

// Sum over the Q lanes holding one column.
template <int Q>
RQ_DEV double column_sum(double v) {
  v = quad_sum(v);
  if (Q == 8) v += dpp_f64<kDppHalfMirror>(v);
  return v;
}

template <int LM, int Q>
__global__ __launch_bounds__(kSqThreads) void sample_qrcp_kernel(SqArgs a) {
  constexpr int kQ = Q;                        // lanes per column
  constexpr int kSqCols = kSqThreads / kQ;     // columns per workgroup
  constexpr int RPL = LM / kQ;                 // rows per lane
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int q = t & (kQ - 1);
  const int cl = t / kQ;                       // local column
  const int wg = blockIdx.x;
  const int c = wg * kSqCols + cl;             // input position of the owned column
  const bool own = c < a.N;
  if (prior_timeout(a.status)) return;

  __shared__ double s_wv[kSqWaves];
  __shared__ int s_wp[kSqWaves], s_ww[kSqWaves];
  __shared__ double s_all[kSpecCap];
  __shared__ double s_v[kSqWaves][LM];         // each wave's copy of the reflector

  double x[RPL];
#pragma unroll
  for (int i = 0; i < RPL; ++i) {
    const int r = q + kQ * i;
    x[i] = (own && r < a.ell) ? canonical(a.B[r + (int64_t)c * a.ldb]) : 0.0;
  }
  double nu2;
  {
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      if (i & 1)
        s1 += x[i] * x[i];
      else
        s0 += x[i] * x[i];
    }
    nu2 = column_sum<kQ>(s0 + s1);
  }
  int pos = own ? c : INT_MAX;
  bool active = own;
  bool flagged = false;

  for (int j = 0; j < a.steps; ++j) {
    // ---- local best candidate: wave reduction, then every wave reduces the
    // 16 wave winners itself (no single-thread pass, no extra barrier) -------
    const bool lead = active && q == 0;
    double bv = lead ? nu2 : -1.0;
    int bp = lead ? pos : INT_MAX;
    int who = cl;
    if (lead && !flagged && !(nu2 <= 1.7976931348623157e308)) {
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
    {
      double v = (lane < kSqWaves) ? s_wv[lane] : -1.0;
      int p = (lane < kSqWaves) ? s_wp[lane] : INT_MAX;
      int w = (lane < kSqWaves) ? s_ww[lane] : 0;
      wave_argmax(v, p, w);
      const int owner = (p == INT_MAX) ? -1 : w;
      double* rec = a.rec + ((int64_t)j * a.nwg + wg) * a.rs;
      if (cl == owner) {
#pragma unroll
        for (int i = 0; i < RPL; ++i) publish(rec + 2 + q + kQ * i, x[i]);
      }
      if (owner < 0 && t < LM) publish(rec + 2 + t, 0.0);
      if (t == 0) {
        publish(rec, v);
        publish(rec + 1, (double)p);
      }
    }
    // ---- exchange: wait for every workgroup's record of this step -------------
    const double* rj = a.rec + (int64_t)j * a.nwg * a.rs;
    // all candidates (value, position) and, when they fit in LDS, their columns,
    // each thread polling up to kPoll words at once
    const bool spec = a.nwg * (LM + 2) <= kSpecCap;
    const int per = spec ? LM + 2 : 2;
    bool ok = true;
    {
      const int total = a.nwg * per;
      unsigned long long b[kPoll];
#pragma unroll
      for (int k = 0; k < kPoll; ++k) {
        const int e = t + k * kSqThreads;
        const int w = e / per, f = e - w * per;
        b[k] = (e < total) ? peek(rj + (int64_t)w * a.rs + f) : 0ull;
      }
      uint32_t it = 0;
      while (true) {
        bool all = true;
#pragma unroll
        for (int k = 0; k < kPoll; ++k) all = all && b[k] != kUnpublished;
        if (all) break;
        if (!keep_waiting(it, a.abort_flag, a.status)) {
          ok = false;
          break;
        }
#pragma unroll
        for (int k = 0; k < kPoll; ++k) {
          const int e = t + k * kSqThreads;
          const int w = e / per, f = e - w * per;
          if (e < total && b[k] == kUnpublished) b[k] = peek(rj + (int64_t)w * a.rs + f);
        }
      }
#pragma unroll
      for (int k = 0; k < kPoll; ++k) {
        const int e = t + k * kSqThreads;
        if (e < total) s_all[e] = __longlong_as_double((long long)b[k]);
      }
    }
    if (__syncthreads_or(!ok)) return;
    // every wave finds the same winner and forms the same reflector
    int wwg = 0, wpos;
    {
      double v = -1.0;
      int p = INT_MAX, w = 0;
      for (int i = lane; i < a.nwg; i += 64) {
        const double vi = s_all[i * per];
        const int pi = (int)s_all[i * per + 1];
        if (better(vi, pi, v, p)) {
          v = vi;
          p = pi;
          w = i;
        }
      }
      wave_argmax(v, p, w);
      wpos = p;
      wwg = w;
    }
    if (wpos == INT_MAX) {          // every workgroup sees the same: consistent exit
      if (t == 0 && wg == 0) raise_status(a.status, kErrNoPivot);
      return;
    }
    if (!spec) {
      // columns did not fit: fetch the winner's column into the front of s_all
      __syncthreads();
      if (t < LM) {
        const double* src = rj + (int64_t)wwg * a.rs + 2 + t;
        unsigned long long bt = peek(src);
        uint32_t it = 0;
        while (bt == kUnpublished) {
          if (!keep_waiting(it, a.abort_flag, a.status)) {
            ok = false;
            break;
          }
          bt = peek(src);
        }
        s_all[2 + t] = __longlong_as_double((long long)bt);
      }
      if (__syncthreads_or(!ok)) return;
      wwg = 0;
    }
    const double* col = s_all + (spec ? wwg * (LM + 2) : 0) + 2;   // winner's column in LDS
    double s2 = 0.0;
    if (lane >= j && lane < LM) s2 += col[lane] * col[lane];
    if (lane + 64 >= j && lane + 64 < LM) s2 += col[lane + 64] * col[lane + 64];
    s2 = wave_sum(s2);
    const double alpha = col[j];
    double beta = 0.0, tau = 0.0, scale = 0.0;
    if (s2 > 0.0) {
      reflector_coeffs(alpha, s2, beta, scale, tau);
    }
    // ---- positions: j <-> wpos ----------------------------------------------
    if (active) {
      if (pos == wpos) {
        pos = j;
        active = false;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
          const int r = q + kQ * i;
          x[i] = (r < j) ? x[i] : (r == j ? beta : 0.0);
        }
      } else if (pos == j) {
        pos = wpos;
      }
    }
    // ---- apply the reflection to the remaining columns ---------------------------
    // Each wave writes the reflector once into its own LDS row and reads it back
    // (LDS operations of one wave complete in order; no workgroup barrier).
    for (int r = lane; r < LM; r += 64) s_v[wave][r] = (r < j) ? 0.0 : (r == j ? 1.0 : col[r] * scale);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (active) {
      double v[RPL];
      double d0 = 0.0, d1 = 0.0;
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        v[i] = s_v[wave][q + kQ * i];
        if (i & 1)
          d1 += v[i] * x[i];
        else
          d0 += v[i] * x[i];
      }
      const double d = tau * column_sum<kQ>(d0 + d1);
      double n0 = 0.0, n1 = 0.0;
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        x[i] -= d * v[i];
        const double sq = (q + kQ * i > j) ? x[i] * x[i] : 0.0;
        if (i & 1)
          n1 += sq;
        else
          n0 += sq;
      }
      nu2 = column_sum<kQ>(n0 + n1);
    }
    // No barrier here: the next step rewrites s_wv only after this step's
    // __syncthreads_or (which follows every read of s_wv), and s_all only after
    // its own first barrier (which follows this step's last read of s_all);
    // s_v belongs to one wave.
  }
  // Every workgroup loaded its columns before the first barrier, so the
  // in-place write of the permuted sample cannot overwrite unread input.
  if (own) {
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
      const int r = q + kQ * i;
      if (r < a.ell) a.B[r + (int64_t)pos * a.ldb] = x[i];
    }
    if (q == 0) {
      if (a.src_top && pos < a.steps) a.src_top[pos] = c;
      if (a.dst_low && c < a.steps) a.dst_low[c] = (pos >= a.steps) ? pos : -1;
      if (a.perm) a.perm[pos] = c;
    }
  }
}

int sq_lm(int ell) {
  if (ell <= 0 || ell > 96) return 0;
  return ((ell + 7) / 8) * 8;
}

int sq_record_stride(int lm) { return ((lm + 2 + 7) / 8) * 8; }

// Every workgroup of the persistent kernel must be resident at once, so the
// wider layout (8 lanes per column, twice the workgroups) is used only within
// the caller's workgroup allowance.
int sq_groups(int64_t N, int max_groups) {
  const int64_t g8 = (N + 127) / 128;
  return (int)(g8 <= max_groups ? g8 : (N + 255) / 256);
}

int sq_max_groups(int64_t N) { return (int)((N + 127) / 128); }

template <int LM>
static hipError_t launch_lm(const SqArgs& a, hipStream_t s) {
  // the layout follows from the workgroup count chosen by sq_groups
  const bool wide = (int64_t)a.nwg * 128 >= a.N;
  if (a.nwg < 1 || (int64_t)a.nwg * 256 < a.N) return hipErrorInvalidValue;
  if (wide)
    hipLaunchKernelGGL((sample_qrcp_kernel<LM, 8>), dim3(a.nwg), dim3(kSqThreads), 0, s, a);
  else
    hipLaunchKernelGGL((sample_qrcp_kernel<LM, 4>), dim3(a.nwg), dim3(kSqThreads), 0, s, a);
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
