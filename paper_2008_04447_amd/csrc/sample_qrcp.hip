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
// Work that is the same for the whole workgroup (its record, the winner, the
// reflector's coefficients) is done by wave 0 alone and shared through LDS: with
// four waves per SIMD, repeating it in every wave would cost four times its
// latency on every step.
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
  __shared__ int s_wp[kSqWaves];
  __shared__ double s_cand[kSqWaves][LM];      // each wave's best column
  __shared__ double s_all[kSpecCap];
  __shared__ double s_hh[3];                   // beta, scale, tau of the step's reflector
  __shared__ int s_hp[2];                      // winner position, its record (-2: timed out)

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

  // Record words this thread polls in every step: all candidates (value,
  // position) and, when they fit in LDS, their columns.  The offsets within a
  // step's records are the same for every step.
  const bool spec = a.nwg * (LM + 2) <= kSpecCap;
  const int per = spec ? LM + 2 : 2;
  const int total = a.nwg * per;
  int off[kPoll];
#pragma unroll
  for (int k = 0; k < kPoll; ++k) {
    const int e = t + k * kSqThreads;
    const int w = e / per, f = e - w * per;
    off[k] = (e < total) ? w * a.rs + f : -1;
  }

  for (int j = 0; j < a.steps; ++j) {
    // ---- each wave's best column (its values go to LDS) ---------------------
    const bool lead = active && q == 0;
    double bv = lead ? nu2 : -1.0;
    int bp = lead ? pos : INT_MAX;
    int who = cl;
    if (lead && !flagged && !(nu2 <= 1.7976931348623157e308)) {
      raise_status(a.status, kErrNonFinite);
      flagged = true;
    }
    wave_argmax(bv, bp, who);
    if (bp != INT_MAX && cl == who) {
#pragma unroll
      for (int i = 0; i < RPL; ++i) s_cand[wave][q + kQ * i] = x[i];
    }
    if (lane == 0) {
      s_wv[wave] = bv;
      s_wp[wave] = bp;
    }
    __syncthreads();
    // ---- wave 0 publishes the workgroup's record; the other waves go straight
    // to polling (one wave doing this keeps the SIMDs free of repeated work)
    if (wave == 0) {
      double v = (lane < kSqWaves) ? s_wv[lane] : -1.0;
      int p = (lane < kSqWaves) ? s_wp[lane] : INT_MAX;
      int w = lane;
      wave_argmax(v, p, w);
      double* rec = a.rec + ((int64_t)j * a.nwg + wg) * a.rs;
      if (p != INT_MAX) {
        for (int r = lane; r < LM; r += 64) publish(rec + 2 + r, s_cand[w][r]);
      } else {
        for (int r = lane; r < LM; r += 64) publish(rec + 2 + r, 0.0);
      }
      if (lane == 0) {
        publish(rec, v);
        publish(rec + 1, (double)p);
      }
    }
    // ---- exchange: wait for every workgroup's record of this step -------------
    const double* rj = a.rec + (int64_t)j * a.nwg * a.rs;
    bool ok = true;
    {
      unsigned long long b[kPoll];
#pragma unroll
      for (int k = 0; k < kPoll; ++k) b[k] = (off[k] >= 0) ? peek(rj + off[k]) : 0ull;
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
        for (int k = 0; k < kPoll; ++k)
          if (off[k] >= 0 && b[k] == kUnpublished) b[k] = peek(rj + off[k]);
      }
#pragma unroll
      for (int k = 0; k < kPoll; ++k) {
        const int e = t + k * kSqThreads;
        if (e < total) s_all[e] = __longlong_as_double((long long)b[k]);
      }
    }
    if (__syncthreads_or(!ok)) return;
    // ---- wave 0 finds the winner and forms its reflector; the others wait -----
    if (wave == 0) {
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
      bool okc = true;
      if (p != INT_MAX && !spec) {
        // columns did not fit: fetch the winner's column into the front of s_all
        for (int r = lane; r < LM && okc; r += 64) {
          const double* src = rj + (int64_t)w * a.rs + 2 + r;
          unsigned long long bt = peek(src);
          uint32_t it = 0;
          while (bt == kUnpublished) {
            if (!keep_waiting(it, a.abort_flag, a.status)) {
              okc = false;
              break;
            }
            bt = peek(src);
          }
          s_all[2 + r] = __longlong_as_double((long long)bt);
        }
        w = 0;
        // lane 0 reads words other lanes of this wave wrote
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      const bool wave_ok = __builtin_amdgcn_ballot_w64(!okc) == 0;
      if (lane == 0) {
        s_hp[0] = p;
        s_hp[1] = wave_ok ? w : -2;
        if (p != INT_MAX && wave_ok) {
          // the winner's value is the sum of squares of its rows j.., exactly
          // the s2 its reflector needs
          const double alpha = s_all[(spec ? w * (LM + 2) : 0) + 2 + j];
          double beta = 0.0, tau = 0.0, scale = 0.0;
          if (v > 0.0) reflector_coeffs(alpha, v, beta, scale, tau);
          s_hh[0] = beta;
          s_hh[1] = scale;
          s_hh[2] = tau;
        }
      }
    }
    __syncthreads();
    const int wpos = s_hp[0], wwg = s_hp[1];
    if (wpos == INT_MAX) {          // every workgroup sees the same: consistent exit
      if (t == 0 && wg == 0) raise_status(a.status, kErrNoPivot);
      return;
    }
    if (wwg < 0) return;            // the winner's column never arrived (status raised)
    const double beta = s_hh[0], scale = s_hh[1], tau = s_hh[2];
    const double* col = s_all + (spec ? wwg * (LM + 2) : 0) + 2;   // winner's column in LDS
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
    // The Householder vector is formed on the fly from the winner's column in LDS
    // (every lane of a column group reads the same words: broadcast reads).
    if (active) {
      double v[RPL];
      double d0 = 0.0, d1 = 0.0;
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const int r = q + kQ * i;
        v[i] = (r < j) ? 0.0 : (r == j ? 1.0 : col[r] * scale);
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
    // No barrier here: the next step rewrites s_wv, s_wp and s_cand only after
    // this step's barriers (wave 0 read them before the first), s_all only
    // after its own first barrier (which follows this step's last read of
    // s_all), and s_hh, s_hp only after its own poll barrier.
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
