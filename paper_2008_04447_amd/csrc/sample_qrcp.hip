// Partial QRCP of the (b+p) x N sample (the pivot block of Algorithms 3-5).
//
// Each sample column is held in registers by a group of Q = 4 lanes for the
// whole kernel: lane q of the group keeps rows q, q+4, q+8, ... (ell <= 96,
// padded with zero rows); a workgroup of 256 threads holds 64 columns (one
// wave per SIMD), or of 512 or 1024 threads 128 or 256 columns when the
// launch's workgroup allowance calls for fewer, wider workgroups (the
// reflection is issue-bound: waves that share a SIMD queue behind each other on
// every step).  A pivot step needs the column of largest trailing
// 2-norm over all workgroups, so every step has one cross-workgroup exchange:
// each workgroup publishes a record for its best column (see the published
// records in device_common.hpp) holding (norm^2, position, tau, beta) and the
// Householder vector that column would define.  Every workgroup polls the
// heads (norm^2, position) of all records, which go out first, finds the
// winner and then reads that one record's tau, beta and vector, so the step
// moves two round trips of small reads (fetching every record whole in one
// round trip moved 40 KB per workgroup and step and measured slower).  Norms
// of rows j+1.. are recomputed from the transformed columns (no downdating).
// Ties go to the lowest current position; positions follow the
// transpositions j <-> p_j.
//
// Work that is the same for the whole workgroup (its record, the winner) is
// done by wave 0 alone: with several waves per SIMD, repeating it in every
// wave would cost several times its latency on every step.
#include <algorithm>

#include "device_common.hpp"
#include "kernels.hpp"
#include "rqrcp.h"

namespace rq {

constexpr int kHead = 4;                        // record words besides the vector: norm^2, position, tau, beta
constexpr int kHeadPer = 4;                     // record heads one lane of wave 0 polls

template <int NT>
struct SqShape {
  static constexpr int kWaves = NT / 64;
};
static_assert(kHeadPer * 64 >= RQ_MAX_N / 256, "every workgroup's head is polled");

// Sum over the Q lanes holding one column.
template <int Q>
RQ_DEV double column_sum(double v) {
  v = quad_sum(v);
  if (Q == 8) v += dpp_f64<kDppHalfMirror>(v);
  return v;
}

// Wave 0: the winner (norm^2 v, position p, workgroup w) over the heads of all
// records of a step; lane l polls the records l, l + 64, ....  Returns this
// lane's wait status; the result is wave-uniform.
RQ_DEV bool poll_winner(const double* rj, const SqArgs& a, int lane, double& v, int& p, int& w) {
  unsigned long long hv[kHeadPer], hp[kHeadPer];
#pragma unroll
  for (int k = 0; k < kHeadPer; ++k) {
    const int g = lane + 64 * k;
    hv[k] = (g < a.nwg) ? peek(rj + 2 * g) : 0ull;
    hp[k] = (g < a.nwg) ? peek(rj + 2 * g + 1) : 0ull;
  }
  bool ok = true;
  uint32_t it = 0;
  while (true) {
    bool all = true;
#pragma unroll
    for (int k = 0; k < kHeadPer; ++k) all = all && hv[k] != kUnpublished && hp[k] != kUnpublished;
    if (all) break;
    if (!keep_waiting(it, a.abort_flag, a.status)) {
      ok = false;
      break;
    }
#pragma unroll
    for (int k = 0; k < kHeadPer; ++k) {
      const int g = lane + 64 * k;
      if (g < a.nwg && hv[k] == kUnpublished) hv[k] = peek(rj + 2 * g);
      if (g < a.nwg && hp[k] == kUnpublished) hp[k] = peek(rj + 2 * g + 1);
    }
  }
  v = -1.0;
  p = INT_MAX;
  w = 0;
#pragma unroll
  for (int k = 0; k < kHeadPer; ++k) {
    const int g = lane + 64 * k;
    if (ok && g < a.nwg) {
      const double vk = __longlong_as_double((long long)hv[k]);
      const int pk = (int)__longlong_as_double((long long)hp[k]);
      if (better(vk, pk, v, p)) {
        v = vk;
        p = pk;
        w = g;
      }
    }
  }
  wave_argmax(v, p, w);
  return ok;
}

// The release word (optional) tells a stream waiting on it that every
// workgroup holds its compute unit: workgroup 0 sets it once the first step's
// heads are all in, and again on its way out, so that a wait on it ends
// whatever path the kernel takes.
RQ_DEV void sq_release(const SqArgs& a) {
  __hip_atomic_store(a.release, a.release_value, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <int LM, int Q, int NT>
RQ_DEV void sample_qrcp_body(const SqArgs& a) {
  constexpr int kQ = Q;                        // lanes per column
  constexpr int kSqCols = NT / kQ;             // columns per workgroup
  constexpr int kSqWaves = SqShape<NT>::kWaves;
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
  __shared__ double s_rec[kHead + LM];         // the winner's record (words 2..)
  __shared__ int s_hp;                         // winner position

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
    // ---- each wave's best column (its values go to LDS) ---------------------
    // All kQ lanes of a column hold bitwise the same norm (see column_sum), so
    // the wave maximum skips the stages inside a column group.
    double bv = active ? nu2 : -1.0;
    int bp = active ? pos : INT_MAX;
    int who = cl;
    if (active && q == 0 && !flagged && !(nu2 <= 1.7976931348623157e308)) {
      raise_status(a.status, kErrNonFinite);
      flagged = true;
    }
    group_wave_argmax<kQ>(bv, bp, who);
    if (bp != INT_MAX && cl == who) {
#pragma unroll
      for (int i = 0; i < RPL; ++i) s_cand[wave][q + kQ * i] = x[i];
    }
    if (lane == 0) {
      s_wv[wave] = bv;
      s_wp[wave] = bp;
    }
    __syncthreads();
    double* rj = a.rec + (int64_t)j * a.nwg * a.rs;   // this step's area
    bool ok = true;
    if (wave == 0) {
      // ---- the workgroup's best column and its reflector, published --------
      // The head (norm^2, position), which every workgroup polls to find the
      // winner, goes out first; tau, beta and the vector follow while the
      // other records are still arriving (only the winner's are read).
      double v = (lane < kSqWaves) ? s_wv[lane] : -1.0;
      int p = (lane < kSqWaves) ? s_wp[lane] : INT_MAX;
      int w = lane;
      row0_argmax(v, p, w);
      double* head = rj + 2 * wg;
      double* body = rj + 2 * a.nwg + (int64_t)wg * (a.rs - 2);
      if (lane == 0) {
        publish(head, v);
        publish(head + 1, (double)p);
      }
      double beta = 0.0, scale = 0.0, tau = 0.0;
      if (p != INT_MAX) {
        // v is the sum of squares of the column's rows j.., the s2 of its reflector
        if (v > 0.0) reflector_coeffs(s_cand[w][j], v, beta, scale, tau);
        for (int r = lane; r < LM; r += 64)
          publish(body + 2 + r, (r < j) ? 0.0 : (r == j ? 1.0 : s_cand[w][r] * scale));
      } else {
        for (int r = lane; r < LM; r += 64) publish(body + 2 + r, 0.0);
      }
      if (lane == 0) {
        publish(body, tau);
        publish(body + 1, beta);
      }
      // ---- the winner over all workgroups, from the record heads ----------
      double wv;
      int wp, ww;
      ok = poll_winner(rj, a, lane, wv, wp, ww);
      if (j == 0 && wg == 0 && lane == 0 && ok && a.release) sq_release(a);
      if (__builtin_amdgcn_ballot_w64(!ok) == 0 && wp != INT_MAX) {
        // fetch the winner's tau, beta and vector (words 2.. of its record)
        for (int r = 2 + lane; r < a.rs && ok; r += 64) {
          const double* src = rj + 2 * a.nwg + (int64_t)ww * (a.rs - 2) + (r - 2);
          unsigned long long bt = peek(src);
          uint32_t it = 0;
          while (bt == kUnpublished) {
            if (!keep_waiting(it, a.abort_flag, a.status)) {
              ok = false;
              break;
            }
            bt = peek(src);
          }
          s_rec[r] = __longlong_as_double((long long)bt);
        }
      }
      if (lane == 0) s_hp = wp;
    }
    if (__syncthreads_or(!ok)) return;
    const int wpos = s_hp;
    if (wpos == INT_MAX) {          // every workgroup sees the same: consistent exit
      if (t == 0 && wg == 0) raise_status(a.status, kErrNoPivot);
      return;
    }
    const double tau = s_rec[2], beta = s_rec[3];
    const double* vh = s_rec + kHead;                           // the winner's Householder vector
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
    if (active) {
      double d0 = 0.0, d1 = 0.0;
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        const double vi = vh[q + kQ * i];
        if (i & 1)
          d1 += vi * x[i];
        else
          d0 += vi * x[i];
      }
      const double d = tau * column_sum<kQ>(d0 + d1);
      // 512-thread workgroups keep the vector's values in registers across the
      // reduction (one batch of LDS reads per step).  At 1024 threads (128
      // registers per lane) that would spill, so there the vector is read from
      // LDS again; the empty asm keeps the compiler from reusing the reads.
      if constexpr (NT >= 1024) asm volatile("" ::: "memory");
      double n0 = 0.0, n1 = 0.0;
#pragma unroll
      for (int i = 0; i < RPL; ++i) {
        x[i] -= d * vh[q + kQ * i];
        const double xm = (q + kQ * i > j) ? x[i] : 0.0;
        if (i & 1)
          n1 = fma(xm, xm, n1);
        else
          n0 = fma(xm, xm, n0);
      }
      nu2 = column_sum<kQ>(n0 + n1);
    }
    // No barrier here: the next step rewrites s_wv, s_wp and s_cand only after
    // this step's second barrier (wave 0 read them before it), and s_rec and
    // s_hp only after its own first barrier, which follows this step's last
    // read of them.
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

template <int LM, int Q, int NT>
__global__ __launch_bounds__(NT) void sample_qrcp_kernel(SqArgs a) {
  sample_qrcp_body<LM, Q, NT>(a);
  if (a.release && blockIdx.x == 0 && threadIdx.x == 0) sq_release(a);
}

int sq_lm(int ell) {
  if (ell <= 0 || ell > 96) return 0;
  return ((ell + 7) / 8) * 8;
}

// A step's area holds nwg x (lm + 4) words: first the heads (norm^2, position)
// of all workgroups, packed so that a poll of every head touches few cache
// lines, then each workgroup's body (tau, beta, the lm-word vector).
int sq_record_stride(int lm) { return lm + kHead; }

// Every workgroup of the persistent kernel must be resident at once, so the
// workgroup count stays within the caller's allowance: 256-thread workgroups of
// 64 columns (one wave per SIMD: the shortest step) when they fit, else
// 512-thread workgroups of 128 columns, else 1024-thread ones of 256.
int sq_groups(int64_t N, int max_groups) {
  // wave 0 polls at most kHeadPer heads per lane
  max_groups = std::min(max_groups, kHeadPer * 64);
  const int64_t g4 = (N + 63) / 64, g8 = (N + 127) / 128;
  if (g4 <= max_groups) return (int)g4;
  return (int)(g8 <= max_groups ? g8 : (N + 255) / 256);
}

int sq_max_groups(int64_t N) { return (int)((N + 63) / 64); }

template <int LM>
static hipError_t launch_lm(const SqArgs& a, hipStream_t s) {
  // the layout follows from the workgroup count chosen by sq_groups
  if (a.nwg < 1 || (int64_t)a.nwg * 256 < a.N) return hipErrorInvalidValue;
  if ((int64_t)a.nwg * 64 >= a.N)
    hipLaunchKernelGGL((sample_qrcp_kernel<LM, 4, 256>), dim3(a.nwg), dim3(256), 0, s, a);
  else if ((int64_t)a.nwg * 128 >= a.N)
    hipLaunchKernelGGL((sample_qrcp_kernel<LM, 4, 512>), dim3(a.nwg), dim3(512), 0, s, a);
  else
    hipLaunchKernelGGL((sample_qrcp_kernel<LM, 4, 1024>), dim3(a.nwg), dim3(1024), 0, s, a);
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
