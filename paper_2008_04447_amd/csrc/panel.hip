// Unpivoted Householder QR of the M x bj panel of selected columns, with the
// compact-WY matrix T built on the fly (Section 2.1: Q = I - Y T Y^T).
//
// The panel is split by rows over ceil(M / 256) workgroups and held in
// registers.  Thread t of a 1024-thread workgroup owns column c = t / 16 (< 64)
// and row group g = t % 16, i.e. the workgroup rows g, g + 16, ..., g + 240, so
// each wave holds four whole columns and every per-column reduction over the
// workgroup's rows is a 16-lane shuffle inside one wave.
// Reflector j needs one reduction over all rows.  Instead of a norm followed by
// a second pass for v^T a_c, each workgroup reduces the Gram row a_j^T a_c and
// the row-j entries a_c(j); from these every workgroup derives
//   v^T a_c = (a_j^T a_c - alpha a_c(j)) / (alpha - beta) + a_c(j)
// and applies the reflection locally, so one exchange per column suffices.
// The same exchange also carries Y(:, c)^T y_{j-1} for the forward recurrence
// T[:j-1, j-1] = -tau_{j-1} T[:j-1, :j-1] (Y^T y_{j-1}); one extra exchange at
// the end finishes the last column of T.  The partial sums travel as published
// records (device_common.hpp); all sums over workgroups are taken in one fixed
// order, so every workgroup derives bitwise the same reflector.
#include "device_common.hpp"
#include "kernels.hpp"

namespace rq {

constexpr int kPanelThreads = 1024;
constexpr int kPC = 64;                                  // max panel columns
constexpr int kPG = kPanelThreads / kPC;                 // row groups (16 lanes of a wave)
constexpr int kPR = kPanelRows / kPG;                    // rows per thread (16)
constexpr int kRC = 32;                                  // records per combine chunk
constexpr int kPollP = (2 * kRC * kPC + kPC + kPanelThreads - 1) / kPanelThreads;   // words per thread

__global__ __launch_bounds__(kPanelThreads) void panel_kernel(PanelArgs a) {
  const int t = threadIdx.x;
  const int g = t % kPG;           // row group
  const int c = t / kPG;           // column
  const int wg = blockIdx.x;
  const int rbase = wg * kPanelRows;
  const int bj = a.bj;
  const bool colok = c < bj;
  if (prior_timeout(a.status)) return;

  __shared__ double s_bc[2][kPanelRows];   // column j (before its reflection), by step parity
  __shared__ double s_S[kPC][kPC + 1];     // workgroup 0: S[q][i] = y_q^T y_i for q < i
  __shared__ double s_tau[kPC];
  __shared__ double s_words[2 * kRC * kPC + kPC];   // one chunk of record words
  __shared__ double s_T[kPC][kPC + 1];

  double x[kPR];
#pragma unroll
  for (int i = 0; i < kPR; ++i) {
    const int r = rbase + g + kPG * i;
    x[i] = (colok && r < a.M) ? canonical(a.A[r + (int64_t)c * a.lda]) : 0.0;
  }
  if (wg == 0) {
    for (int e = t; e < kPC * (kPC + 1); e += kPanelThreads) (&s_T[0][0])[e] = 0.0;
  }
  double prev_scale = 0.0;

  for (int j = 0; j <= bj; ++j) {
    const int buf = j & 1;
    // ---- publish column j of this workgroup's rows ----------------------------
    // (s_bc[buf] was last read in step j - 2; the exchange of step j - 1 lies between)
    if (c == j && j < bj) {
#pragma unroll
      for (int i = 0; i < kPR; ++i) s_bc[buf][g + kPG * i] = x[i];
    }
    __syncthreads();
    // ---- partial sums over this workgroup's rows -----------------------------
    double pg = 0.0, pt = 0.0, pp = 0.0;
    if (j < bj && colok && c >= j) {
#pragma unroll
      for (int i = 0; i < kPR; ++i) {
        const int r = rbase + g + kPG * i;
        const double aj = s_bc[buf][g + kPG * i];
        pg += (r >= j) ? aj * x[i] : 0.0;
        pt += (r == j) ? x[i] : 0.0;
      }
    }
    if (j >= 2 && c < j - 1) {
      // y_{j-1}: reflector of the previous step, rebuilt from its broadcast column
#pragma unroll
      for (int i = 0; i < kPR; ++i) {
        const int r = rbase + g + kPG * i;
        const double yv = (r == j - 1) ? 1.0 : s_bc[buf ^ 1][g + kPG * i] * prev_scale;
        pp += (r >= j - 1) ? x[i] * yv : 0.0;
      }
    }
    pg = row16_sum(pg);
    pt = row16_sum(pt);
    pp = row16_sum(pp);
    double* rec = a.rec + ((int64_t)j * a.nwg + wg) * (3 * kPC);
    if (g == 0) {
      publish(rec + c, pg);
      publish(rec + kPC + c, pt);
      publish(rec + 2 * kPC + c, pp);
    }
    // ---- combine over workgroups --------------------------------------------
    // The Gram words of every record (and, in workgroup 0, the T words) are
    // waited for with coalesced loads into LDS, kRC records at a time; then lane
    // g sums records g, g + 16, ... in increasing order, and the 16 lanes are
    // summed.  Every wave also forms column j's sums itself.
    const double* rj = a.rec + (int64_t)j * a.nwg * (3 * kPC);
    const int jj = j < bj ? j : 0;
    const bool need_p = wg == 0;
    double sg = 0.0, sgj = 0.0, sp = 0.0, topc = 0.0, alpha = 0.0;
    bool ok = true;
    for (int wb = 0; wb < a.nwg; wb += kRC) {
      const int nrec = min(kRC, a.nwg - wb);
      const int ng = nrec * kPC;                         // Gram words of this chunk
      const int np = need_p ? ng : 0;                    // T words (workgroup 0)
      const int ntop = wb == 0 ? kPC : 0;                // row-j words of workgroup 0
      const int total = ng + np + ntop;
      // word e: [0, ng) Gram, [ng, ng + np) T, then the row-j words
      auto addr = [&](int e) -> const double* {
        if (e < ng) return rj + (int64_t)(wb + e / kPC) * 3 * kPC + (e % kPC);
        if (e < ng + np) {
          const int f = e - ng;
          return rj + (int64_t)(wb + f / kPC) * 3 * kPC + 2 * kPC + (f % kPC);
        }
        return rj + kPC + (e - ng - np);
      };
      unsigned long long bw[kPollP];
#pragma unroll
      for (int k = 0; k < kPollP; ++k) {
        const int e = t + k * kPanelThreads;
        bw[k] = (e < total) ? peek(addr(e)) : 0ull;
      }
      uint32_t it = 0;
      while (ok) {
        bool all = true;
#pragma unroll
        for (int k = 0; k < kPollP; ++k) all = all && bw[k] != kUnpublished;
        if (all) break;
        if (!keep_waiting(it, a.abort_flag, a.status)) {
          ok = false;
          break;
        }
#pragma unroll
        for (int k = 0; k < kPollP; ++k) {
          const int e = t + k * kPanelThreads;
          if (e < total && bw[k] == kUnpublished) bw[k] = peek(addr(e));
        }
      }
#pragma unroll
      for (int k = 0; k < kPollP; ++k) {
        const int e = t + k * kPanelThreads;
        if (e < total) s_words[e] = __longlong_as_double((long long)bw[k]);
      }
      if (__syncthreads_or(!ok)) return;
      for (int w = g; w < nrec; w += kPG) {
        sg += s_words[w * kPC + c];
        sgj += s_words[w * kPC + jj];
        if (need_p) sp += s_words[ng + w * kPC + c];
      }
      if (wb == 0) {
        topc = s_words[ng + np + c];
        alpha = s_words[ng + np + jj];
      }
      __syncthreads();                                   // s_words is refilled by the next chunk
    }
    sg = row16_sum(sg);
    sgj = row16_sum(sgj);
    // ---- column j-1 of S = Y^T Y (workgroup 0); T is formed after the loop ----
    if (wg == 0 && j >= 1) {
      sp = row16_sum(sp);
      if (g == 0) s_S[c][j - 1] = sp;
    }
    if (j == bj) break;
    // ---- reflector j and its application -------------------------------------
    const double s2 = sgj;
    double beta = 0.0, tau = 0.0, scale = 0.0;
    if (s2 > 0.0) {
      const double sn = sqrt(s2);
      beta = (alpha >= 0.0) ? -sn : sn;
      scale = 1.0 / (alpha - beta);
      tau = (beta - alpha) / beta;
    } else if (!(s2 == 0.0)) {
      if (t == 0) raise_status(a.status, kErrNonFinite);
    }
    if (colok && c > j) {
      const double w = scale * (sg - alpha * topc) + topc;
      const double coef = tau * w;
#pragma unroll
      for (int i = 0; i < kPR; ++i) {
        const int r = rbase + g + kPG * i;
        const double vr = (r > j) ? s_bc[buf][g + kPG * i] * scale : (r == j ? 1.0 : 0.0);
        x[i] -= coef * vr;
      }
    } else if (c == j) {
#pragma unroll
      for (int i = 0; i < kPR; ++i) {
        const int r = rbase + g + kPG * i;
        x[i] = (r > j) ? x[i] * scale : (r == j ? beta : x[i]);
      }
    }
    if (wg == 0 && t == 0) {
      a.tau[j] = tau;
      s_tau[j] = tau;
    }
    prev_scale = scale;
  }
  __syncthreads();
  // ---- T by the forward recurrence T[:i, i] = -tau_i T[:i, :i] S[:i, i],
  // T[i, i] = tau_i (workgroup 0; 16 lanes per row of T) ----------------------
  if (wg == 0) {
    for (int i = 0; i < bj; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < kPC / kPG; ++k) {
        const int q = g + kPG * k;
        acc += (q >= c && q < i) ? s_T[c][q] * s_S[q][i] : 0.0;
      }
      acc = row16_sum(acc);
      if (g == 0) {
        if (c < i)
          s_T[c][i] = -s_tau[i] * acc;
        else if (c == i)
          s_T[i][i] = s_tau[i];
      }
      __syncthreads();
    }
  }
  // ---- write back: R / reflector tails into the panel, explicit Y, T --------
#pragma unroll
  for (int i = 0; i < kPR; ++i) {
    const int r = rbase + g + kPG * i;
    if (r < a.M) {
      if (colok) a.A[r + (int64_t)c * a.lda] = x[i];
      const double yv = colok ? ((r < c) ? 0.0 : (r == c ? 1.0 : x[i])) : 0.0;
      a.Y[r + (int64_t)c * a.ldy] = yv;
    }
  }
  if (wg == 0 && a.T) {
    for (int e = t; e < bj * bj; e += kPanelThreads) {
      const int i = e % bj, q = e / bj;
      a.T[i + (int64_t)q * a.ldt] = (i <= q) ? s_T[i][q] : 0.0;
    }
  }
}

hipError_t launch_panel(const PanelArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(panel_kernel, dim3(a.nwg), dim3(kPanelThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace rq
