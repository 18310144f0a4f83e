// Unpivoted Householder QR of the M x bj panel of selected columns, with the
// compact-WY matrix T built on the fly (Section 2.1: Q = I - Y T Y^T).
//
// The panel is split by rows over ceil(M / 256) workgroups and held in
// registers: thread (c, g) of a 1024-thread workgroup owns column c (< 64) and
// a contiguous run of 16 rows (16 row groups, one per wave).
// Reflector j needs one reduction over all rows.  Instead of a norm followed by
// a second pass for v^T a_c, each workgroup reduces the Gram row a_j^T a_c and
// the row-j entries a_c(j); from these every workgroup derives
//   v^T a_c = (a_j^T a_c - alpha a_c(j)) / (alpha - beta) + a_c(j)
// and applies the reflection locally, so one exchange per column suffices.
// The same exchange also carries Y(:, c)^T y_{j-1} for the forward recurrence
// T[:j-1, j-1] = -tau_{j-1} T[:j-1, :j-1] (Y^T y_{j-1}); one extra exchange at
// the end finishes the last column of T.
#include "device_common.hpp"
#include "kernels.hpp"

namespace rq {

constexpr int kPanelThreads = 1024;
constexpr int kPC = 64;                                  // max panel columns
constexpr int kPG = kPanelThreads / kPC;                 // row groups
constexpr int kPR = kPanelRows / kPG;                    // rows per thread (16)

__global__ __launch_bounds__(kPanelThreads) void panel_kernel(PanelArgs a) {
  const int t = threadIdx.x;
  const int c = t % kPC;           // column
  const int g = t / kPC;           // row group (= wave)
  const int wg = blockIdx.x;
  const int row0 = wg * kPanelRows + g * kPR;   // first panel row held by this thread
  const int bj = a.bj;
  const bool colok = c < bj;
  if (prior_timeout(a.status)) return;

  __shared__ double s_bc[2][kPanelRows];   // column j and reflector j-1, this workgroup's rows
  __shared__ double s_red[kPG][3 * kPC];
  __shared__ double s_G[kPC], s_top[kPC], s_p[kPC];
  __shared__ double s_T[kPC][kPC + 1];
  __shared__ double s_tau[kPC];

  double x[kPR];
#pragma unroll
  for (int i = 0; i < kPR; ++i) {
    const int r = row0 + i;
    x[i] = (colok && r < a.M) ? a.A[r + (int64_t)c * a.lda] : 0.0;
  }
  if (t < kPC) {
    for (int q = 0; q < kPC; ++q) s_T[t][q] = 0.0;
  }

  for (int j = 0; j <= bj; ++j) {
    // ---- publish column j and reflector j-1 of this workgroup's rows --------
    __syncthreads();
    if (c == j && j < bj) {
#pragma unroll
      for (int i = 0; i < kPR; ++i) s_bc[0][g * kPR + i] = x[i];
    }
    if (c == j - 1) {
#pragma unroll
      for (int i = 0; i < kPR; ++i) {
        const int r = row0 + i;
        s_bc[1][g * kPR + i] = (r < j - 1) ? 0.0 : (r == j - 1 ? 1.0 : x[i]);
      }
    }
    __syncthreads();
    // ---- partial sums over this workgroup's rows -----------------------------
    double pg = 0.0, pt = 0.0, pp = 0.0;
    if (j < bj && colok && c >= j) {
#pragma unroll
      for (int i = 0; i < kPR; ++i) {
        const int r = row0 + i;
        const double aj = s_bc[0][g * kPR + i];
        pg += (r >= j) ? aj * x[i] : 0.0;
        pt += (r == j) ? x[i] : 0.0;
      }
    }
    if (j >= 2 && c < j - 1) {
#pragma unroll
      for (int i = 0; i < kPR; ++i) {
        const int r = row0 + i;
        pp += (r >= j - 1) ? x[i] * s_bc[1][g * kPR + i] : 0.0;
      }
    }
    s_red[g][c] = pg;
    s_red[g][kPC + c] = pt;
    s_red[g][2 * kPC + c] = pp;
    __syncthreads();
    double* rec = a.rec + ((int64_t)(j & 1) * a.nwg + wg) * (3 * kPC);
    if (t < 3 * kPC) {
      double s = 0.0;
      for (int q = 0; q < kPG; ++q) s += s_red[q][t];
      rec[t] = s;
    }
    if (!grid_barrier(a.counter, a.abort_flag, (uint32_t)a.nwg, (uint32_t)j, a.status)) return;
    // ---- combine in a fixed order: 4 interleaved partial sums over workgroups,
    // every thread keeping several independent loads in flight -----------------
    const double* rj = a.rec + (int64_t)(j & 1) * a.nwg * (3 * kPC);
    {
      const int q = t & (kPC - 1), part = t / kPC;
      double sg = 0.0, sp = 0.0;
      if (wg == 0) {
#pragma unroll 8
        for (int w = part; w < a.nwg; w += kPG) {
          sg += rj[(int64_t)w * 3 * kPC + q];
          sp += rj[(int64_t)w * 3 * kPC + 2 * kPC + q];
        }
      } else {
#pragma unroll 8
        for (int w = part; w < a.nwg; w += kPG) sg += rj[(int64_t)w * 3 * kPC + q];
      }
      s_red[part][q] = sg;
      s_red[part][2 * kPC + q] = sp;
      if (t < kPC) {
        const int owner = j / kPanelRows;          // workgroup holding row j
        s_top[t] = (j < bj && owner < a.nwg) ? rj[(int64_t)owner * 3 * kPC + kPC + t] : 0.0;
      }
    }
    __syncthreads();
    if (t < kPC) {
      double g0 = 0.0, p0 = 0.0;
      for (int q = 0; q < kPG; ++q) {
        g0 += s_red[q][t];
        p0 += s_red[q][2 * kPC + t];
      }
      s_G[t] = g0;
      s_p[t] = p0;
    }
    __syncthreads();
    // ---- T column j-1 (workgroup 0) -------------------------------------------
    if (wg == 0 && j >= 1 && t < kPC) {
      const int jc = j - 1;
      double acc = 0.0;
#pragma unroll 8
      for (int q = 0; q < kPC; ++q) acc += (q >= t && q < jc) ? s_T[t][q] * s_p[q] : 0.0;
      if (t < jc) {
        s_T[t][jc] = -s_tau[jc] * acc;
      } else if (t == jc) {
        s_T[jc][jc] = s_tau[jc];
      }
    }
    if (j == bj) break;
    // ---- reflector j and its application -------------------------------------
    const double alpha = s_top[j];
    const double s2 = s_G[j];
    double beta = 0.0, tau = 0.0, scale = 0.0;
    if (s2 > 0.0) {
      const double sn = sqrt(s2);
      beta = (alpha >= 0.0) ? -sn : sn;
      scale = 1.0 / (alpha - beta);
      tau = (beta - alpha) / beta;
    } else if (!(s2 == 0.0)) {
      if (t == 0) raise_status(a.status, kErrNonFinite);
    }
    if (t == 0) s_tau[j] = tau;
    if (colok && c > j) {
      const double w = scale * (s_G[c] - alpha * s_top[c]) + s_top[c];
      const double coef = tau * w;
#pragma unroll
      for (int i = 0; i < kPR; ++i) {
        const int r = row0 + i;
        const double vr = (r > j) ? s_bc[0][g * kPR + i] * scale : (r == j ? 1.0 : 0.0);
        x[i] -= coef * vr;
      }
    } else if (c == j) {
#pragma unroll
      for (int i = 0; i < kPR; ++i) {
        const int r = row0 + i;
        x[i] = (r > j) ? x[i] * scale : (r == j ? beta : x[i]);
      }
    }
    if (wg == 0 && t == 0) a.tau[j] = tau;
  }
  __syncthreads();
  // ---- write back: R / reflector tails into the panel, explicit Y, T --------
#pragma unroll
  for (int i = 0; i < kPR; ++i) {
    const int r = row0 + i;
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
