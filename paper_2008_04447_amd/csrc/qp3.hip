// Plain column-pivoted QR on the GPU: Algorithm 2 (QRCP with BLAS-3
// reflection blocking, Section 2.1), the baseline RQRCP is compared with.
//
// Per column j of a block starting at column i (jb = j - i reflectors so far):
//   pivot kernel (a workgroup per 256 rows of column j): argmax of the trailing
//     norms (ties: lowest position), swap columns j <-> p, norms, jpvt and the
//     stored inner products W^T; bring column j up to date with the block's
//     earlier reflectors, exchange the partial norms through published records,
//     form its reflector, and the partials of u = Y(j:, 0:jb)^T v;
//   gemv kernel (all columns): the adjusted inner products
//     w_c = tau (v^T A(j:, c) - u^T W^T(0:jb, c)) over the whole trailing matrix,
//     the update of row j, and the norm downdate nu_c^2 -= A(j, c)^2 with an
//     exact recomputation when cancellation makes the downdate unreliable.
// At the end of a block the trailing matrix receives A -= Y W^T (the MFMA
// update kernel) and its column norms are recomputed exactly.
#include <algorithm>
#include <cmath>

#include "device_common.hpp"
#include "host.hpp"

namespace rq {

constexpr int kQpThreads = 256;
constexpr int kQpRows = 256;                // rows of column j handled by one workgroup

struct Qp3Args {
  double* A;
  int64_t lda;
  int m, n, i, j;     // block start i, current column j
  int nwg;            // workgroups of the pivot kernel
  double* vn1;        // current trailing norms
  double* vn2;        // norms at their last exact computation
  int64_t* jpvt;
  double* Wt;         // inner products, Wt[q + c * 64]
  double* part;       // per-workgroup partials u_q: [nwg][72] (second half of the area)
  double* xrec;       // records of the pivot exchange: column jb of the block at xrec + jb * xstride
  int xstride;        // 2 x the workgroups of the block's first column (the most of any)
  uint32_t* abort_flag;
  double* tau;
  int64_t* status;
};

constexpr int kQpRec = 72;                  // doubles per workgroup record

// Pivot step of column j, spread over nwg workgroups that each own 256 rows
// of column j (rows j + 256 w ...).  Every workgroup finds the same pivot from
// the norms, swaps its share of the two columns, brings its rows of column j up
// to date with the block's reflectors and publishes its partial norm; after one
// exchange each workgroup forms the same reflector, scales its rows and
// publishes its partial u = Y^T v, which the gemv kernel sums.
template <int JB>
__global__ __launch_bounds__(kQpThreads) void qp3_pivot_kernel(Qp3Args a) {
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int i = a.i, j = a.j, jb = j - i;   // jb <= JB
  const int wg = blockIdx.x;
  if (prior_timeout(a.status)) return;
  constexpr int kWaves = kQpThreads / 64;
  __shared__ double s_wv[kWaves];
  __shared__ int s_wp[kWaves];
  __shared__ double s_w[64];
  __shared__ double s_red[kWaves];
  __shared__ int s_piv;
  __shared__ double s_sc[3];
  // 1. argmax of the trailing norms (identical in every workgroup).  The first
  // kBatch norms of each thread are requested before anything waits, then this
  // thread's row of the block's reflectors Y(r, 0:jb), which does not depend on
  // the pivot and stays in registers for the column update (step 3) and the
  // partial u (step 5).  Every load here is unconditional (indices clamped to
  // valid columns), so all of them are in flight together.
  constexpr int kBatch = 32;
  const int r = j + wg * kQpRows + t;
  const bool mine = r < a.m;
  const int rr = mine ? r : j;   // rows past m read row j and contribute zero
  double nv[kBatch];
#pragma unroll
  for (int h = 0; h < kBatch; ++h) nv[h] = a.vn1[min(j + t + h * kQpThreads, a.n - 1)];
  double y[JB];
#pragma unroll
  for (int q = 0; q < JB; ++q) y[q] = a.A[rr + (int64_t)(i + min(q, max(jb - 1, 0))) * a.lda];
  // no load may be moved below this point (into the branches that use them)
  asm volatile("" ::: "memory");
  // A slot past the last column holds column n-1's norm under a larger
  // position, so it loses to column n-1 itself (equal values: lower position
  // wins) and can never be the winner; no slot needs a range test.
  double bv = -1.0;
  int bp = INT_MAX;
#pragma unroll
  for (int h = 0; h < kBatch; ++h) {
    const int c = j + t + h * kQpThreads;
    if (better(nv[h], c, bv, bp)) {
      bv = nv[h];
      bp = c;
    }
  }
  for (int c0 = j + t + kBatch * kQpThreads; c0 < a.n; c0 += kBatch * kQpThreads) {
#pragma unroll
    for (int h = 0; h < kBatch; ++h) nv[h] = a.vn1[min(c0 + h * kQpThreads, a.n - 1)];
#pragma unroll
    for (int h = 0; h < kBatch; ++h) {
      const int c = c0 + h * kQpThreads;
      if (better(nv[h], c, bv, bp)) {
        bv = nv[h];
        bp = c;
      }
    }
  }
  int who = 0;
  wave_argmax(bv, bp, who);
  if (lane == 0) {
    s_wv[wave] = bv;
    s_wp[wave] = bp;
  }
  __syncthreads();
  if (t == 0) {
    double v = s_wv[0];
    int p = s_wp[0];
    for (int w = 1; w < kWaves; ++w)
      if (better(s_wv[w], s_wp[w], v, p)) {
        v = s_wv[w];
        p = s_wp[w];
      }
    if (p == INT_MAX || !(v <= 1.7976931348623157e308)) {
      if (wg == 0) raise_status(a.status, kErrNonFinite);
      p = j;
    }
    s_piv = p;
  }
  __syncthreads();
  const int p = s_piv;
  // 2. the loads that depend on the pivot, in flight together: W^T of the new
  // column j and this thread's rows of columns p and j (rows above j are
  // swapped at the end of the kernel, off the exchange's path)
  double wq = 0.0, xp = 0.0, xj = 0.0;
  if (t < jb) wq = a.Wt[t + (int64_t)p * 64];
  if (mine) {
    xp = a.A[r + (int64_t)p * a.lda];
    if (p != j) xj = a.A[r + (int64_t)j * a.lda];
  }
  // rows 0..j-1 of columns j and p, swapped at the end (strided over the
  // workgroups, up to 8 row pairs per thread requested here)
  const int sw_stride = a.nwg * kQpThreads;
  const int sw_r0 = wg * kQpThreads + t;
  double cj[8], cp[8];
  if (p != j) {
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const int rw = min(sw_r0 + h * sw_stride, max(j - 1, 0));
      cj[h] = a.A[rw + (int64_t)j * a.lda];
      cp[h] = a.A[rw + (int64_t)p * a.lda];
    }
  }
  if (t < 64) s_w[t] = wq;
  __syncthreads();   // s_w is read by every wave below
  // 3. own rows of column j (after the swap), brought up to date
  double x = 0.0;
  if (mine) {
    if (p != j) a.A[r + (int64_t)p * a.lda] = xj;
    x = xp;
#pragma unroll
    for (int q = 0; q < JB; ++q)
      if (q < jb) x -= y[q] * s_w[q];
  }
  double ss = (mine && r > j) ? x * x : 0.0;
  ss = wave_sum(ss);
  if (lane == 0) s_red[wave] = ss;
  __syncthreads();
  // publish this workgroup's partial norm (and, from workgroup 0, whose thread
  // 0 holds row j, the leading entry) in this column's record slots
  double* xr = a.xrec + (int64_t)jb * a.xstride;
  if (t == 0) {
    double sacc = 0.0;
    for (int w = 0; w < kWaves; ++w) sacc += s_red[w];
    publish(xr + 2 * wg, sacc);                 // a sum: never the sentinel pattern
    if (wg == 0) publish(xr + 1, canonical(x));
  }
  // 4. wait for every workgroup's record, then form the reflector, identical
  // in every workgroup (the partials summed in the same fixed order everywhere)
  __shared__ int s_ok;
  if (wave == 0) {
    double part = 0.0, alpha = 0.0;
    uint32_t it = 0;
    bool ok = true;
    for (int w = lane; ok && w < a.nwg; w += 64) {
      unsigned long long bits;
      while ((bits = peek(xr + 2 * w)) == kUnpublished)
        if (!keep_waiting(it, a.abort_flag, a.status)) {
          ok = false;
          break;
        }
      if (ok) part += __longlong_as_double((long long)bits);
    }
    if (ok) {
      unsigned long long bits;
      while ((bits = peek(xr + 1)) == kUnpublished)
        if (!keep_waiting(it, a.abort_flag, a.status)) {
          ok = false;
          break;
        }
      alpha = __longlong_as_double((long long)bits);
    }
    const bool all_ok = __all(ok);
    const double tail = wave_sum(all_ok ? part : 0.0);
    const double s2 = tail + alpha * alpha;
    double beta = 0.0, tau = 0.0, scale = 0.0;
    if (s2 > 0.0) {
      const double sn = sqrt(s2);
      beta = (alpha >= 0.0) ? -sn : sn;
      scale = 1.0 / (alpha - beta);
      tau = (beta - alpha) / beta;
    }
    if (lane == 0) {
      s_sc[0] = beta;
      s_sc[1] = tau;
      s_sc[2] = scale;
      s_ok = all_ok ? 1 : 0;
    }
  }
  __syncthreads();
  if (!s_ok) return;
  // Every workgroup has published, so has finished reading the norms and
  // W^T(:, p): workgroup 0 may now swap the per-column metadata.
  if (wg == 0 && p != j) {
    if (t < jb) {
      const double w0 = a.Wt[t + (int64_t)j * 64];
      a.Wt[t + (int64_t)j * 64] = a.Wt[t + (int64_t)p * 64];
      a.Wt[t + (int64_t)p * 64] = w0;
    }
    if (t == 0) {
      double y0 = a.vn1[j];
      a.vn1[j] = a.vn1[p];
      a.vn1[p] = y0;
      y0 = a.vn2[j];
      a.vn2[j] = a.vn2[p];
      a.vn2[p] = y0;
      const int64_t q = a.jpvt[j];
      a.jpvt[j] = a.jpvt[p];
      a.jpvt[p] = q;
    }
  }
  const double beta = s_sc[0], tau = s_sc[1], scale = s_sc[2];
  double v = 0.0;
  if (mine) {
    v = (r == j) ? 1.0 : x * scale;
    a.A[r + (int64_t)j * a.lda] = (r == j) ? beta : v;
  }
  if (wg == 0 && t == 0) a.tau[j] = tau;
  // 5. partial u_q = sum over own rows of Y(r, q) v(r), q < jb: each wave sums
  // its 64 rows per reflector, and the four waves' sums are added in a fixed order
  double* rec2 = a.part + ((int64_t)a.nwg + wg) * kQpRec;
  {
    __shared__ double s_uq[kWaves][64];
#pragma unroll
    for (int q = 0; q < JB; ++q) {
      if (q < jb) {
        const double su = wave_sum(mine ? y[q] * v : 0.0);
        if (lane == 0) s_uq[wave][q] = su;
      }
    }
    __syncthreads();
    if (t < 64)
      rec2[t] = (t < jb) ? (s_uq[0][t] + s_uq[1][t]) + (s_uq[2][t] + s_uq[3][t]) : 0.0;
  }
  // 6. swap rows 0..j-1 of columns j and p: the first 8 row pairs of each
  // thread were loaded in step 2, the rest (when j > 8 x the threads) here
  if (p != j) {
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const int rw = sw_r0 + h * sw_stride;
      if (rw < j) {
        a.A[rw + (int64_t)j * a.lda] = cp[h];
        a.A[rw + (int64_t)p * a.lda] = cj[h];
      }
    }
    for (int r0 = sw_r0 + 8 * sw_stride; r0 < j; r0 += 8 * sw_stride) {
#pragma unroll
      for (int h = 0; h < 8; ++h) {
        const int rw = min(r0 + h * sw_stride, j - 1);
        cj[h] = a.A[rw + (int64_t)j * a.lda];
        cp[h] = a.A[rw + (int64_t)p * a.lda];
      }
#pragma unroll
      for (int h = 0; h < 8; ++h) {
        const int rw = r0 + h * sw_stride;
        if (rw < j) {
          a.A[rw + (int64_t)j * a.lda] = cp[h];
          a.A[rw + (int64_t)p * a.lda] = cj[h];
        }
      }
    }
  }
}

// Four trailing columns per workgroup.  The four waves split the rows (wave w
// takes the 64-row chunks w, w + 4, ...) so that every column is streamed by
// the whole workgroup, 10 loads in flight per wave; at 64 registers eight
// waves share a SIMD, so the 2000 workgroups of an 8000-column step are
// resident at once.  The partial inner products are combined in LDS in a fixed
// order and wave w then finishes column w (row update and norm downdate).
__global__ __launch_bounds__(256) void qp3_gemv_kernel(Qp3Args a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = a.i, j = a.j, jb = j - i;
  const double tau = a.tau[j];
  const double* v = a.A + (int64_t)j * a.lda;   // v(j) = 1 implied, tails below
  const double tol = 1.4901161193847656e-08;    // sqrt(eps): downdate reliability bound
  __shared__ double s_up[4][64];
  __shared__ double s_dot[4][4];
  {
    // u = sum of the pivot workgroups' partials: wave w adds those of
    // workgroups w, w + 4, ... (8 loads in flight per batch); the four wave
    // sums are added in a fixed order in the epilogue
    constexpr int kB = 8;
    double su = 0.0;
    if (lane < jb) {
      for (int w0 = wave; w0 < a.nwg; w0 += 4 * kB) {
        double pp[kB];
#pragma unroll
        for (int h = 0; h < kB; ++h)
          pp[h] = a.part[((int64_t)a.nwg + min(w0 + 4 * h, a.nwg - 1)) * kQpRec + lane];
#pragma unroll
        for (int h = 0; h < kB; ++h)
          if (w0 + 4 * h < a.nwg) su += pp[h];
      }
    }
    s_up[wave][lane] = su;
  }
  const int c0 = j + 1 + blockIdx.x * 4;
  // what the epilogue of wave w (column c0 + w) reads besides the inner
  // product is final already (the pivot kernel swapped rows j.. and the
  // metadata): request it now so that the epilogue waits on no load
  const int c = c0 + wave;
  const int cc = min(c, a.n - 1);
  double wq = 0.0, yj = 0.0;
  if (lane < jb) {
    wq = a.Wt[lane + (int64_t)cc * 64];
    yj = a.A[j + (int64_t)(i + lane) * a.lda];   // Y(j, q)
  }
  const double rowj = a.A[j + (int64_t)cc * a.lda];
  const double nv1 = a.vn1[cc], nv2 = a.vn2[cc];
  asm volatile("" ::: "memory");   // keep these loads here, ahead of the stream
  {
    const double* cols[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) cols[s] = a.A + (int64_t)min(c0 + s, a.n - 1) * a.lda;
    double acc[4][2] = {};
    int r = j + 1 + wave * 64 + lane;
    for (; r + 256 < a.m; r += 512) {
      double vv[2], xx[4][2];
#pragma unroll
      for (int h = 0; h < 2; ++h) vv[h] = v[r + 256 * h];
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int h = 0; h < 2; ++h) xx[s][h] = cols[s][r + 256 * h];
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int h = 0; h < 2; ++h) acc[s][h] = fma(vv[h], xx[s][h], acc[s][h]);
    }
    if (r < a.m) {
      const double v0 = v[r];
#pragma unroll
      for (int s = 0; s < 4; ++s) acc[s][0] = fma(v0, cols[s][r], acc[s][0]);
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const double d = wave_sum(acc[s][0] + acc[s][1]);
      if (lane == 0) s_dot[wave][s] = d;
    }
  }
  __syncthreads();
  const int s = wave;
  if (c < a.n) {
    const double* col = a.A + (int64_t)c * a.lda;
    const double dot = ((s_dot[0][s] + s_dot[1][s]) + (s_dot[2][s] + s_dot[3][s])) + rowj;
    double corr = 0.0, yw = 0.0;
    if (lane < jb) {
      corr = ((s_up[0][lane] + s_up[1][lane]) + (s_up[2][lane] + s_up[3][lane])) * wq;
      yw = yj * wq;   // Y(j, q) W^T(q, c)
    }
    corr = wave_sum(corr);
    yw = wave_sum(yw);
    const double w = tau * (dot - corr);
    const double rowv = rowj - yw - w;
    if (lane == 0) {
      a.Wt[jb + (int64_t)c * 64] = w;
      a.A[j + (int64_t)c * a.lda] = rowv;
    }
    // norm downdate with the reliability test of LAPACK's blocked QRCP
    double nv = nv1;
    bool redo = false;
    if (nv != 0.0) {
      double tt = fabs(rowv) / nv;
      tt = fmax(0.0, (1.0 + tt) * (1.0 - tt));
      const double ratio = nv / nv2;
      if (tt * ratio * ratio <= tol)
        redo = true;
      else
        nv *= sqrt(tt);
    }
    if (redo) {
      // exact norm of rows j+1.. of column c brought up to date with the block
      double acc = 0.0;
      for (int rr = j + 1 + lane; rr < a.m; rr += 64) {
        double x = col[rr];
        for (int q = 0; q < jb; ++q) x -= a.A[rr + (int64_t)(i + q) * a.lda] * a.Wt[q + (int64_t)c * 64];
        x -= v[rr] * w;
        acc += x * x;
      }
      nv = sqrt(wave_sum(acc));
      if (lane == 0) a.vn2[c] = nv;
    }
    if (lane == 0) a.vn1[c] = nv;
  }
}

// Exact column norms of rows r0..m-1 for columns c0..n-1 (one wave per column).
__global__ __launch_bounds__(256) void qp3_norms_kernel(const double* A, int64_t lda, int m, int r0,
                                                        int c0, int n, double* vn1, double* vn2) {
  const int lane = threadIdx.x & 63;
  const int c = c0 + blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= n) return;
  const double* col = A + (int64_t)c * lda;
  double s0 = 0.0, s1 = 0.0;
  int r = r0 + lane;
  for (; r + 64 < m; r += 128) {
    s0 += col[r] * col[r];
    s1 += col[r + 64] * col[r + 64];
  }
  for (; r < m; r += 64) s0 += col[r] * col[r];
  const double nv = sqrt(wave_sum(s0 + s1));
  if (lane == 0) {
    vn1[c] = nv;
    vn2[c] = nv;
  }
}

size_t qrcp_workspace_bytes(int64_t m, int64_t n, int64_t k) {
  if (n <= 0 || k <= 0) return 0;
  const int max_nwg = (int)((m + kQpRows - 1) / kQpRows);
  const size_t n_part = (size_t)2 * max_nwg * kQpRec;
  const size_t n_xrec = (size_t)64 * 2 * max_nwg;
  return 2 * padded_bytes(n) + padded_bytes((size_t)64 * n) + padded_bytes(n_part) +
         padded_bytes(n_xrec);
}

}  // namespace rq

using namespace rq;

extern "C" rq_status qrcp_factor(rq_handle h, int64_t m, int64_t n, int64_t k, int64_t nb,
                                 double* A, int64_t lda, int64_t* jpvt, double* tau) {
  if (!h) return -1;
  if (m < 0) return -2;
  if (n < 0 || n > RQ_MAX_N) return -3;
  if (k < 0 || k > std::min(m, n)) return -4;
  if (nb < 1 || nb > 64) return -5;
  if (!valid_ptr(A, m * n)) return -6;
  if (lda < std::max<int64_t>(1, m)) return -7;
  if (!valid_ptr(jpvt, n)) return -8;
  if (!valid_ptr(tau, k)) return -9;
  if (n == 0) return RQ_OK;
  if (k > 0 && !rows_fit(h, std::max(m, n))) return RQ_E_UNSUPPORTED;
  DeviceGuard guard(h->device);
  hipStream_t s = h->stream;
  RQ_CHECK(h, launch_iota(jpvt, (int)n, s));
  if (k == 0) return RQ_OK;
  const int max_nwg = (int)((m + kQpRows - 1) / kQpRows);
  const size_t n_part = (size_t)2 * max_nwg * kQpRec;
  RQ_TRY(reserve(h, qrcp_workspace_bytes(m, n, k)));
  Carve cv(h->ws);
  double* vn1 = cv.take<double>(n);
  double* vn2 = cv.take<double>(n);
  double* Wt = cv.take<double>((size_t)64 * n);
  double* part = cv.take<double>(n_part);
  double* xrec = cv.take<double>((size_t)64 * 2 * max_nwg);
  {
    KTimer kt(h, K_QP3_ROW, 2.0 * m * n, 8.0 * m * n);
    hipLaunchKernelGGL(qp3_norms_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, A, lda,
                       (int)m, 0, 0, (int)n, vn1, vn2);
    RQ_CHECK(h, hipGetLastError());
  }
  Qp3Args a{};
  a.A = A;
  a.lda = lda;
  a.m = (int)m;
  a.n = (int)n;
  a.vn1 = vn1;
  a.vn2 = vn2;
  a.jpvt = jpvt;
  a.Wt = Wt;
  a.part = part;
  a.xrec = xrec;
  a.abort_flag = h->sync + 1;
  a.tau = tau;
  a.status = h->status;
  for (int64_t i = 0; i < k; i += nb) {
    const int64_t iend = std::min(k, i + nb);
    a.i = (int)i;
    // record slots of the block's pivot exchanges start as the sentinel (the
    // launch also clears the abort flag)
    a.xstride = 2 * (int)((m - i + kQpRows - 1) / kQpRows);
    RQ_CHECK(h, launch_exchange_prep(h->sync, xrec, (int64_t)(iend - i) * a.xstride, s));
    for (int64_t j = i; j < iend; ++j) {
      a.j = (int)j;
      const double jb = (double)(j - i);
      {
        KTimer kt(h, K_QP3_PIVOT, 4.0 * (m - j) * (jb + 1),
                  8.0 * ((double)(m - j) * (jb + 2) + 2.0 * m));
        a.nwg = (int)((m - j + kQpRows - 1) / kQpRows);
        const int jbi = (int)(j - i);
        if (jbi <= 8)
          hipLaunchKernelGGL(qp3_pivot_kernel<8>, dim3(a.nwg), dim3(kQpThreads), 0, s, a);
        else if (jbi <= 16)
          hipLaunchKernelGGL(qp3_pivot_kernel<16>, dim3(a.nwg), dim3(kQpThreads), 0, s, a);
        else if (jbi <= 32)
          hipLaunchKernelGGL(qp3_pivot_kernel<32>, dim3(a.nwg), dim3(kQpThreads), 0, s, a);
        else
          hipLaunchKernelGGL(qp3_pivot_kernel<64>, dim3(a.nwg), dim3(kQpThreads), 0, s, a);
        RQ_CHECK(h, hipGetLastError());
      }
      const int64_t nt = n - j - 1;
      if (nt > 0) {
        KTimer kt(h, K_QP3_GEMV, 2.0 * (m - j) * (double)nt,
                  8.0 * ((double)(m - j) * nt + (double)(m - j)));
        hipLaunchKernelGGL(qp3_gemv_kernel, dim3((unsigned)((nt + 3) / 4)), dim3(256), 0, s, a);
        RQ_CHECK(h, hipGetLastError());
      }
    }
    // block reflection of the trailing matrix, then exact norms again
    const int64_t j1 = iend;                      // first column after the block
    const int kb = (int)(iend - i);
    if (j1 < n && j1 < m) {
      {
        KTimer kt(h, K_UPDATE, 2.0 * kb * (double)(m - j1) * (n - j1),
                  8.0 * (2.0 * (m - j1) * (double)(n - j1)));
        RQ_CHECK(h, launch_update(A + j1 + j1 * lda, lda, (int)(m - j1), (int)(n - j1),
                                  A + j1 + i * lda, lda, Wt + j1 * 64, 64, kb, h->update_wgs, s));
      }
      KTimer kt(h, K_QP3_ROW, 2.0 * (double)(m - j1) * (n - j1), 8.0 * (double)(m - j1) * (n - j1));
      hipLaunchKernelGGL(qp3_norms_kernel, dim3((unsigned)((n - j1 + 3) / 4)), dim3(256), 0, s, A,
                         lda, (int)m, (int)j1, (int)j1, (int)n, vn1, vn2);
      RQ_CHECK(h, hipGetLastError());
    }
  }
  return RQ_OK;
}
