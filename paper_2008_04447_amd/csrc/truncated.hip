// Truncated factorizations: TRQRCP (Algorithm 5) and TUXV (Algorithm 6).
//
// TRQRCP never writes A.  Its state is the reflectors Y (m x k), the
// connection matrix T (k x k), the inner products W^T (k x n) and the finished
// rows of R (k x n), with columns kept in the current pivoted order through
// the index map jpvt (A itself is read through jpvt).  Per block:
//   sample pivots -> permute jpvt, W^T, R rows -> selected columns
//   A(:, sel) - Y W^T(:, sel) -> panel QR (Y2, T2, R11) -> inner products
//   W2^T = T2^T (Y2^T A - (Y2^T Y) W^T) -> T composition
//   T12 = -T1 (Y1^T Y2) T2 -> new R rows A(rows, :) - Y W^T -> sample update.
// TUXV then takes Z0 = R P^T, the QR of Z0^T (giving V), Z1 = A V and the QR of
// Z1 (giving U and the upper triangular X).
#include <algorithm>

#include "host.hpp"

namespace rq {

// Workspace pieces shared by the truncated routines.
struct TrWork {
  double* sample;   // ell x n
  double* wt;       // k x n, leading dimension k
  double* awork;    // m x 64 (selected columns, then panel in place)
  double* ybuf;     // m x 64 explicit reflectors of the current panel
  double* prec;     // panel exchange records
  SqWork sw;
  double* sbuf;     // 64 x n
  double* gbuf;     // 64 x k   (Y2^T Y)
  double* x1;       // k x 64
  double* tblk;     // 64 x 64
  double* mhat;     // 64 x 64
  double* part;     // split-K partials
  __bf16* lbf;      // BF16 staging of the left operand (mixed path)
};

static size_t split_part_bound(int64_t n, int64_t k) {
  // split-K partials: ks * 64 * N <= 64 (65536 + N) for every product here, and
  // the sketch's ks * ell * n fits the same bound (ell <= 96 < 2 * 64, ks <= 32)
  return (size_t)64 * (65536 + (size_t)n + (size_t)k) + (size_t)32 * 96 * (size_t)n;
}

static size_t trwork_doubles(int64_t m, int64_t n, int64_t k, int ell) {
  const int64_t mn = std::max(m, n);   // the QR of Z0^T in TUXV has n rows
  return padded_bytes((size_t)ell * n) + padded_bytes((size_t)k * n) + padded_bytes((size_t)m * 64) +
         padded_bytes((size_t)mn * 64) + padded_bytes(panel_rec_doubles(mn)) +
         padded_bytes(sq_rec_doubles(ell, n)) + padded_bytes(bf16_stage_doubles(mn)) +
         padded_bytes((size_t)64 * n) + padded_bytes((size_t)64 * k) + padded_bytes((size_t)k * 64) +
         2 * padded_bytes(64 * 64) + padded_bytes(split_part_bound(n, k)) + 4 * 64 * sizeof(int) + 4096;
}

static TrWork carve_trwork(Carve& cv, int64_t m, int64_t n, int64_t k, int ell) {
  TrWork w;
  w.sample = cv.take<double>((size_t)ell * n);
  w.wt = cv.take<double>((size_t)k * n);
  w.awork = cv.take<double>((size_t)m * 64);
  w.ybuf = cv.take<double>((size_t)std::max(m, n) * 64);
  w.prec = cv.take<double>(panel_rec_doubles(std::max(m, n)));
  w.sw.rec = cv.take<double>(sq_rec_doubles(ell, n));
  w.sbuf = cv.take<double>((size_t)64 * n);
  w.gbuf = cv.take<double>((size_t)64 * k);
  w.x1 = cv.take<double>((size_t)k * 64);
  w.tblk = cv.take<double>(64 * 64);
  w.mhat = cv.take<double>(64 * 64);
  w.part = cv.take<double>(split_part_bound(n, k));
  w.lbf = reinterpret_cast<__bf16*>(cv.take<double>(bf16_stage_doubles(std::max(m, n))));
  w.sw.src_top = cv.take<int>(64);
  w.sw.dst_low = cv.take<int>(64);
  return w;
}

// out(P x N) = L^T-style product of gemm_lx with split-K and a fixed-order
// reduction; out has leading dimension ldout.
static rq_status gemm_lx_reduced(rq_handle h, int cls, GemmArgs g, double* part, double* out,
                                 int64_t ldout) {
  int ks, kc;
  plan_split(g.K, g.N, &ks, &kc);
  g.ksplit = ks;
  g.kchunk = kc;
  g.alpha = 1.0;
  g.beta = 0.0;
  if (ks == 1) {
    g.out = out;
    g.ldout = ldout;
    KTimer kt(h, cls, 2.0 * g.P * (double)g.K * g.N, 8.0 * ((double)g.K * g.N + (double)g.P * g.N));
    RQ_CHECK(h, launch_gemm_lx(g, h->stream));
    return RQ_OK;
  }
  g.out = part;
  g.ldout = 64;
  g.split_stride = (int64_t)64 * g.N;
  {
    KTimer kt(h, cls, 2.0 * g.P * (double)g.K * g.N,
              8.0 * ((double)g.K * g.N + (double)ks * g.P * g.N));
    RQ_CHECK(h, launch_gemm_lx(g, h->stream));
  }
  KTimer kt(h, K_REDUCE, (double)(ks - 1) * g.P * g.N, 8.0 * (ks + 1.0) * g.P * g.N);
  RQ_CHECK(h, launch_reduce(part, 64, g.split_stride, ks, g.P, g.N, out, ldout, nullptr, 0, 0,
                            h->stream));
  return RQ_OK;
}

// The TRQRCP block loop (FP64).  A is m x n double, never written.
static rq_status trqrcp_core(rq_handle h, int64_t m, int64_t n, int64_t k, int64_t b, int ell,
                             const void* Av, bool f32, int64_t lda, const double* Omega, int64_t ldo,
                             int64_t* jpvt, double* Y, int64_t ldy, double* T, int64_t ldt,
                             double* R, int64_t ldr, TrWork& w) {
  hipStream_t s = h->stream;
  {
    KTimer kt(h, K_OTHER, 0.0, 8.0 * ((double)m * k + (double)k * k + (double)k * n));
    RQ_CHECK(h, launch_fill(Y, ldy, (int)m, (int)k, 0.0, false, s));
    RQ_CHECK(h, launch_fill(T, ldt, (int)k, (int)k, 0.0, false, s));
    RQ_CHECK(h, launch_fill(R, ldr, (int)k, (int)n, 0.0, false, s));
    RQ_CHECK(h, launch_iota(jpvt, (int)n, s));
  }
  const double* A = static_cast<const double*>(Av);
  const float* Af = static_cast<const float*>(Av);
  if (f32)
    RQ_TRY(sketch_bf16(h, ell, m, n, Omega, ldo, Af, lda, w.sample, ell, w.part, w.lbf));
  else
    RQ_TRY(sketch_fp64(h, ell, m, n, Omega, ldo, A, lda, w.sample, ell, w.part));
  for (int64_t col0 = 0; col0 < k; col0 += b) {
    const int bj = (int)std::min<int64_t>(b, k - col0);
    const int64_t N = n - col0, M = m - col0, Nt = N - bj;
    // 1. sample pivots (nothing runs beside them: the launch may take every
    //    compute unit the handle's launches may fill)
    RQ_TRY(run_sample_qrcp(h, w.sample + col0 * ell, ell, ell, N, bj, w.sw, /*perm=*/nullptr,
                           /*signal_side=*/false, /*panel_rec=*/nullptr, /*panel_m=*/0,
                           /*panel_bj=*/0, /*groups=*/h->update_wgs));
    // 2. permute the index map, W^T and the finished R rows (A is not moved)
    {
      KTimer kt(h, K_PERMUTE, 0.0, 32.0 * bj * (double)(2 * col0 + 1));
      RQ_CHECK(h, launch_permute(w.wt + col0 * k, k, (int)col0, bj, N, w.sw.src_top,
                                 w.sw.dst_low, jpvt + col0, s));
      if (col0 > 0)
        RQ_CHECK(h, launch_permute(R + col0 * ldr, ldr, (int)col0, bj, N, w.sw.src_top,
                                   w.sw.dst_low, nullptr, s));
    }
    // 3. selected columns of A - Y W^T, rows col0..m-1
    {
      KTimer kt(h, K_TR_SELECT, 2.0 * (double)M * bj * col0, 8.0 * (double)M * bj * 2.0);
      RQ_CHECK(h, launch_gather_cols(Av, f32, lda, (int)col0, jpvt + col0, w.awork, m, (int)M, bj,
                                     s));
      // one pass over Y(col0:, 0:col0); W^T's columns are staged in the split-K
      // buffer, free until this block's inner products
      if (col0 > 0)
        RQ_CHECK(h, launch_gemm_nn_tall(w.awork, m, (int)M, bj, Y + col0, ldy, w.wt + col0 * k, k,
                                        (int)col0, -1.0, 1.0, w.part, s));
    }
    // 4. panel QR of the selected block: Y2, T2, R11
    double* tau_scratch = w.mhat;   // tau values also sit on the diagonal of T2
    RQ_TRY(run_panel(h, w.awork, m, M, bj, w.prec, tau_scratch, w.ybuf, m, w.tblk, 64));
    {
      KTimer kt(h, K_OTHER, 0.0, 16.0 * ((double)M * bj + 2.0 * bj * bj));
      RQ_CHECK(h, launch_copy2d(w.ybuf, m, Y + col0 + col0 * ldy, ldy, (int)M, bj, s));
      RQ_CHECK(h, launch_copy2d(w.tblk, 64, T + col0 + col0 * ldt, ldt, bj, bj, s));
      RQ_CHECK(h, launch_copy_upper(w.awork, m, bj, bj, R + col0 + col0 * ldr, ldr, s));
    }
    // 5a. G = Y2^T Y(:, 0:col0) (Y2 is zero above row col0)
    if (col0 > 0) {
      GemmArgs g{};
      g.L = w.ybuf;
      g.sLp = m;
      g.sLk = 1;
      g.X = Y + col0;
      g.ldx = ldy;
      g.P = bj;
      g.K = (int)M;
      g.N = (int)col0;
      RQ_TRY(gemm_lx_reduced(h, K_TR_SMALL, g, w.part, w.gbuf, 64));
      // 6. T12 = -T11 (G^T T2)
      KTimer kt(h, K_TR_SMALL, 2.0 * (double)col0 * bj * (bj + col0) / 2.0, 8.0 * col0 * (double)col0);
      RQ_CHECK(h, launch_tcompose(T, ldt, (int)col0, bj, w.gbuf, w.tblk, 64, w.x1, s));
    }
    if (Nt > 0) {
      // 5b. S = Y2^T A P over the trailing positions (the one pass over A per block)
      if (f32) {
        GemmArgsF g{};
        g.L = w.ybuf;
        g.sLp = m;
        g.sLk = 1;
        g.X = Af + col0;
        g.ldx = lda;
        g.xcol = jpvt + col0 + bj;
        g.P = bj;
        g.K = (int)M;
        g.N = (int)Nt;
        RQ_TRY(gemm_lx_bf16_reduced(h, K_INNER_BF16, g, w.part, w.sbuf, 64, w.lbf));
      } else {
        GemmArgs g{};
        g.L = w.ybuf;
        g.sLp = m;
        g.sLk = 1;
        g.X = A + col0;
        g.ldx = lda;
        g.xcol = jpvt + col0 + bj;
        g.P = bj;
        g.K = (int)M;
        g.N = (int)Nt;
        RQ_TRY(gemm_lx_reduced(h, K_INNER, g, w.part, w.sbuf, 64));
      }
      // 5c. S -= G W^T(0:col0, trailing)
      if (col0 > 0) {
        GemmArgs u{};
        u.L = w.gbuf;
        u.sLp = 1;
        u.sLk = 64;
        u.X = w.wt + (col0 + bj) * k;
        u.ldx = k;
        u.P = bj;
        u.K = (int)col0;
        u.N = (int)Nt;
        u.ksplit = 1;
        u.kchunk = (int)(((col0 + 15) / 16) * 16);
        u.out = w.sbuf;
        u.ldout = 64;
        u.alpha = -1.0;
        u.beta = 1.0;
        u.C = w.sbuf;
        u.ldc = 64;
        KTimer kt(h, K_TR_SMALL, 2.0 * bj * (double)col0 * Nt, 8.0 * ((double)col0 * Nt + 2.0 * bj * Nt));
        RQ_CHECK(h, launch_gemm_lx(u, s));
      }
      // 5d. W2^T = T2^T S
      {
        KTimer kt(h, K_REDUCE, (double)bj * bj * Nt, 16.0 * bj * (double)Nt);
        RQ_CHECK(h, launch_reduce_t(w.sbuf, 64, 0, 1, (int)Nt, w.wt + col0 + (col0 + bj) * k, k,
                                    false, w.tblk, 64, bj, true, s));
      }
      // 7. new R rows: A(rows_J, trailing) - Y(rows_J, :) W^T(:, trailing)
      {
        KTimer kt(h, K_TR_ROWS, 2.0 * bj * (double)(col0 + bj) * Nt,
                  8.0 * ((double)(col0 + bj) * Nt + 3.0 * bj * Nt));
        RQ_CHECK(h, launch_gather_cols(Av, f32, lda, (int)col0, jpvt + col0 + bj,
                                       R + col0 + (col0 + bj) * ldr, ldr, bj, (int)Nt, s));
        GemmArgs u{};
        u.L = Y + col0;
        u.sLp = 1;
        u.sLk = ldy;
        u.X = w.wt + (col0 + bj) * k;
        u.ldx = k;
        u.P = bj;
        u.K = (int)(col0 + bj);
        u.N = (int)Nt;
        u.ksplit = 1;
        u.kchunk = (int)(((col0 + bj + 15) / 16) * 16);
        u.out = R + col0 + (col0 + bj) * ldr;
        u.ldout = ldr;
        u.alpha = -1.0;
        u.beta = 1.0;
        u.C = R + col0 + (col0 + bj) * ldr;
        u.ldc = ldr;
        RQ_CHECK(h, launch_gemm_lx(u, s));
      }
      // 8. sample update
      if (col0 + bj < k)
        RQ_TRY(run_sample_update(h, w.sample + col0 * ell, ell, R + col0 + col0 * ldr, ldr,
                                 R + col0 + (col0 + bj) * ldr, ldr, bj, Nt, w.mhat));
    }
  }
  return RQ_OK;
}

// Householder QR of an M x K block in place (panels of 64, no pivoting); the
// T of panel J goes to Tb[:, 64 J : 64 J + bj] (leading dimension 64).
static rq_status qr_blocked(rq_handle h, double* A, int64_t lda, int64_t M, int64_t K, double* tau,
                            double* Tb, TrWork& w) {
  hipStream_t s = h->stream;
  for (int64_t c0 = 0; c0 < K; c0 += 64) {
    const int bj = (int)std::min<int64_t>(64, K - c0);
    const int64_t Mj = M - c0, Nt = K - c0 - bj;
    RQ_TRY(run_panel(h, A + c0 + c0 * lda, lda, Mj, bj, w.prec, tau + c0, w.ybuf, M, Tb + c0 * 64,
                     64));
    if (Nt <= 0) continue;
    GemmArgs g{};
    g.L = w.ybuf;
    g.sLp = M;
    g.sLk = 1;
    g.X = A + c0 + (c0 + bj) * lda;
    g.ldx = lda;
    g.P = bj;
    g.K = (int)Mj;
    g.N = (int)Nt;
    RQ_TRY(gemm_lx_reduced(h, K_INNER, g, w.part, w.sbuf, 64));
    {
      KTimer kt(h, K_REDUCE, (double)bj * bj * Nt, 16.0 * 64 * (double)Nt);
      RQ_CHECK(h, launch_reduce_t(w.sbuf, 64, 0, 1, (int)Nt, w.x1, 64, true, Tb + c0 * 64, 64, bj,
                                  true, s));
    }
    KTimer kt(h, K_UPDATE, 2.0 * bj * (double)Mj * Nt, 8.0 * 2.0 * Mj * (double)Nt);
    RQ_CHECK(h, launch_update(A + c0 + (c0 + bj) * lda, lda, (int)Mj, (int)Nt, w.ybuf, M, w.x1, 64,
                              bj, h->update_wgs, s));
  }
  return RQ_OK;
}

// Q[:, 0:K] = H_1 ... H_K [I; 0] from an in-place QR (reverse accumulation).
static rq_status form_q(rq_handle h, const double* A, int64_t lda, int64_t M, int64_t K,
                        const double* Tb, double* Q, int64_t ldq, TrWork& w) {
  hipStream_t s = h->stream;
  {
    KTimer kt(h, K_OTHER, 0.0, 8.0 * (double)M * K);
    RQ_CHECK(h, launch_fill(Q, ldq, (int)M, (int)K, 0.0, true, s));
  }
  const int64_t last = ((K - 1) / 64) * 64;
  for (int64_t c0 = last; c0 >= 0; c0 -= 64) {
    const int bj = (int)std::min<int64_t>(64, K - c0);
    const int64_t Mj = M - c0;
    {
      KTimer kt(h, K_OTHER, 0.0, 16.0 * (double)Mj * 64);
      RQ_CHECK(h, launch_explicit_y(A + c0 + c0 * lda, lda, (int)Mj, bj, w.ybuf, M, s));
    }
    GemmArgs g{};
    g.L = w.ybuf;
    g.sLp = M;
    g.sLk = 1;
    g.X = Q + c0;
    g.ldx = ldq;
    g.P = bj;
    g.K = (int)Mj;
    g.N = (int)K;
    RQ_TRY(gemm_lx_reduced(h, K_INNER, g, w.part, w.sbuf, 64));
    {
      KTimer kt(h, K_REDUCE, (double)bj * bj * K, 16.0 * 64 * (double)K);
      RQ_CHECK(h, launch_reduce_t(w.sbuf, 64, 0, 1, (int)K, w.x1, 64, true, Tb + c0 * 64, 64, bj,
                                  false, s));
    }
    KTimer kt(h, K_UPDATE, 2.0 * bj * (double)Mj * K, 8.0 * 2.0 * Mj * (double)K);
    RQ_CHECK(h, launch_update(Q + c0, ldq, (int)Mj, (int)K, w.ybuf, M, w.x1, 64, bj, h->update_wgs,
                              s));
  }
  return RQ_OK;
}

// V staged for the product Z1 = A V: BF16 (mixed) or FP64, one buffer for both.
static size_t vstage_doubles(int64_t n, int64_t k) {
  return std::max((size_t)(gemm_nn_bf16_stage_elems((int)k, (int)n) + 3) / 4,
                  (size_t)gemm_nn_tall_stage_doubles((int)k, (int)n));
}

// TUXV state beside the TRQRCP work: Y, T, R, Z0^T, Z1, two T stacks, tau, the
// staging of V and an identity column map (carved in this order by tuxv_core).
static size_t tuxv_extra_bytes(int64_t m, int64_t n, int64_t k) {
  return padded_bytes((size_t)m * k) + padded_bytes((size_t)k * k) + padded_bytes((size_t)k * n) +
         padded_bytes((size_t)n * k) + padded_bytes((size_t)m * k) + 2 * padded_bytes((size_t)64 * k) +
         padded_bytes((size_t)k + 64) +
         padded_bytes(vstage_doubles(n, k)) + padded_bytes((size_t)std::max(n, k)) +
         (k <= RQ_MAX_SVD ? singular_values_workspace_bytes(k) : 0);
}

size_t truncated_workspace_bytes(int64_t m, int64_t n, int64_t k, int ell, bool tuxv) {
  size_t w = trwork_doubles(m, n, k, ell);
  if (tuxv) w += tuxv_extra_bytes(m, n, k);
  return w;
}

static rq_status check_common(rq_handle h, rq_prec prec, int64_t m, int64_t n, int64_t k,
                              int64_t b, int64_t p, const void* A, int64_t lda,
                              const double* Omega, int64_t ldo) {
  if (!h) return -1;
  if (prec != RQ_FP64 && prec != RQ_MIXED_BF16) return -2;
  if (m < 0) return -3;
  if (n < 0 || n > RQ_MAX_N) return -4;
  if (k < 0 || k > std::min(m, n)) return -5;
  if (b < 1 || b > RQ_MAX_B) return -6;
  if (p < 0 || b + p > RQ_MAX_ELL || (k > 0 && b + p > m)) return -7;
  if (!valid_ptr(A, m * n)) return -8;
  if (lda < std::max<int64_t>(1, m)) return -9;
  if (!valid_ptr(Omega, k > 0 ? (b + p) * m : 0)) return -10;
  if (ldo < b + p) return -11;
  return RQ_OK;
}

}  // namespace rq

using namespace rq;

extern "C" rq_status trqrcp_truncate(rq_handle h, rq_prec prec, int64_t m, int64_t n, int64_t k,
                                     int64_t b, int64_t p, const void* A, int64_t lda,
                                     const double* Omega, int64_t ldo, int64_t* jpvt, double* Y,
                                     int64_t ldy, double* T, int64_t ldt, double* R,
                                     int64_t ldr) {
  RQ_TRY(check_common(h, prec, m, n, k, b, p, A, lda, Omega, ldo));
  if (!valid_ptr(jpvt, n)) return -12;
  if (!valid_ptr(Y, m * k)) return -13;
  if (ldy < std::max<int64_t>(1, m)) return -14;
  if (!valid_ptr(T, k * k)) return -15;
  if (ldt < std::max<int64_t>(1, k)) return -16;
  if (!valid_ptr(R, k * n)) return -17;
  if (ldr < std::max<int64_t>(1, k)) return -18;
  if (n == 0) return RQ_OK;
  if (k > 0 && !rows_fit(h, std::max(m, n))) return RQ_E_UNSUPPORTED;
  DeviceGuard guard(h->device);
  if (k == 0) {
    RQ_CHECK(h, launch_iota(jpvt, (int)n, h->stream));
    return RQ_OK;
  }
  const int ell = (int)(b + p);
  RQ_TRY(reserve(h, trwork_doubles(m, n, k, ell)));
  Carve cv(h->ws);
  TrWork w = carve_trwork(cv, m, n, k, ell);
  return trqrcp_core(h, m, n, k, b, ell, A, prec == RQ_MIXED_BF16, lda, Omega, ldo, jpvt, Y, ldy,
                     T, ldt, R, ldr, w);
}

// Algorithm 6 with jmax alternations: after Z1 = A V1 and its QR, each further
// step forms Z = U^T A and the LQ of Z (QR of Z^T) for a new V and a lower X,
// then Z = A V and its QR for a new U and an upper X, until jmax steps.
static rq_status tuxv_core(rq_handle h, rq_prec prec, int64_t m, int64_t n, int64_t k, int64_t b,
                           int64_t p, const void* A, int64_t lda, const double* Omega, int64_t ldo,
                           double* U, int64_t ldu, double* X, int64_t ldx, double* V, int64_t ldv,
                           int64_t* jpvt, double* sigma, int64_t jmax) {
  RQ_TRY(check_common(h, prec, m, n, k, b, p, A, lda, Omega, ldo));
  if (!valid_ptr(U, m * k)) return -12;
  if (ldu < std::max<int64_t>(1, m)) return -13;
  if (!valid_ptr(X, k * k)) return -14;
  if (ldx < std::max<int64_t>(1, k)) return -15;
  if (!valid_ptr(V, n * k)) return -16;
  if (ldv < std::max<int64_t>(1, n)) return -17;
  if (!valid_ptr(jpvt, n)) return -18;
  if (sigma && k > RQ_MAX_SVD) return RQ_E_UNSUPPORTED;
  if (n == 0 || k == 0) {
    if (n > 0) RQ_CHECK(h, launch_iota(jpvt, (int)n, h->stream));
    return RQ_OK;
  }
  if (!rows_fit(h, std::max(m, n))) return RQ_E_UNSUPPORTED;
  DeviceGuard guard(h->device);
  const int ell = (int)(b + p);
  // TRQRCP state (Y, T, R) plus the two QR work arrays live in the workspace.
  const size_t extra = tuxv_extra_bytes(m, n, k);
  RQ_TRY(reserve(h, trwork_doubles(m, n, k, ell) + extra));
  Carve cv(h->ws);
  TrWork w = carve_trwork(cv, m, n, k, ell);
  double* Yw = cv.take<double>((size_t)m * k);
  double* Tw = cv.take<double>((size_t)k * k);
  double* Rw = cv.take<double>((size_t)k * n);
  double* Z0T = cv.take<double>((size_t)n * k);
  double* Z1 = cv.take<double>((size_t)m * k);
  double* Tb = cv.take<double>((size_t)64 * k);
  double* Tb2 = cv.take<double>((size_t)64 * k);
  double* tauq = cv.take<double>((size_t)k + 64);
  double* vstage = cv.take<double>(vstage_doubles(n, k));                             // V staged
  int64_t* ident = cv.take<int64_t>((size_t)std::max(n, k));                          // 0, 1, 2, ...
  double* svdw = k <= RQ_MAX_SVD ? cv.take<double>(singular_values_workspace_bytes(k) / 8) : nullptr;
  const bool f32 = prec == RQ_MIXED_BF16;
  hipStream_t s = h->stream;
  // 1. TRQRCP: A P ~ Q R
  RQ_TRY(trqrcp_core(h, m, n, k, b, ell, A, f32, lda, Omega, ldo, jpvt, Yw, m, Tw, k, Rw, k, w));
  // 2. Z0 = R P^T, stored transposed (n x k)
  {
    KTimer kt(h, K_OTHER, 0.0, 16.0 * (double)k * n);
    RQ_CHECK(h, launch_scatter_t(Rw, k, (int)k, (int)n, jpvt, Z0T, n, s));
  }
  // 3. LQ of Z0 = QR of Z0^T: V = Q[:, 0:k]
  RQ_TRY(qr_blocked(h, Z0T, n, n, k, tauq, Tb, w));
  RQ_TRY(form_q(h, Z0T, n, n, k, Tb, V, ldv, w));
  for (int64_t j = 1;; j += 2) {
    // 4. Z1 = A V (the one extra pass over A)
    {
      // algorithmic bytes: A once (FP32 or FP64), V and Z1 in FP64
      KTimer kt(h, f32 ? K_INNER_BF16 : K_INNER, 2.0 * (double)m * n * k,
                (f32 ? 4.0 : 8.0) * (double)m * n + 8.0 * ((double)n * k + (double)m * k));
      if (f32)
        RQ_CHECK(h, launch_gemm_nn_bf16(Z1, m, (int)m, (int)k, static_cast<const float*>(A), lda, V,
                                        ldv, (int)n, reinterpret_cast<__bf16*>(vstage), s));
      else
        RQ_CHECK(h, launch_gemm_nn_tall(Z1, m, (int)m, (int)k, static_cast<const double*>(A), lda,
                                        V, ldv, (int)n, 1.0, 0.0, vstage, s));
    }
    // 5. QR of Z1: U = Q[:, 0:k], X = upper factor
    RQ_TRY(qr_blocked(h, Z1, m, m, k, tauq, Tb2, w));
    {
      KTimer kt(h, K_OTHER, 0.0, 16.0 * (double)k * k);
      RQ_CHECK(h, launch_copy_upper(Z1, m, (int)k, (int)k, X, ldx, s));
    }
    RQ_TRY(form_q(h, Z1, m, m, k, Tb2, U, ldu, w));
    if (j == jmax) break;
    // 6. Z = U^T A (k x n, rows of U^T in chunks of 64 into R's place), its
    // transpose into Z0T, and the LQ of Z: V = Q of Z^T, X = R^T (lower)
    if (j == 1) RQ_CHECK(h, launch_iota(ident, (int)std::max(n, k), s));
    for (int64_t c0 = 0; c0 < k; c0 += 64) {
      const int pc = (int)std::min<int64_t>(64, k - c0);
      if (f32) {
        GemmArgsF g{};
        g.L = U + c0 * ldu;
        g.sLp = ldu;
        g.sLk = 1;
        g.X = static_cast<const float*>(A);
        g.ldx = lda;
        g.P = pc;
        g.K = (int)m;
        g.N = (int)n;
        RQ_TRY(gemm_lx_bf16_reduced(h, K_INNER_BF16, g, w.part, Rw + c0, k, w.lbf));
      } else {
        GemmArgs g{};
        g.L = U + c0 * ldu;
        g.sLp = ldu;
        g.sLk = 1;
        g.X = static_cast<const double*>(A);
        g.ldx = lda;
        g.P = pc;
        g.K = (int)m;
        g.N = (int)n;
        RQ_TRY(gemm_lx_reduced(h, K_INNER, g, w.part, Rw + c0, k));
      }
    }
    {
      KTimer kt(h, K_OTHER, 0.0, 16.0 * (double)k * n);
      RQ_CHECK(h, launch_scatter_t(Rw, k, (int)k, (int)n, ident, Z0T, n, s));
    }
    RQ_TRY(qr_blocked(h, Z0T, n, n, k, tauq, Tb, w));
    {
      KTimer kt(h, K_OTHER, 0.0, 32.0 * (double)k * k);
      RQ_CHECK(h, launch_copy_upper(Z0T, n, (int)k, (int)k, Tw, k, s));
      RQ_CHECK(h, launch_scatter_t(Tw, k, (int)k, (int)k, ident, X, ldx, s));
    }
    RQ_TRY(form_q(h, Z0T, n, n, k, Tb, V, ldv, w));
    if (j + 1 == jmax) break;
  }
  // 7. singular values of X (the SVD of the small factor, Section 4.2)
  if (sigma) RQ_TRY(run_singular_values(h, k, X, ldx, sigma, svdw));
  return RQ_OK;
}

extern "C" rq_status tuxv_svd(rq_handle h, rq_prec prec, int64_t m, int64_t n, int64_t k,
                              int64_t b, int64_t p, const void* A, int64_t lda,
                              const double* Omega, int64_t ldo, double* U, int64_t ldu, double* X,
                              int64_t ldx, double* V, int64_t ldv, int64_t* jpvt, double* sigma) {
  return tuxv_core(h, prec, m, n, k, b, p, A, lda, Omega, ldo, U, ldu, X, ldx, V, ldv, jpvt, sigma,
                   1);
}

extern "C" rq_status tuxv_svd_iter(rq_handle h, rq_prec prec, int64_t m, int64_t n, int64_t k,
                                   int64_t b, int64_t p, const void* A, int64_t lda,
                                   const double* Omega, int64_t ldo, double* U, int64_t ldu,
                                   double* X, int64_t ldx, double* V, int64_t ldv, int64_t* jpvt,
                                   double* sigma, int64_t jmax) {
  if (!h) return -1;
  if (jmax < 1) return -20;
  return tuxv_core(h, prec, m, n, k, b, p, A, lda, Omega, ldo, U, ldu, X, ldx, V, ldv, jpvt, sigma,
                   jmax);
}
