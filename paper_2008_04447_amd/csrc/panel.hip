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
//
// Well-conditioned panels take a shorter route with a handful of exchanges per
// panel instead of one per column: two passes of Cholesky QR (Gram matrix
// G = X^T X reduced over workgroups, G = R^T R, X <- X R^{-1}; the second pass
// restores orthogonality) give Q and R, and the Householder vectors with the
// same sign convention as the column-by-column QR are then reconstructed from
// Q by an LU factorization without pivoting of Q11 - S, S = diag(+-1) chosen
// at each step against the pivot's sign: Y = (Q - [S; 0]) U^{-1} with
// Y11 = L11, T = -U S L11^{-T}, and the triangular factor is S R.  This is the
// same reflector set the Householder QR produces, up to rounding.  The route is
// taken only when the first Cholesky factor has positive pivots whose largest
// to smallest ratio is at most kCondMax; otherwise every workgroup reaches the
// same decision and falls back to the column-by-column loop, with the panel
// still untouched in registers.
#include "device_common.hpp"
#include "kernels.hpp"

namespace rq {

constexpr int kPanelThreads = 1024;
constexpr int kPC = 64;                                  // max panel columns
constexpr int kPG = kPanelThreads / kPC;                 // row groups (16 lanes of a wave)
constexpr int kPR = kPanelRows / kPG;                    // rows per thread (16)
constexpr int kRC = 32;                                  // records per combine chunk
constexpr int kPollP = (2 * kRC * kPC + kPC + kPanelThreads - 1) / kPanelThreads;   // words per thread
constexpr int kLd = kPC + 1;                             // row stride of 64 x 64 matrices in LDS
constexpr int kRegion = 4416;                            // doubles per LDS region
constexpr int kWords = kPC * kPC;                        // one 64 x 64 matrix as record words
constexpr double kCondMax = 16384.0;

// Waits for `total` record words (at most MAXW per thread): word e comes from
// src(e) and is handed to put(e, value).  False on timeout/abort.
template <int MAXW, class Src, class Put>
RQ_DEV bool wait_words(Src src, int total, Put put, int t, uint32_t* abort_flag,
                       int64_t* status) {
  unsigned long long b[MAXW];
#pragma unroll
  for (int k = 0; k < MAXW; ++k) {
    const int e = t + k * kPanelThreads;
    b[k] = (e < total) ? peek(src(e)) : 0ull;
  }
  uint32_t it = 0;
  bool ok = true;
  while (true) {
    bool all = true;
#pragma unroll
    for (int k = 0; k < MAXW; ++k) all = all && b[k] != kUnpublished;
    if (all) break;
    if (!keep_waiting(it, abort_flag, status)) {
      ok = false;
      break;
    }
#pragma unroll
    for (int k = 0; k < MAXW; ++k) {
      const int e = t + k * kPanelThreads;
      if (e < total && b[k] == kUnpublished) b[k] = peek(src(e));
    }
  }
#pragma unroll
  for (int k = 0; k < MAXW; ++k) {
    const int e = t + k * kPanelThreads;
    if (e < total) put(e, __longlong_as_double((long long)b[k]));
  }
  return ok;
}

// The two 64 x 64 factorizations of the Cholesky-QR route, blocked by four
// columns per workgroup barrier.
// Wave w keeps rows 4w..4w+3 in registers for the whole factorization (lane =
// column).  A block step applies the four column updates of the current block
// to every row below it, each element taking them one after the other in the
// sweep's order, with the block rows read once from LDS and the entries of a
// wave's own columns taken by readlane; the wave owning the next four rows then
// eliminates them among themselves and writes them to LDS, final, while the
// waves above compute the block's four columns of the triangular inverses.
// Every entry sees the same operations in the same order as in the sweeps, so
// the results are those of the one-column-per-step sweeps; each row is
// written once.

// Cholesky G = R^T R of the leading n x n block and R^{-1}.  On entry A holds G
// (upper part read); on exit R's strict upper part is stored transposed in A's
// strict lower part (A[j][k] = R[k][j], j > k), its diagonal in diag[], and
// Minv holds R^{-1} (upper, zero elsewhere):
// Minv[i][k] = -(sum_{l=i}^{k-1} Minv[i][l] R[l][k]) / R[k][k].  1 / R[k][k] is
// kept past Minv's 64 rows.  Returns false when a pivot is not positive or not
// finite (same value in all threads).
RQ_DEV bool chol_inv(double* A, double* Minv, double* diag, int n, int t) {
  // the wave index as a scalar: the row indices derived from it select
  // readlane sources directly (no readfirstlane before every broadcast)
  const int lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int g = t & 15, row = t >> 4;
  double* const rv = Minv + kPC * kLd;
  for (int e = t; e < kPC * kLd; e += kPanelThreads) Minv[e] = 0.0;
  double a[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) a[q] = A[(4 * wave + q) * kLd + lane];
  bool ok = true;
  __syncthreads();
  // the calling wave's rows k1..k1+3 among themselves, then stored
  auto block_rows = [&](int k1) {
    double blk[4][4];
#pragma unroll
    for (int c1 = 0; c1 < 4; ++c1)
#pragma unroll
      for (int c = 0; c < 4; ++c) blk[c1][c] = (c1 <= c) ? readlane_f64(a[c1], k1 + c) : 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int k = k1 + c;
      if (k >= n) break;
      const double d = blk[c][c];
      ok = ok && (d > 0.0) && (d < 1.7976931348623157e308);
      const double rinv = rsqrt_nr(d);
      const double dinv = rinv * rinv;
      if (lane == 0) {
        diag[k] = d * rinv;
        rv[k] = rinv;
      }
      if (lane > k && lane < n) A[lane * kLd + k] = a[c] * rinv;   // row k of R, transposed
      const double ckj = a[c] * dinv;
#pragma unroll
      for (int c2 = c + 1; c2 < 4; ++c2) {
        if (k1 + c2 <= lane && lane < n) a[c2] -= blk[c][c2] * ckj;
#pragma unroll
        for (int c3 = c2; c3 < 4; ++c3) blk[c2][c3] -= blk[c][c2] * (blk[c][c3] * dinv);
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (k1 + q < n && k1 + q <= lane && lane < n) A[(k1 + q) * kLd + lane] = a[q];
  };
  if (wave == 0) block_rows(0);
  __syncthreads();
  for (int k0 = 0; k0 < n; k0 += 4) {
    // the wave owning the next block is on the critical path: it goes first
    const bool owner = wave == k0 / 4 + 1 && k0 + 4 < n;
    if (owner) __builtin_amdgcn_s_setprio(3);
    // rows below the block: A[i][j] -= A[k][i] A[k][j] / d, k = k0..k0+3, i <= j
    if (4 * wave >= k0 + 4 && 4 * wave < n) {
      double ak[4], dv[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int k = min(k0 + c, n - 1);
        ak[c] = A[k * kLd + lane];
        dv[c] = rv[k] * rv[k];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 4 * wave + q;
        if (i >= n) break;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (k0 + c >= n) break;
          const double aki = readlane_f64(ak[c], i);
          if (lane >= i && lane < n) a[q] -= aki * (ak[c] * dv[c]);
        }
      }
    }
    if (owner) {
      block_rows(k0 + 4);
      __builtin_amdgcn_s_setprio(0);
    }
    // columns k0..k0+3 of R^{-1} (rows up to k0 + 3).  A lane's terms of the
    // dot products sit at l = row + g + 16 m, so at most one falls inside the
    // block: the four partial sums over l < k0 are formed first, and each
    // column then adds that one term from the block values kept in registers.
    if (row <= k0 + 3) {
      double P[4] = {0.0, 0.0, 0.0, 0.0};
      int l = row + g;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        if (l < k0) {
          const double mi = Minv[row * kLd + l];
#pragma unroll
          for (int c = 0; c < 4; ++c) P[c] += mi * A[(k0 + c) * kLd + l];
          l += 16;
        }
      }
      double mv[3] = {0.0, 0.0, 0.0};   // Minv[row][k0 + c] for the block
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int k = k0 + c;
        if (k >= n) break;
        double acc = P[c];
        if (l < k) {
          const int b = l - k0;
          acc += (b == 0 ? mv[0] : (b == 1 ? mv[1] : mv[2])) * A[k * kLd + l];
        }
        acc = row16_sum(acc);
        const double val = (row < k) ? -acc * rv[k] : (row == k ? rv[k] : 0.0);
        if (c < 3) mv[c] = val;
        if (g == 0 && row <= k) Minv[row * kLd + k] = val;
      }
    }
    __syncthreads();
  }
  return !__syncthreads_or(!ok);
}

// LU factorization without pivoting of the leading n x n block of A = Q11 - S,
// with S[k] = -sign(pivot) chosen at step k (so |U[k][k]| >= 1), plus U^{-1}
// (Z) and L^{-1} (W, unit lower).  On exit A holds U's strict upper part and
// the unscaled multipliers below the diagonal (L[i][k] = A[i][k] rcp[k]);
// udiag[k] = U[k][k], rcp[k] = 1 / U[k][k], sgn[k] = S[k].  Row r of Z and
// column r of W follow from their own earlier entries:
// Z[r][k] = -(sum_{l=r}^{k-1} Z[r][l] U[l][k]) / U[k][k],
// W[k][r] = -sum_{l=r}^{k-1} L[k][l] W[l][r].
RQ_DEV void lu_signed(double* A, double* Z, double* W, double* sgn, double* udiag, double* rcp,
                        int n, int t) {
  const int lane = t & 63, wave = __builtin_amdgcn_readfirstlane(t >> 6);   // scalar, as in chol_inv
  const int g = t & 15, row = t >> 4;
  for (int e = t; e < kPC * kLd; e += kPanelThreads) {
    Z[e] = 0.0;
    W[e] = 0.0;
  }
  double a[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) a[q] = A[(4 * wave + q) * kLd + lane];
  // the calling wave's rows k1..k1+3 among themselves, then stored
  auto block_rows = [&](int k1) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int k = k1 + c;
      if (k >= n) break;
      const double p = readlane_f64(a[c], k);
      const double sk = (p >= 0.0) ? -1.0 : 1.0;
      const double ukk = p - sk;
      const double uinv = rcp_nr(ukk);
      if (lane == 0) {
        sgn[k] = sk;
        udiag[k] = ukk;
        rcp[k] = uinv;
      }
      const double ukj = uinv * a[c];
#pragma unroll
      for (int c2 = c + 1; c2 < 4; ++c2) {
        const double m = readlane_f64(a[c2], k);                  // L multiplier A[k1 + c2][k]
        if (k1 + c2 < n && lane > k && lane < n) a[c2] -= m * ukj;
      }
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (k1 + q < n && lane < n) A[(k1 + q) * kLd + lane] = a[q];
  };
  if (wave == 0) block_rows(0);
  __syncthreads();
  for (int k0 = 0; k0 < n; k0 += 4) {
    // the wave owning the next block is on the critical path: it goes first
    const bool owner = wave == k0 / 4 + 1 && k0 + 4 < n;
    if (owner) __builtin_amdgcn_s_setprio(3);
    // rows below the block: A[i][j] -= A[i][k] (A[k][j] / U[k][k]), j > k, the
    // multiplier A[i][k] read from the row itself after the block's earlier columns
    if (4 * wave >= k0 + 4 && 4 * wave < n) {
      double ak[4], rk[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int k = min(k0 + c, n - 1);
        ak[c] = A[k * kLd + lane];
        rk[c] = rcp[k];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = 4 * wave + q;
        if (i >= n) break;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int k = k0 + c;
          if (k >= n) break;
          const double m = readlane_f64(a[q], k);
          if (lane > k && lane < n) a[q] -= m * (rk[c] * ak[c]);
        }
      }
    }
    if (owner) {
      block_rows(k0 + 4);
      __builtin_amdgcn_s_setprio(0);
    }
    // column k of U^{-1} (rows < k) and row k of L^{-1} (columns < k), k = k0..k0+3,
    // with the partial sums over l < k0 first as for R^{-1} above
    if (row <= k0 + 3) {
      double pz[4] = {0.0, 0.0, 0.0, 0.0}, pw[4] = {0.0, 0.0, 0.0, 0.0};
      int l = row + g;
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        if (l < k0) {
          const double zi = Z[row * kLd + l];
          const double wi = W[l * kLd + row];
          const double rl = rcp[l];
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            pz[c] += zi * A[l * kLd + k0 + c];
            pw[c] += A[(k0 + c) * kLd + l] * rl * wi;
          }
          l += 16;
        }
      }
      double zv[3] = {0.0, 0.0, 0.0}, wv[3] = {0.0, 0.0, 0.0};   // Z[row][k0 + c], W[k0 + c][row]
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int k = k0 + c;
        if (k >= n) break;
        double az = pz[c], aw = pw[c];
        if (l < k) {
          const int b = l - k0;
          const double zl = b == 0 ? zv[0] : (b == 1 ? zv[1] : zv[2]);
          const double wl = b == 0 ? wv[0] : (b == 1 ? wv[1] : wv[2]);
          az += zl * A[l * kLd + k];
          aw += A[k * kLd + l] * rcp[l] * wl;
        }
        az = row16_sum(az);
        aw = row16_sum(aw);
        const double zval = (row < k) ? -az * rcp[k] : (row == k ? rcp[k] : 0.0);
        const double wval = (row < k) ? -aw : (row == k ? 1.0 : 0.0);
        if (c < 3) {
          zv[c] = zval;
          wv[c] = wval;
        }
        if (g == 0 && row <= k) {
          Z[row * kLd + k] = zval;
          W[k * kLd + row] = wval;
        }
      }
    }
    __syncthreads();
  }
}

// The 16 waves of the workgroup each own one 16 x 16 block (p, q) of a 64 x 64
// result (p = wave / 4, q = wave % 4); lane l then holds rows 16 p + l/16 + 4 v,
// column 16 q + l % 16 (v = accumulator element), the FP64 MFMA output layout.
// Gram of a 64-row chunk X (LDS, row-major): acc += X[:, p-block]^T X[:, q-block].
RQ_DEV dx4 gram_chunk(const double* X, dx4 acc, int p, int q, int lane) {
#pragma unroll
  for (int k0 = 0; k0 < kPC; k0 += 4) {
    const double* r = X + (k0 + (lane >> 4)) * kLd;
    acc = mfma_f64(r[16 * p + (lane & 15)], r[16 * q + (lane & 15)], acc);
  }
  return acc;
}
// Product of a 64-row chunk X with an upper-triangular 64 x 64 matrix B (both
// LDS, row-major): column block q of the result needs rows k < 16 (q + 1) of B
// only.
RQ_DEV dx4 product_chunk(const double* X, const double* B, int p, int q, int lane) {
  dx4 acc = {0.0, 0.0, 0.0, 0.0};
  const int kend = 16 * (q + 1);
#pragma unroll
  for (int k0 = 0; k0 < kPC; k0 += 4) {
    if (k0 < kend) {
      const double a = X[(16 * p + (lane & 15)) * kLd + k0 + (lane >> 4)];
      const double b = B[(k0 + (lane >> 4)) * kLd + 16 * q + (lane & 15)];
      acc = mfma_f64(a, b, acc);
    }
  }
  return acc;
}

// x <- x B for this workgroup's 256 x 64 tile (held as x[i] = row g + 16 i of
// column c) and an upper-triangular B, staged through X in four chunks of 64
// rows.  Rows of the panel below `keep_below` (global index) keep their values.
RQ_DEV void tile_times(double (&x)[kPR], double* X, const double* B, int t, int rbase,
                       int keep_below) {
  const int g = t % kPG, c = t / kPG, lane = t & 63, wave = t >> 6;
  const int p = wave >> 2, q = wave & 3;
#pragma unroll
  for (int ch = 0; ch < 4; ++ch) {
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) X[(g + 16 * ii) * kLd + c] = x[4 * ch + ii];
    __syncthreads();
    const dx4 acc = product_chunk(X, B, p, q, lane);
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) X[(16 * p + (lane >> 4) + 4 * v) * kLd + 16 * q + (lane & 15)] = acc[v];
    __syncthreads();
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int r = rbase + g + 16 * (4 * ch + ii);
      if (r >= keep_below) x[4 * ch + ii] = X[(g + 16 * ii) * kLd + c];
    }
    __syncthreads();
  }
}

// x <- x B as tile_times (keep_below = 0), with the product's chunks staged in
// a second region Y (so each chunk needs two barriers instead of four) and the
// Gram matrix of the result accumulated from them and published as record
// words: the values and operation order of tile_times followed by tile_gram.
RQ_DEV void tile_times_gram(double (&x)[kPR], double* X, double* Y, const double* B, double* rec,
                            int t) {
  const int g = t % kPG, c = t / kPG, lane = t & 63, wave = t >> 6;
  const int p = wave >> 2, q = wave & 3;
  dx4 gacc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ch = 0; ch < 4; ++ch) {
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) X[(g + 16 * ii) * kLd + c] = x[4 * ch + ii];
    __syncthreads();   // X complete; every wave is done with Y of the previous chunk
    const dx4 acc = product_chunk(X, B, p, q, lane);
#pragma unroll
    for (int v = 0; v < 4; ++v) Y[(16 * p + (lane >> 4) + 4 * v) * kLd + 16 * q + (lane & 15)] = acc[v];
    __syncthreads();   // Y complete; every wave is done with X
    gacc = gram_chunk(Y, gacc, p, q, lane);
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) x[4 * ch + ii] = Y[(g + 16 * ii) * kLd + c];
  }
#pragma unroll
  for (int v = 0; v < 4; ++v)
    publish(rec + (16 * p + (lane >> 4) + 4 * v) * kPC + 16 * q + (lane & 15), gacc[v]);
}

// Gram matrix of this workgroup's tile, published as record words (row-major).
RQ_DEV void tile_gram(const double (&x)[kPR], double* X, double* rec, int t) {
  const int g = t % kPG, c = t / kPG, lane = t & 63, wave = t >> 6;
  const int p = wave >> 2, q = wave & 3;
  dx4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ch = 0; ch < 4; ++ch) {
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) X[(g + 16 * ii) * kLd + c] = x[4 * ch + ii];
    __syncthreads();
    acc = gram_chunk(X, acc, p, q, lane);
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < 4; ++v)
    publish(rec + (16 * p + (lane >> 4) + 4 * v) * kPC + 16 * q + (lane & 15), acc[v]);
}

// Sum of the workgroups' Gram matrices: reduce-scatter (workgroup w sums its
// slice of the entries over all records, in workgroup order) through `part`,
// then every workgroup gathers the whole sum into G (LDS, row-major).
RQ_DEV bool gram_allreduce(const double* recs, double* red, double* G, double* stage, int nwg,
                           int wg, int t, uint32_t* abort_flag, int64_t* status) {
  const int S = (kWords + nwg - 1) / nwg;
  const int lo = wg * S;
  const int len = max(0, min(kWords, lo + S) - lo);
  const int ln = max(len, 1);
  bool ok = wait_words<5>([&](int e) { return recs + (int64_t)(e / ln) * kWords + lo + e % ln; },
                          nwg * len, [&](int e, double v) { stage[e] = v; }, t, abort_flag, status);
  if (__syncthreads_or(!ok)) return false;
  for (int e = t; e < len; e += kPanelThreads) {
    double sum = 0.0;
    for (int w = 0; w < nwg; ++w) sum += stage[w * len + e];
    publish(red + lo + e, sum);
  }
  ok = wait_words<kWords / kPanelThreads>([&](int e) { return red + e; }, kWords,
                                          [&](int e, double v) { G[(e >> 6) * kLd + (e & 63)] = v; },
                                          t, abort_flag, status);
  return !__syncthreads_or(!ok);
}

// First half of the Cholesky-QR route: the two passes give Q (written to
// qbuf, all 64 columns) and workgroup 0 forms R = R2 R1 (to rbuf); the panel
// itself is not written.  When a gate fails, the fallback flag hands the
// untouched panel to the column-by-column route and the second half exits.
__global__ __launch_bounds__(kPanelThreads) void panel_cholqr_kernel(PanelArgs a) {
  const int t = threadIdx.x;
  const int g = t % kPG;           // row group
  const int c = t / kPG;           // column
  const int wg = blockIdx.x;
  const int rbase = wg * kPanelRows;
  const int bj = a.bj;
  const bool colok = c < bj;
  if (prior_timeout(a.status)) return;

  // LDS: four 64 x 64 regions shared by the two routes, plus small vectors
  __shared__ double s_reg[4][kRegion];
  __shared__ double s_vec[5][kPC];

  double x[kPR];
#pragma unroll
  for (int i = 0; i < kPR; ++i) {
    const int r = rbase + g + kPG * i;
    x[i] = (colok && r < a.M) ? canonical(a.A[r + (int64_t)c * a.lda]) : 0.0;
  }

  {
    // ---------------- two-pass Cholesky QR and reconstruction ----------------
    double* const G = s_reg[0];
    double* const RB = s_reg[1];
    double* const X = s_reg[2];
    double* const D = s_reg[3];
    double* const diag = s_vec[1];
    double* const e1 = a.crec;                                   // [nwg][4096] Gram parts
    double* const e2 = e1 + (int64_t)a.nwg * kWords;             // [4096] Gram sum
    double* const e3 = e2 + kWords;                              // second pass
    double* const e4 = e3 + (int64_t)a.nwg * kWords;
    // pass 1
    tile_gram(x, X, e1 + (int64_t)wg * kWords, t);
    if (!gram_allreduce(e1, e2, G, X, a.nwg, wg, t, a.abort_flag, a.status)) return;
    bool good = chol_inv(G, D, diag, bj, t);
    double dmax = 0.0, dmin = 1.7976931348623157e308;
    for (int k = 0; k < bj; ++k) {
      dmax = fmax(dmax, diag[k]);
      dmin = fmin(dmin, diag[k]);
    }
    good = good && dmax <= kCondMax * dmin;
    if (!good) {
      // every workgroup reaches the same decision; the panel is untouched
      if (wg == 0 && t == 0) *a.fallback = 1u;
      return;
    }
    {
      // R1 in upper form into RB (read by R = R2 R1 in workgroup 0)
      for (int e = t; e < kPC * kPC; e += kPanelThreads) {
        const int i = e >> 6, j = e & 63;
        RB[i * kLd + j] = (i < bj && j < bj) ? (i == j ? diag[i] : (j > i ? G[j * kLd + i] : 0.0)) : 0.0;
      }
      // Q1 = X R1^{-1} and, for pass 2, its Gram matrix (G is free: R1 is in RB)
      tile_times_gram(x, X, G, D, e3 + (int64_t)wg * kWords, t);
      if (!gram_allreduce(e3, e4, G, X, a.nwg, wg, t, a.abort_flag, a.status)) return;
      // G = Q1^T Q1 = I + E, E of the order of kappa^2 eps.  With max |E| <= 1e-10
      // the factor and its inverse have closed forms to within rounding:
      // R2 = I + F, F = triu(E) - diag(E) / 2, since R2^T R2 - G = F^T F, and
      // R2^{-1} = I - F, since (I + F)(I - F) = I - F^2, both with entries of at
      // most 64 max|E|^2 <= 1e-18.  Otherwise (and for non-finite G) the
      // Cholesky sweep; every workgroup holds the same G and decides alike.
      double em = 0.0;
      for (int e = t; e < kPC * kPC; e += kPanelThreads) {
        const int i = e >> 6, j = e & 63;
        if (i < bj && j < bj && i <= j) {
          const double v = fabs(G[i * kLd + j] - (i == j ? 1.0 : 0.0));
          em = (v > em || v != v) ? v : em;
        }
      }
      // The offset is about kappa^2 eps.  Beyond 1e-4 (kappa of the panel
      // beyond about 7e5, which the diagonal ratio of the first factor does not
      // bound, as for Kahan-like columns) the two passes lose accuracy in R
      // (about 3e-10 relative at kappa = 1e8): every workgroup sees the same G
      // and leaves the panel untouched for the column-by-column route, as when
      // the first factorization fails.
      if (__syncthreads_or(!(em <= 1e-4))) {
        if (wg == 0 && t == 0) *a.fallback = 1u;
        return;
      }
      // Within 64 eps of the identity, Q1 is already orthonormal to working
      // precision: Q = Q1 and R = R1 (R2 taken as I, its product skipped).
      const bool ident = !__syncthreads_or(!(em <= 64.0 * 2.220446049250313e-16));
      if (ident) {
        for (int e = t; e < kPC * kLd; e += kPanelThreads) {
          const int i = e / kLd, j = e - i * kLd;
          if (i < bj && j < bj) {
            if (i == j)
              diag[i] = 1.0;
            else if (i < j)
              G[j * kLd + i] = 0.0;
          }
        }
        __syncthreads();
      } else if (!__syncthreads_or(!(em <= 1e-10))) {
        // R2 transposed into G's lower part and its diagonal into diag, as the
        // sweep leaves them; D = R2^{-1} (upper)
        for (int e = t; e < kPC * kLd; e += kPanelThreads) {
          const int i = e / kLd, j = e - i * kLd;
          double dv = 0.0;
          if (i < bj && j < bj) {
            if (i == j) {
              diag[i] = 0.5 * (1.0 + G[i * kLd + i]);
              dv = 0.5 * (3.0 - G[i * kLd + i]);
            } else if (i < j) {
              const double f = G[i * kLd + j];
              G[j * kLd + i] = f;
              dv = -f;
            }
          }
          D[e] = dv;
        }
        __syncthreads();
      } else if (!chol_inv(G, D, diag, bj, t)) {
        // the second factorization failed (the same G, so the same outcome, in
        // every workgroup): the column-by-column route factors the panel
        if (wg == 0 && t == 0) *a.fallback = 1u;
        return;
      }
      if (!ident) tile_times(x, X, D, t, rbase, 0);              // Q = Q1 R2^{-1}
      if (wg == 0) {
        // R = R2 R1 (R2 upper: diag and G's lower part transposed), the 16 x 16
        // block (bp, bq) per wave on the matrix cores; lane holds rows
        // 16 bp + kq + 4 v, column 16 bq + l16
        const int lane = t & 63, wave = t >> 6;
        const int bp = wave >> 2, bq = wave & 3, l16 = lane & 15, kq = lane >> 4;
        const int brow = 16 * bp + l16;                           // A-operand row of this lane
        dx4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k0 = 0; k0 < kPC; k0 += 4) {
          const int k = k0 + kq;
          const double av = (brow < bj && k < bj && k >= brow)
                                ? (k == brow ? diag[brow] : G[k * kLd + brow])
                                : 0.0;
          acc = mfma_f64(av, RB[k * kLd + 16 * bq + l16], acc);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) a.rbuf[(16 * bp + kq + 4 * v) * kPC + 16 * bq + l16] = acc[v];
      }
    }
  }
  // Q (all 64 columns: zero beyond bj) for the second half
#pragma unroll
  for (int i = 0; i < kPR; ++i) {
    const int r = rbase + g + kPG * i;
    if (r < a.M) a.qbuf[r + (int64_t)c * a.ldq] = x[i];
  }
}

// Second half of the Cholesky-QR route (skipped when the first half handed
// the panel to the column-by-column route): workgroup 0 factors Q11 - S = LU
// without pivoting and publishes U^{-1} and S; then Y = (Q - [S; 0]) U^{-1}
// (Y11 = L11), T = -U S L11^{-T}, the triangular factor S R, written back with
// tau, and L11^{-1} and S for the inner products that use Q in place of Y.
__global__ __launch_bounds__(kPanelThreads) void panel_cholqr_b_kernel(PanelArgs a) {
  const int t = threadIdx.x;
  const int g = t % kPG;           // row group
  const int c = t / kPG;           // column
  const int wg = blockIdx.x;
  const int rbase = wg * kPanelRows;
  const int bj = a.bj;
  const bool colok = c < bj;
  if (prior_timeout(a.status)) return;
  if (*a.fallback) return;         // the column-by-column route factored the panel

  __shared__ double s_reg[4][kRegion];
  __shared__ double s_vec[5][kPC];
  double* const s_tau = s_vec[0];
  double (*const s_T)[kLd] = reinterpret_cast<double (*)[kLd]>(s_reg[1]);

  double x[kPR];
#pragma unroll
  for (int i = 0; i < kPR; ++i) {
    const int r = rbase + g + kPG * i;
    x[i] = (r < a.M) ? a.qbuf[r + (int64_t)c * a.ldq] : 0.0;
  }
  {
    double* const G = s_reg[0];
    double* const RB = s_reg[1];
    double* const X = s_reg[2];
    double* const D = s_reg[3];
    double* const rcp = s_vec[2];
    double* const sgn = s_vec[3];
    double* const udiag = s_vec[4];
    double* const e5 = a.crec + 2 * ((int64_t)a.nwg * kWords + kWords);   // [4096 + 64] U^{-1}, S
    {
      if (wg == 0) {
        // the 16 x 16 block (bp, bq) of a 64 x 64 product per wave, on the
        // matrix cores; lane holds rows 16 bp + kq + 4 v, column 16 bq + l16
        const int lane = t & 63, wave = t >> 6;
        const int bp = wave >> 2, bq = wave & 3, l16 = lane & 15, kq = lane >> 4;
        const int brow = 16 * bp + l16;                           // A-operand row of this lane
        // R = R2 R1 from the first half, and Q11 into G; then its signed LU
        // with U^{-1} in X and L^{-1} in RB
        for (int e = t; e < kWords; e += kPanelThreads) D[(e >> 6) * kLd + (e & 63)] = a.rbuf[e];
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) G[(g + 16 * ii) * kLd + c] = x[ii];
        __syncthreads();
        lu_signed(G, X, RB, sgn, udiag, rcp, bj, t);
        for (int e = t; e < kWords; e += kPanelThreads) publish(e5 + e, X[(e >> 6) * kLd + (e & 63)]);
        if (t < kPC) publish(e5 + kWords + t, t < bj ? sgn[t] : 0.0);
        // L^{-1} (unit lower, zero beyond bj) and S for the inner products
        for (int e = t; e < kWords; e += kPanelThreads) {
          const int i = e >> 6, q = e & 63;
          a.linv[e] = (i < bj && q < bj) ? RB[i * kLd + q] : 0.0;
        }
        if (t < kPC) a.sgnb[t] = t < bj ? sgn[t] : 0.0;
        // T = -U S L^{-T}: T[i][j] = -sum_{k=i..j} U[i][k] S[k] W[j][k]
        // (U: udiag and G's strict upper part; W = L^{-1} in RB, read transposed)
        dx4 tacc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k0 = 0; k0 < kPC; k0 += 4) {
          const int k = k0 + kq;
          const double av = (brow < bj && k < bj && k >= brow)
                                ? (k == brow ? udiag[brow] : G[brow * kLd + k]) * sgn[k]
                                : 0.0;
          const double bv = (k < bj) ? RB[(16 * bq + l16) * kLd + k] : 0.0;
          tacc = mfma_f64(av, bv, tacc);
        }
        __syncthreads();                                         // every wave is done with W
#pragma unroll
        for (int v = 0; v < 4; ++v) RB[(16 * bp + kq + 4 * v) * kLd + 16 * bq + l16] = -tacc[v];
        if (t < bj) {
          s_tau[t] = -udiag[t] * sgn[t];
          a.tau[t] = s_tau[t];
        }
        // rows 0..bj-1: S R above and on the diagonal, L below
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          const int r = g + 16 * ii;
          if (r < bj && colok)
            x[ii] = (r <= c) ? sgn[r] * D[r * kLd + c] : G[r * kLd + c] * rcp[c];
        }
        __syncthreads();
      }
      bool okw = true;
      if (wg != 0)
        okw = wait_words<5>([&](int e) { return e5 + e; }, kWords + kPC,
                            [&](int e, double v) {
                              if (e < kWords)
                                X[(e >> 6) * kLd + (e & 63)] = v;
                              else
                                sgn[e - kWords] = v;
                            },
                            t, a.abort_flag, a.status);
      if (__syncthreads_or(!okw)) return;
      // Y = Q U^{-1} below row bj
      tile_times(x, G, X, t, rbase, bj);
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


__global__ __launch_bounds__(kPanelThreads) void panel_kernel(PanelArgs a) {
  const int t = threadIdx.x;
  const int g = t % kPG;           // row group
  const int c = t / kPG;           // column
  const int wg = blockIdx.x;
  const int rbase = wg * kPanelRows;
  const int bj = a.bj;
  const bool colok = c < bj;
  if (prior_timeout(a.status)) return;
  if (a.fallback && *a.fallback == 0u) return;   // the Cholesky-QR route produced the panel

  // LDS: four 64 x 64 regions shared by the two routes, plus small vectors
  __shared__ double s_reg[4][kRegion];
  __shared__ double s_bc[2][kPanelRows];   // column j (before its reflection), by step parity
  __shared__ double s_vec[5][kPC];
  double* const s_tau = s_vec[0];
  double (*const s_T)[kLd] = reinterpret_cast<double (*)[kLd]>(s_reg[1]);

  double x[kPR];
#pragma unroll
  for (int i = 0; i < kPR; ++i) {
    const int r = rbase + g + kPG * i;
    x[i] = (colok && r < a.M) ? canonical(a.A[r + (int64_t)c * a.lda]) : 0.0;
  }

  {
  if (wg == 0) {
    for (int e = t; e < kPC * kLd; e += kPanelThreads) (&s_T[0][0])[e] = 0.0;
  }
  double (*const s_S)[kLd] = reinterpret_cast<double (*)[kLd]>(s_reg[0]);
  double* const s_words = s_reg[2];
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
      reflector_coeffs(alpha, s2, beta, scale, tau);
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


hipError_t launch_panel_first(const PanelArgs& a, hipStream_t s) {
  if (a.crec) {
    hipLaunchKernelGGL(panel_cholqr_kernel, dim3(a.nwg), dim3(kPanelThreads), 0, s, a);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(panel_kernel, dim3(a.nwg), dim3(kPanelThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_panel_second(const PanelArgs& a, hipStream_t s) {
  if (!a.crec) return hipSuccess;
  hipLaunchKernelGGL(panel_cholqr_b_kernel, dim3(a.nwg), dim3(kPanelThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_panel(const PanelArgs& a, hipStream_t s) {
  const hipError_t e = launch_panel_first(a, s);
  return e != hipSuccess ? e : launch_panel_second(a, s);
}

}  // namespace rq
