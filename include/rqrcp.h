/*
 * rqrcp.h -- C ABI of the MI355X (gfx950) randomized column-pivoted QR library.
 *
 * Method: Duersch & Gu, "Randomized Projection for Rank-Revealing Matrix
 * Factorizations and Low-Rank Approximations" (arXiv:2008.04447).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Matrices are column-major.  Element (i, j) of X with leading dimension ldx
 *   is X[i + j * ldx].  Sizes and leading dimensions are int64_t.
 * - Every matrix/vector pointer is a DEVICE pointer on the handle's device,
 *   allocated and owned by the caller.  The library owns only its workspace,
 *   which lives in the handle, grows on demand (hipMalloc) and is freed by
 *   rq_destroy.
 * - Calls are asynchronous on the handle's stream: they validate arguments on
 *   the host, enqueue kernels and return.  Outputs are valid once the stream
 *   has been synchronized (rq_sync_status does that and reports device-side
 *   errors).  One handle must not be used from two host threads at once;
 *   separate handles are independent.
 * - Return value (rq_status): RQ_OK (0); a negative value -i when argument i
 *   (1-based, counting the handle as argument 1) is invalid, checked before
 *   anything is enqueued; or one of the positive RQ_E_* codes below.
 * - Indices are 0-based.  jpvt[j] = c means column j of A P is column c of A.
 * - Householder vectors follow the paper's reflector (Section 2): for a column
 *   x, beta = -sign(x_0) ||x|| with sign(0) = +1, H = I - tau v v^T with
 *   v_0 = 1 and tau = (beta - x_0) / beta; an all-zero column gives tau = 0.
 * - Omega is the (b + p) x m Gaussian compression matrix of the sketch
 *   B = Omega A (Section 3).  It is always passed explicitly; the library draws
 *   no random numbers.
 */
#ifndef RQRCP_H
#define RQRCP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rq_status;

enum {
  RQ_OK = 0,
  RQ_E_HIP = 1001,         /* a HIP runtime call failed                        */
  RQ_E_NOMEM = 1002,       /* workspace allocation failed                      */
  RQ_E_UNSUPPORTED = 1003, /* valid arguments outside the library's limits     */
  RQ_E_DEVICE = 1004       /* reported by rq_sync_status: see device_error bits */
};

/* device_error bits reported by rq_sync_status */
enum {
  RQ_DEV_BARRIER_TIMEOUT = 1, /* a cross-workgroup wait exceeded its bound */
  RQ_DEV_NONFINITE = 2,       /* NaN/Inf met in a norm or pivot decision   */
  RQ_DEV_NO_PIVOT = 4         /* no admissible pivot column was found      */
};

/* Arithmetic of the bulk contractions.  The panel factorization, the norms
 * and the sample QRCP are FP64 in both modes. */
typedef enum {
  RQ_FP64 = 0,        /* everything in FP64                                   */
  RQ_MIXED_BF16 = 1   /* sketch and bulk inner products on BF16 MFMA, FP32
                         accumulation; A given in FP32                        */
} rq_prec;

typedef struct rq_handle_s* rq_handle;

/* Operations, for rq_workspace_query and the serving loop's requests. */
enum {
  RQ_OP_TRQRCP = 0,      /* trqrcp_truncate                                    */
  RQ_OP_TUXV = 1,        /* tuxv_svd / tuxv_svd_iter                           */
  RQ_OP_RQRCP = 2,       /* rqrcp_factor                                       */
  RQ_OP_RSRQRCP = 3,     /* rsrqrcp_factor                                     */
  RQ_OP_QRCP = 4,        /* qrcp_factor (b = nb, p ignored)                    */
  RQ_OP_SKETCH = 5,      /* rq_sketch (b + p = ell, k ignored)                 */
  RQ_OP_SAMPLE_QRCP = 6  /* rq_sample_qrcp (b + p = ell, k = steps, m ignored) */
};

/* Library limits (checked by every entry point):
 * 1 <= b <= 64, p >= 0, b + p <= 96, n <= 65536.  The persistent kernels put
 * one workgroup of 256 rows (or sample columns) on each compute unit, all
 * resident at once, so a factorization also needs max(m, n) <= 256 x the
 * device's compute units (65536 on MI355X), and rq_sketch needs m < 2^31;
 * larger valid sizes return RQ_E_UNSUPPORTED before anything is enqueued. */
#define RQ_MAX_B 64
#define RQ_MAX_ELL 96
#define RQ_MAX_N 65536

/* Create a handle on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  The stream is borrowed:
 * the caller keeps ownership and must keep it alive while the handle is used.
 * Errors: -1 h == NULL, -2 bad device, RQ_E_HIP. */
rq_status rq_create(rq_handle* h, int device, void* hip_stream);

/* Release the handle and its workspace (waits for its stream first). */
rq_status rq_destroy(rq_handle h);

/* Re-point the handle at another stream of the same device. */
rq_status rq_set_stream(rq_handle h, void* hip_stream);

/* Wait for all work enqueued through `h`, then report and clear the device
 * status word: *device_error receives an OR of RQ_DEV_* bits (0 = clean) and
 * the call returns RQ_E_DEVICE when it is nonzero.  device_error may be NULL. */
rq_status rq_sync_status(rq_handle h, int64_t* device_error);

/* Last HIP error string seen by the handle (static storage, never NULL). */
const char* rq_last_error(rq_handle h);

/*
 * Workspace.  Each entry point carves its scratch (samples, split-K partials,
 * exchange records, reflector buffers) out of one device buffer owned by the
 * handle, which grows with hipMalloc when a call needs more and is never
 * shrunk.  rq_workspace_query reports, without touching the device, the bytes
 * the call `op` (RQ_OP_*) would need for the given sizes, so a caller can
 * budget HBM or grow the buffer ahead of time with rq_workspace_reserve (for
 * example before a timed or captured region, after which no call of at most
 * those sizes allocates); rq_workspace_size reports the current size.  The
 * sizes mean what they mean for the entry point named by op; see the RQ_OP_*
 * list for the ones an op ignores.
 * Errors of the query: -1 h, -2 op, -3 prec, -4 m, -5 n, -6 k, -7 b, -8 p,
 * -9 bytes == NULL; reserve returns RQ_E_NOMEM when the allocation fails.
 */
rq_status rq_workspace_query(rq_handle h, int32_t op, rq_prec prec, int64_t m, int64_t n, int64_t k,
                             int64_t b, int64_t p, size_t* bytes);
rq_status rq_workspace_reserve(rq_handle h, size_t bytes);
rq_status rq_workspace_size(rq_handle h, size_t* bytes);

/*
 * rqrcp_factor -- RQRCP, Algorithm 4 (Section 3.4), with the sample update
 * formula eq. (update1): B1 = S12 - S11 R11^{-1} R12, B2 = S22.
 *
 * Factors the first k columns of A P = Q R blockwise with blocks of b pivots
 * chosen by a partial QRCP of the (b+p) x n_J sample, updating the sample
 * instead of re-projecting.  k = min(m, n) is the full factorization.
 *
 *  m, n      rows and columns of A (m, n >= 0)
 *  k         number of reflectors, 0 <= k <= min(m, n)
 *  b, p      block size and oversampling; ell = b + p rows of Omega (ell <= m)
 *  A, lda    in: A (m x n).  out: LAPACK geqp3 layout -- rows 0..k-1 hold R on
 *            and above the diagonal, reflector tails below the diagonal of the
 *            first k columns (unit diagonal implicit), and rows k..m-1 of
 *            columns k..n-1 hold the transformed trailing matrix.  lda >= m.
 *  Omega, ldo  in: ell x m compression matrix, ldo >= ell.  Not modified.
 *  jpvt      out[n]: column permutation (0-based).
 *  tau       out[k]: reflector coefficients.
 *  T, ldt    out: b x k block-T (like dgeqrt): for the block starting at column
 *            c0 with width bJ, T[0:bJ, c0:c0+bJ] is upper triangular with
 *            H_c0 ... H_{c0+bJ-1} = I - Y_J T_J Y_J^T.  ldt >= b.  May be NULL.
 *  info      out: device int64 (may be NULL).  eq. (update1) needs R11
 *            nonsingular (Section 3.2).  After each block's panel every
 *            diagonal entry of its R11 is tested against eps max(m, n) |R_00|
 *            (eps = 2^-52, R_00 the first diagonal entry of R); the first time
 *            one is not larger, *info receives its 1-based column index and
 *            from then on each next sample is a fresh projection of the updated
 *            trailing matrix, B = Omega(:, 0:m-c) A^[J] with Omega's leading
 *            m - c columns (c = the next block's first column: repeated
 *            sampling, Section 3.4, with the given Omega) instead of the sample
 *            update.  *info = 0 when the sample update was used throughout.
 *            A rank-deficient A thus factors with finite R and a valid
 *            permutation; it is a numerical warning, not an error.
 * Streams: part of the work (the inner products beside the panel, the
 * trailing update beside the next sample QRCP) runs on a second stream the
 * handle owns, ordered against the handle's stream on the device; the
 * handle's stream alone is what the caller synchronizes.  The first call on a
 * handle creates that stream and blocks the host once, for at most about
 * 4 ms, while two one-wave kernels on streams of the library's own (never the
 * caller's) check that kernels of two streams run concurrently; where they do
 * not (a profiler's counter collection, kernel serialization) the streams are
 * ordered with events instead of device words.
 * Argument numbers for errors: h=1 m=2 n=3 k=4 b=5 p=6 A=7 lda=8 Omega=9
 * ldo=10 jpvt=11 tau=12 T=13 ldt=14 info=15.
 */
rq_status rqrcp_factor(rq_handle h, int64_t m, int64_t n, int64_t k, int64_t b, int64_t p,
                       double* A, int64_t lda, const double* Omega, int64_t ldo,
                       int64_t* jpvt, double* tau, double* T, int64_t ldt, int64_t* info);

/*
 * rsrqrcp_factor -- RQRCP with repeated sampling (Section 3.4): Algorithm 4
 * with the sample update replaced by a fresh sample of the trailing matrix,
 * B^[J] = Omega^[J] A^[J], after each block's trailing update.  It is the
 * baseline the sample update formula is measured against (one more pass over
 * the trailing matrix per block) and the fallback when a sample update would
 * lose accuracy.
 *
 * Same arguments, layout and results as rqrcp_factor, except:
 *  Omegas, ldo  in: nblk = ceil(k / b) slices of ell x m, ldo >= ell; slice J
 *            starts at Omegas + J * ostride, and block J (first column J b)
 *            uses its first m - J b columns as Omega^[J].  Not modified.
 *  ostride   distance between slices in doubles, ostride >= ldo * m.
 * Argument numbers for errors: h=1 m=2 n=3 k=4 b=5 p=6 A=7 lda=8 Omegas=9
 * ldo=10 ostride=11 jpvt=12 tau=13 T=14 ldt=15.
 */
rq_status rsrqrcp_factor(rq_handle h, int64_t m, int64_t n, int64_t k, int64_t b, int64_t p,
                         double* A, int64_t lda, const double* Omegas, int64_t ldo,
                         int64_t ostride, int64_t* jpvt, double* tau, double* T, int64_t ldt);

/*
 * qrcp_factor -- plain column-pivoted QR on the GPU, Algorithm 2 (QRCP with
 * BLAS-3 reflection blocking, Section 2.1): every pivot is the column of
 * largest trailing 2-norm of the full matrix, the column is brought up to date
 * with the block's earlier reflectors, and the adjusted inner products
 * w_j^T = tau_j (y_j^T A - (y_j^T Y) W^T) pass over the whole trailing matrix.
 * Norms are downdated and recomputed when cancellation makes the downdate
 * unreliable.  This is the baseline RQRCP is measured against.
 *
 * Same layout and meaning of A, jpvt, tau as rqrcp_factor; nb is the
 * reflection block size (1 <= nb <= 64).
 * Argument numbers: h=1 m=2 n=3 k=4 nb=5 A=6 lda=7 jpvt=8 tau=9.
 */
rq_status qrcp_factor(rq_handle h, int64_t m, int64_t n, int64_t k, int64_t nb,
                      double* A, int64_t lda, int64_t* jpvt, double* tau);

/*
 * trqrcp_truncate -- truncated RQRCP without trailing update, Algorithm 5
 * (Section 4.1).  A is never modified.  The selected columns are rebuilt from
 * A - Y W^T just before their panel QR, the inner products use the
 * block-reflector composition W2^T = T2^T (Y2^T A - (Y2^T Y1) W1^T), and the
 * new rows of R are rebuilt from A - Y W^T before the sample update.
 *
 *  prec      RQ_FP64: A is double.  RQ_MIXED_BF16: A is float; the sketch and
 *            Y2^T A run on BF16 MFMA (round-to-nearest-even inputs, FP32
 *            accumulation), everything else in FP64.
 *  m, n, k, b, p   as rqrcp_factor, k <= min(m, n); k < b is allowed (then the
 *            single block uses bJ = k, Algorithm 3's single-sample case).
 *  A, lda    in: A (m x n), double or float per prec.
 *  Omega, ldo  in: ell x m, double.
 *  jpvt      out[n]: first k entries are the selected columns.
 *  Y, ldy    out: m x k double, reflectors with explicit unit diagonal and
 *            zeros above it (ldy >= m).
 *  T, ldt    out: k x k double upper triangular, Q = I - Y T Y^T (ldt >= k).
 *  R, ldr    out: k x n double, columns in pivoted order: A P ~ Q[:, :k] R
 *            (ldr >= k).
 * Argument numbers: h=1 prec=2 m=3 n=4 k=5 b=6 p=7 A=8 lda=9 Omega=10 ldo=11
 * jpvt=12 Y=13 ldy=14 T=15 ldt=16 R=17 ldr=18.
 */
rq_status trqrcp_truncate(rq_handle h, rq_prec prec, int64_t m, int64_t n, int64_t k,
                          int64_t b, int64_t p, const void* A, int64_t lda,
                          const double* Omega, int64_t ldo, int64_t* jpvt,
                          double* Y, int64_t ldy, double* T, int64_t ldt,
                          double* R, int64_t ldr);

/*
 * tuxv_svd -- TUXV approximation of the truncated SVD, Algorithm 6 with
 * j_max = 1 (Section 4.2): TRQRCP, Z0 = R P^T, LQ of Z0 (QR of Z0^T) giving
 * V (n x k), Z1 = A V, QR of Z1 giving U (m x k) and X (k x k upper), so that
 * A ~ U X V^T (eq. TUXV).  The paper's unused tau argument is dropped.
 *
 *  prec, m, n, k, b, p, A, lda, Omega, ldo   as trqrcp_truncate.
 *  U, ldu    out: m x k double with orthonormal columns (ldu >= m).
 *  X, ldx    out: k x k double upper triangular (ldx >= k).
 *  V, ldv    out: n x k double with orthonormal columns (ldv >= n).
 *  jpvt      out[n]: TRQRCP's column permutation.
 *  sigma     out[k] or NULL: the singular values of X, largest first (the SVD
 *            of the small factor, Section 4.2, which estimates the leading
 *            singular values of A; the diagonal of X gives the cruder QLP
 *            estimates).  Computed on the device as rq_singular_values does;
 *            k <= RQ_MAX_SVD when sigma is requested, else RQ_E_UNSUPPORTED.
 * Argument numbers: h=1 prec=2 m=3 n=4 k=5 b=6 p=7 A=8 lda=9 Omega=10 ldo=11
 * U=12 ldu=13 X=14 ldx=15 V=16 ldv=17 jpvt=18 sigma=19.
 */
rq_status tuxv_svd(rq_handle h, rq_prec prec, int64_t m, int64_t n, int64_t k, int64_t b,
                   int64_t p, const void* A, int64_t lda, const double* Omega, int64_t ldo,
                   double* U, int64_t ldu, double* X, int64_t ldx, double* V, int64_t ldv,
                   int64_t* jpvt, double* sigma);

/*
 * tuxv_svd_iter -- TUXV with jmax >= 1 alternations (Algorithm 6, Section
 * 4.2).  Step 1 is tuxv_svd; each further step alternates the LQ of
 * Z = U^T A (a new V, X = R^T lower triangular) and the QR of Z = A V (a new U,
 * X upper triangular), so A ~ U X V^T with X upper for odd jmax and lower for
 * even jmax.  Every step is one more pass over A (two for U^T A when k > 64:
 * its rows are formed in chunks of 64); in mixed precision the products with
 * A use BF16 operands and FP32 accumulation like the first step.
 * Same arguments and results as tuxv_svd (sigma: the singular values of the
 * final X), plus jmax (argument 20, >= 1).
 */
rq_status tuxv_svd_iter(rq_handle h, rq_prec prec, int64_t m, int64_t n, int64_t k, int64_t b,
                        int64_t p, const void* A, int64_t lda, const double* Omega, int64_t ldo,
                        double* U, int64_t ldu, double* X, int64_t ldx, double* V, int64_t ldv,
                        int64_t* jpvt, double* sigma, int64_t jmax);

/*
 * rq_singular_values -- singular values of a k x k matrix X (device, ld ldx,
 * not modified) into sigma[k] (device), largest first: Householder
 * bidiagonalization in one workgroup, then bisection with Sturm counts on the
 * Golub-Kahan tridiagonal of the bidiagonal factor, one wave per singular
 * value.  The computed values are those of X + dX with ||dX|| = O(k eps ||X||)
 * (as for LAPACK's bidiagonal route).  Used by tuxv_svd for sigma.
 * Limit: k <= RQ_MAX_SVD, else RQ_E_UNSUPPORTED.
 * Argument numbers: h=1 k=2 X=3 ldx=4 sigma=5.
 */
#define RQ_MAX_SVD 1024
rq_status rq_singular_values(rq_handle h, int64_t k, const double* X, int64_t ldx, double* sigma);

/*
 * rq_sketch -- the sketch B = Omega A alone (the first step of Algorithms 3-5).
 *  prec      RQ_FP64 (A double) or RQ_MIXED_BF16 (A float, BF16 MFMA).
 *  ell, m, n sizes: Omega is ell x m, A is m x n, B is ell x n (double).
 * Argument numbers: h=1 prec=2 ell=3 m=4 n=5 Omega=6 ldo=7 A=8 lda=9 B=10 ldb=11.
 */
rq_status rq_sketch(rq_handle h, rq_prec prec, int64_t ell, int64_t m, int64_t n,
                    const double* Omega, int64_t ldo, const void* A, int64_t lda,
                    double* B, int64_t ldb);

/*
 * rq_sample_qrcp -- QRCP(B, b) of Algorithm 4 on its own: `steps` pivots of
 * the ell x n sample B chosen by largest trailing 2-norm (ties: lowest current
 * position), with every column transformed.  On exit B holds
 * [[S11, S12], [0, S22]] in pivoted column order (zeros below the diagonal of
 * the first `steps` columns), and perm[j] (j < n) is the input position of
 * the column now at position j.  A NaN or infinite column never becomes a
 * pivot and sets RQ_DEV_NONFINITE; when no column is left that can be chosen
 * the pivoting stops with RQ_DEV_NO_PIVOT, B keeps its input and perm the
 * identity.  Either bit makes rq_sync_status return RQ_E_DEVICE.
 * Argument numbers: h=1 ell=2 n=3 steps=4 B=5 ldb=6 perm=7.
 */
rq_status rq_sample_qrcp(rq_handle h, int64_t ell, int64_t n, int64_t steps, double* B,
                         int64_t ldb, int64_t* perm);

/*
 * rq_sample_qrcp_noalloc -- rq_sample_qrcp for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops and
 * harnesses that forbid hipMalloc.  Same arguments, results and errors as
 * rq_sample_qrcp, but the exchange records and column maps live in a static
 * device array of the library (about 6.6 MB per device, held until the process
 * ends) instead of the handle's workspace, and the call allocates nothing:
 * no hipMalloc, hipFree or memset, only kernel launches on the handle's stream.
 * Limit: n <= RQ_NOALLOC_MAX_N, else RQ_E_UNSUPPORTED before anything is
 * enqueued.  Every call on one device shares that device's array, which keeps
 * the last call's contents (each call re-marks what it uses), so calls that
 * overlap in time on one device -- from two handles or two streams -- race and
 * must be serialized by the caller.  RQ_E_HIP when the array's device address
 * could not be looked up at rq_create.
 * Argument numbers: h=1 ell=2 n=3 steps=4 B=5 ldb=6 perm=7.
 */
#define RQ_NOALLOC_MAX_N 16384
rq_status rq_sample_qrcp_noalloc(rq_handle h, int64_t ell, int64_t n, int64_t steps, double* B,
                                 int64_t ldb, int64_t* perm);

/*
 * Kernel timing for measurement.  Between rq_profile_start and rq_profile_stop
 * every kernel the handle launches is bracketed by HIP events on the stream it
 * runs on and attributed to a named kernel class together with its algorithmic
 * flop and byte counts (the work the mathematics needs, not what the hardware
 * moved).  rq_profile_stop waits for the stream and folds the events into
 * per-class totals, which rq_profile_get reports (class index 0..count-1).
 * rq_profile_classes restricts the timing to the classes whose bit
 * (1u << index) is set in mask (all classes until it is called): each timed
 * launch records two events, a few microseconds of device time, so a run that
 * measures throughput times only the classes it reports.
 * Errors: -1 null handle, -2 index out of range.
 */
rq_status rq_profile_classes(rq_handle h, uint32_t mask);
rq_status rq_profile_start(rq_handle h);
rq_status rq_profile_stop(rq_handle h);
int32_t rq_profile_count(rq_handle h);
rq_status rq_profile_get(rq_handle h, int32_t index, const char** name, int64_t* launches,
                         double* total_ms, double* flops, double* bytes);

/*
 * Serving loop: continuous batching of TRQRCP / TUXV requests of uneven sizes
 * on one device (not part of the paper; its truncated routines are the work).
 *
 * rq_serve_start creates `slots` execution slots, each with its own HIP stream
 * and library handle whose workspace is reserved for requests up to
 * max_m x max_n with rank <= max_k and b + p <= max_ell, plus one device arena
 * of budget_bytes for request data (A, Omega and the outputs).  A scheduler
 * thread admits queued requests in arrival order whenever a slot is free and a
 * contiguous block of the request's footprint fits in the arena (a request
 * larger than the whole arena is rejected at submit time); admitted requests
 * run concurrently on their slots, so work from different requests overlaps on
 * the device.  Each request is computed exactly as by trqrcp_truncate /
 * tuxv_svd on its own, so results do not depend on what else is running.
 *
 * Request data lives in host memory owned by the caller, which must stay valid
 * until the request completes: A (m x n, column-major, leading dimension m;
 * float for RQ_MIXED_BF16 and RQ_AUTO, double for RQ_FP64) and Omega (ell x m,
 * leading dimension ell) are copied in (page-locked memory keeps the copies
 * asynchronous); outputs are copied back to non-NULL host pointers:
 *   TRQRCP: jpvt[n], out0 = Y (m x k), out1 = T (k x k), out2 = R (k x n);
 *   TUXV:   jpvt[n], out0 = U (m x k), out1 = X (k x k), out2 = V (n x k),
 *           sigma[k] = the singular values of X (computed only when non-NULL).
 *
 * Precision per request.  RQ_FP64 and RQ_MIXED_BF16 run as named.  RQ_AUTO
 * (A in float) lets the server choose from the accuracy the caller needs, tol
 * (> 0, the relative truncation error ||A - approximation||_F / ||A||_F the
 * request expects): BF16 operands round A by a relative 2^-9 on average, and
 * that noise reaches the rank-k result through k of min(m, n) directions, so
 * the mixed path adds an error of about f = 1.5 * 2^-9 * sqrt(k / min(m, n))
 * to the optimum e in quadrature.  The request runs on BF16 MFMA when
 * f <= 0.3 tol (then sqrt(e^2 + f^2) <= 1.05 e for e >= tol) and otherwise in
 * FP64, with A widened to double on the device (rq_serve_route reports the
 * choice for given sizes; rq_result.prec_used the one taken).
 * Latency runs from rq_serve_submit to the moment the scheduler sees the
 * request's completion event (host copies included).
 * rq_serve_stop finishes every submitted request, then frees everything.
 * Errors: -i for invalid argument i, RQ_E_UNSUPPORTED for a request beyond the
 * reserved shape or larger than the arena, RQ_E_NOMEM, RQ_E_HIP.
 */
typedef struct rq_server_s* rq_server;

enum { RQ_REQ_QUEUED = 0, RQ_REQ_RUNNING = 1, RQ_REQ_DONE = 2, RQ_REQ_FAILED = 3 };

enum { RQ_AUTO = 2 };      /* request precision: chosen from tol (above)  */

typedef struct {
  int32_t op;             /* RQ_OP_TRQRCP or RQ_OP_TUXV                    */
  int32_t prec;           /* RQ_FP64, RQ_MIXED_BF16 or RQ_AUTO             */
  int64_t m, n, k, b, p;  /* as trqrcp_truncate                            */
  const void* A;          /* host, m x n                                   */
  const double* Omega;    /* host, (b + p) x m                             */
  int64_t* jpvt;          /* host outputs (NULL: not copied back)          */
  double* out0;
  double* out1;
  double* out2;
  double* sigma;          /* TUXV only: host out[k] or NULL                */
  double tol;             /* RQ_AUTO: required relative error (> 0)        */
} rq_request;

typedef struct {
  int32_t state;          /* RQ_REQ_*                                      */
  int32_t status;         /* rq_status of the request                      */
  int64_t device_error;   /* RQ_DEV_* bits seen by the request's slot      */
  double queue_ms;        /* submit -> admission                           */
  double latency_ms;      /* submit -> completion observed                 */
  double flops;           /* algorithmic flop count of the request         */
  int32_t prec_used;      /* RQ_FP64 or RQ_MIXED_BF16: what ran            */
  int32_t reserved;
} rq_result;

/* The arithmetic a request of these sizes and prec/tol runs in (RQ_FP64 or
 * RQ_MIXED_BF16), by the rule above; -1 for an invalid prec or tol. */
int32_t rq_serve_route(int32_t prec, int64_t m, int64_t n, int64_t k, double tol);

rq_status rq_serve_start(int device, size_t budget_bytes, int32_t slots, int64_t max_m,
                         int64_t max_n, int64_t max_k, int64_t max_ell, rq_server* server);
rq_status rq_serve_submit(rq_server server, const rq_request* req, uint64_t* id);
rq_status rq_serve_poll(rq_server server, uint64_t id, rq_result* result);
rq_status rq_serve_wait(rq_server server, uint64_t id, rq_result* result);
rq_status rq_serve_stats(rq_server server, int64_t* completed, int64_t* peak_bytes,
                         int32_t* peak_running);
rq_status rq_serve_stop(rq_server server);

#ifdef __cplusplus
}
#endif
#endif /* RQRCP_H */
