// Host-side launch interface of the gfx950 kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rq {

// ---- sample QRCP (persistent, one workgroup per 256 sample columns) ----------
struct SqArgs {
  double* B;           // ell x N sample, column-major, leading dimension ldb
  int64_t ldb;
  int ell, N, steps, nwg;
  double* rec;         // exchange records: per step nwg x rs words (heads, then bodies), unpublished at launch
  int rs;
  uint32_t* counter;   // zeroed before launch
  uint32_t* abort_flag;
  int64_t* status;
  int* src_top;        // [steps]: input position of the column ending at q < steps
  int* dst_low;        // [steps]: final position of input column o < steps (or -1 if < steps)
  int64_t* perm;       // [N] or null: perm[final] = input position
  uint64_t* release;   // or null: set to release_value once every workgroup is resident
  uint64_t release_value;   // (after the first exchange), and on every way out
};
int sq_lm(int ell);    // padded register height used for a given ell (0 = unsupported)
int sq_record_stride(int lm);
// Workgroups of the sample QRCP kernel for N columns: 64 columns per workgroup
// when that needs at most max_groups, else 128, else 256 (4 lanes per column).
int sq_groups(int64_t N, int max_groups);
int sq_max_groups(int64_t N);   // upper bound of sq_groups over max_groups (record sizing)
hipError_t launch_sample_qrcp(const SqArgs& a, int lm, hipStream_t s);

// ---- panel Householder QR + compact-WY T (persistent) ----------------------
struct PanelArgs {
  double* A;           // top-left of the M x bj panel, leading dimension lda
  int64_t lda;
  int M, bj, nwg;
  double* rec;         // exchange records [bj + 1][nwg][3 * 64], unpublished at launch
  double* crec;        // null, or the records of the Cholesky-QR route (panel_cholqr_doubles)
  uint32_t* fallback;  // with crec: zero at launch, set when the column-by-column route must run
  uint32_t* counter;
  uint32_t* abort_flag;
  int64_t* status;
  double* tau;         // out[bj]
  double* Y;           // out M x 64 explicit reflectors (unit diagonal, zero-padded)
  int64_t ldy;
  double* T;           // out bj x bj upper triangular (zeros below), leading dim ldt
  int64_t ldt;
  // Cholesky-QR route, between its two halves and for the Q-based products:
  double* qbuf;        // M x 64 Q of the panel (leading dim ldq, zero beyond bj)
  int64_t ldq;
  double* rbuf;        // 64 x 64 R = R2 R1, row-major
  double* linv;        // 64 x 64 L11^{-1} (unit lower, zero beyond bj), row-major
  double* sgnb;        // [64] S (zero beyond bj)
};
constexpr int kPanelRows = 256;   // rows held by one workgroup
// record words of the Cholesky-QR route of the panel for nwg workgroups
inline int64_t panel_cholqr_doubles(int nwg) { return (int64_t)2 * nwg * 4096 + 2 * 4096 + 4096 + 64; }
// The panel's kernels in order: launch_panel_first (the Cholesky-QR passes,
// then the column-by-column route, which runs only when the first hands the
// panel over), launch_panel_second (reconstruction and write-back of the
// Cholesky-QR route; exits when the column route ran); launch_panel does both.
hipError_t launch_panel_first(const PanelArgs& a, hipStream_t s);
hipError_t launch_panel_second(const PanelArgs& a, hipStream_t s);
hipError_t launch_panel(const PanelArgs& a, hipStream_t s);

// ---- FP64 MFMA contraction D(P x N) = L(P x K) X(K x N) --------------------
struct GemmArgs {
  const double* L; int64_t sLp, sLk;   // L(p, k) = L[p * sLp + k * sLk]
  const double* X; int64_t ldx;        // X(k, n) = X[k + n * ldx]
  int P, K, N;
  int ksplit, kchunk;                  // split-K: ksplit partial products of kchunk rows
  double* out; int64_t ldout; int64_t split_stride;
  double alpha, beta;                  // ksplit == 1: out = alpha * LX + beta * C
  const double* C; int64_t ldc;
  const int64_t* xcol = nullptr;       // optional: column n of X is X + xcol[n] * ldx
  const int64_t* skip_if = nullptr;    // optional (K <= 64 only): no work when *skip_if != 0
  // optional (P <= 64, unit k stride only): L_alt in place of L when *alt_if != 0
  const double* L_alt = nullptr;
  const uint32_t* alt_if = nullptr;
};
hipError_t launch_gemm_lx(const GemmArgs& g, hipStream_t s);
// split-K plan of launch_gemm_lx for P output rows (kchunk a multiple of 64)
void plan_split(int K, int N, int* ksplit, int* kchunk, int P = 64);
void plan_split_target(int K, int N, int cols, int target, int* ksplit, int* kchunk);
// split of the ring route (P <= 64) by rounds of `slots` resident workgroups
void plan_split_rounds(int K, int N, int slots, int* ksplit, int* kchunk);

// ---- BF16 MFMA contractions (FP32 accumulate, FP64 results) -----------------
struct GemmArgsF {
  const double* L; int64_t sLp, sLk;   // L(p, k), rounded to BF16
  const float* X; int64_t ldx;         // X(k, n) = X[k + n * ldx], rounded to BF16
  int P, K, N;
  int ksplit, kchunk;                  // kchunk a multiple of 32
  double* out; int64_t ldout; int64_t split_stride;   // partial s at out + s * split_stride
  const int64_t* xcol = nullptr;       // optional column map of X
  __bf16* lbf = nullptr;               // workspace: at least bf16_stage_elems(K) BF16 values
  int kpad = 0;                        // set by the launcher
};
int bf16_stage_kpad(int K);
inline int64_t bf16_stage_elems(int64_t K) { return (int64_t)96 * (((K + 31) / 32) * 32 + 32); }
// Stages L as BF16 into g.lbf, then runs the contraction (two kernels on stream s).
hipError_t launch_gemm_lx_bf16(const GemmArgsF& g, hipStream_t s);
// C(M x N) = Y(M x K) Z(K x N) with Y FP32 and Z FP64, both rounded to BF16
// (ldy, ldc >= M).  Z is first staged into zbf, which holds at least
// gemm_nn_bf16_stage_elems(N, K) BF16 values (two kernels on stream s).
int64_t gemm_nn_bf16_stage_elems(int N, int K);
hipError_t launch_gemm_nn_bf16(double* C, int64_t ldc, int M, int N, const float* Y, int64_t ldy,
                               const double* Z, int64_t ldz, int K, __bf16* zbf, hipStream_t s);

// sum of split-K partials; with T != null the result is Z = T^T W written with
// leading dimension ldz = 64 (rows bj..63 zero) -- the trailing-update operand.
// Fixed-order sum of ks split-K partials (ld 64) into W, Z = T^T W (64 x N, rows
// bj.. zero) and R12(bj x N) -= Y11 Z, Y11 the leading bj x bj block of Y.
// With qflag (the panel's fallback flag): when *qflag == 0 the partials are
// those of P = Q^T A of the Cholesky-QR panel instead, and the kernel writes
// R12 = S P and Z = L11^{-1} (R12_before - S P) (linv row-major, sgn as the
// panel's second half leaves them).
hipError_t launch_reduce_r12(const double* part, int64_t sstride, int ks, int N, double* Z,
                             const double* T, int64_t ldt, const double* Y, int64_t ldy,
                             double* R12, int64_t ldr, int bj, hipStream_t s,
                             const uint32_t* qflag = nullptr, const double* linv = nullptr,
                             const double* sgn = nullptr);
hipError_t launch_reduce(const double* part, int64_t ldp, int64_t sstride, int ks, int P,
                         int N, double* out, int64_t ldout, const double* T, int64_t ldt,
                         int bj, hipStream_t s);
// Z(0:bj, n) = T^T W(:, n) (trans) or T W(:, n) with W the split-K sum; Z leading
// dimension ldz (rows bj..min(ldz,64)-1 are zeroed only when zero_pad is set).
hipError_t launch_reduce_t(const double* part, int64_t ldp, int64_t sstride, int ks, int N,
                           double* Z, int64_t ldz, bool zero_pad, const double* T, int64_t ldt,
                           int bj, bool trans, hipStream_t s);

// C(M x N) -= Y(M x K) Z(K x N) with K = bj <= 64 (Y, Z read only for k < K).
// Tall blocks use workgroups that each fill a compute unit; at most max_wgs of
// them (the units the launch may take beside concurrent persistent kernels).
hipError_t launch_update(double* C, int64_t ldc, int M, int N, const double* Y, int64_t ldy,
                         const double* Z, int64_t ldz, int bj, int max_wgs, hipStream_t s);
// C(M x N) = alpha Y(M x K) Z(K x N) + beta C for tall Y and small N (one pass
// over Y; ldy, ldc >= M; C is not read when beta == 0).  Z is first staged into
// zstage, which holds at least gemm_nn_tall_stage_doubles(N, K) doubles (two
// kernels on stream s).
int64_t gemm_nn_tall_stage_doubles(int N, int K);
hipError_t launch_gemm_nn_tall(double* C, int64_t ldc, int M, int N, const double* Y, int64_t ldy,
                               const double* Z, int64_t ldz, int K, double alpha, double beta,
                               double* zstage, hipStream_t s);
// C(M x N) = beta C + alpha Y(M x K) Z(K x N), any K (FP64 MFMA, 64 x 64 tiles).
hipError_t launch_gemm_nn(double* C, int64_t ldc, int M, int N, const double* Y, int64_t ldy,
                          const double* Z, int64_t ldz, int K, double alpha, double beta,
                          hipStream_t s);
// dst(r, c) = src(r0 + r, col[c]) for r < rows, c < cols (src double or float).
hipError_t launch_gather_cols(const void* src, bool src_f32, int64_t lds, int r0, const int64_t* col,
                              double* dst, int64_t ldd, int rows, int cols, hipStream_t s);
// X(r, c) = value for r < rows, c < cols; with diag set, X(c, c) = 1 additionally.
hipError_t launch_fill(double* X, int64_t ldx, int rows, int cols, double value, bool unit_diag,
                       hipStream_t s);
// Explicit unit-lower reflectors of an in-place QR block: Y(r, c) = 0 (r < c),
// 1 (r == c), A(r, c) (r > c), for c < bj; columns bj..63 zero.
hipError_t launch_explicit_y(const double* A, int64_t lda, int M, int bj, double* Y, int64_t ldy,
                             hipStream_t s);
// Upper triangle of an in-place block: R(r, c) = A(r, c) for r <= c < cols, 0 below.
hipError_t launch_copy_upper(const double* A, int64_t lda, int rows, int cols, double* R,
                             int64_t ldr, hipStream_t s);
// T12 = -T11 (G^T T2): G is bj x c0 (ld 64), T2 bj x bj, T11 c0 x c0; result into
// T(0:c0, c0:c0+bj).  X1 is c0 x 64 scratch.
hipError_t launch_tcompose(double* T, int64_t ldt, int c0, int bj, const double* G,
                           const double* T2, int64_t ldt2, double* X1, hipStream_t s);
// Z0T(col[c], i) = R(i, c) for i < k, c < n  (Z0^T = (R P^T)^T).
hipError_t launch_scatter_t(const double* R, int64_t ldr, int k, int n, const int64_t* col,
                            double* Z0T, int64_t ldz, hipStream_t s);

// Rank check of the sample update and the fresh sample that replaces it once
// R11 is numerically singular (|R11(c, c)| <= thresh |R_00|): *info (zero at
// the start of the factorization) receives col0 + c + 1 the first time, and
// from then on B (ell x N, ld ldb) = Omega(:, 0:M2) (C - Y Z) with C M2 x N,
// Y M2 x bj, Z bj x N.
constexpr int kFreshCols = 16;    // columns of B per workgroup
constexpr int kFreshRows = 32;    // rows of C per LDS chunk
constexpr int kFreshMaxEll = 96;
struct RankCheck {
  int64_t* info; const double* r00; double thresh; int64_t col0;
  const double* Om; int64_t ldo;
  const double* C; int64_t ldc; int M2;
  const double* Y; int64_t ldy;
  const double* Z; int64_t ldz;
  int bj, ell, N;
  double* B; int64_t ldb;
};
// Record areas of the next block's exchanges, set to the sentinel (and the
// handle's counter, abort and fallback words to zero) as exchange_prep2 does.
struct RecordPrep {
  uint32_t* sync;
  double* rec1; int64_t n1;
  double* rec2; int64_t n2;
};
// Omega_hat_11 = S11 R11^{-1} (bj x bj), S11 leading dim lds, R11 leading dim ldr;
// with rk, the rank check above in the same launch; with prep, the record
// areas it names are prepared by extra workgroups of the same launch.
hipError_t launch_omega11(const double* S11, int64_t lds, const double* R11, int64_t ldr,
                          int bj, double* M, int64_t ldm, const RankCheck* rk,
                          const RecordPrep* prep, hipStream_t s);
hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t s);
// dst[i] = (double)src[i] for i < n (contiguous arrays).
hipError_t launch_cast_f32_f64(const float* src, double* dst, int64_t n, hipStream_t s);

// Column permutation of `rows` x (cols col0..) of X given by src_top/dst_low,
// plus the same permutation of jpvt (int64, may be null).  ncols = columns of
// the block (X and jpvt hold at least that many); map entries outside it move
// nothing.
hipError_t launch_permute(double* X, int64_t ldx, int rows, int bj, int64_t ncols,
                          const int* src_top, const int* dst_low, int64_t* jpvt, hipStream_t s);

hipError_t launch_iota(int64_t* v, int n, hipStream_t s);
// Clears the barrier counter, abort flag and panel fallback flag (sync[0..2]) and marks the n record
// words of a persistent kernel's exchange as unpublished.
hipError_t launch_exchange_prep(uint32_t* sync, double* rec, int64_t n, hipStream_t s);
hipError_t launch_exchange_prep2(uint32_t* sync, double* rec1, int64_t n1, double* rec2,
                                 int64_t n2, hipStream_t s);
hipError_t launch_copy2d(const double* src, int64_t lds, double* dst, int64_t ldd, int rows,
                         int cols, hipStream_t s);

}  // namespace rq
