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
  double* rec;         // exchange records [2][nwg][rs]
  int rs;
  uint32_t* counter;   // zeroed before launch
  uint32_t* abort_flag;
  int64_t* status;
  int* src_top;        // [steps]: input position of the column ending at q < steps
  int* dst_low;        // [steps]: final position of input column o < steps (or -1 if < steps)
  int64_t* perm;       // [N] or null: perm[final] = input position
};
int sq_lm(int ell);    // padded register height used for a given ell (0 = unsupported)
int sq_record_stride(int lm);
int sq_columns_per_group();   // sample columns held by one workgroup
hipError_t launch_sample_qrcp(const SqArgs& a, int lm, hipStream_t s);

// ---- panel Householder QR + compact-WY T (persistent) ----------------------
struct PanelArgs {
  double* A;           // top-left of the M x bj panel, leading dimension lda
  int64_t lda;
  int M, bj, nwg;
  double* rec;         // [2][nwg][3 * 64]
  uint32_t* counter;
  uint32_t* abort_flag;
  int64_t* status;
  double* tau;         // out[bj]
  double* Y;           // out M x 64 explicit reflectors (unit diagonal, zero-padded)
  int64_t ldy;
  double* T;           // out bj x bj upper triangular (zeros below), leading dim ldt
  int64_t ldt;
};
constexpr int kPanelRows = 256;   // rows held by one workgroup
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
};
hipError_t launch_gemm_lx(const GemmArgs& g, hipStream_t s);
void plan_split(int K, int N, int* ksplit, int* kchunk);

// sum of split-K partials; with T != null the result is Z = T^T W written with
// leading dimension ldz = 64 (rows bj..63 zero) -- the trailing-update operand.
hipError_t launch_reduce(const double* part, int64_t ldp, int64_t sstride, int ks, int P,
                         int N, double* out, int64_t ldout, const double* T, int64_t ldt,
                         int bj, hipStream_t s);

// C(M x N) -= Y(M x K) Z(K x N), K = 16 * ceil(bj / 16) <= 64, Z leading dim ldz.
hipError_t launch_update(double* C, int64_t ldc, int M, int N, const double* Y, int64_t ldy,
                         const double* Z, int64_t ldz, int bj, hipStream_t s);

// Omega_hat_11 = S11 R11^{-1} (bj x bj), S11 leading dim lds, R11 leading dim ldr.
hipError_t launch_omega11(const double* S11, int64_t lds, const double* R11, int64_t ldr,
                          int bj, double* M, int64_t ldm, hipStream_t s);

// Column permutation of `rows` x (cols col0..) of X given by src_top/dst_low,
// plus the same permutation of jpvt (int64, may be null).
hipError_t launch_permute(double* X, int64_t ldx, int rows, int bj, const int* src_top,
                          const int* dst_low, int64_t* jpvt, hipStream_t s);

hipError_t launch_iota(int64_t* v, int n, hipStream_t s);
hipError_t launch_zero_u32(uint32_t* v, int n, hipStream_t s);
hipError_t launch_copy2d(const double* src, int64_t lds, double* dst, int64_t ldd, int rows,
                         int cols, hipStream_t s);

}  // namespace rq
