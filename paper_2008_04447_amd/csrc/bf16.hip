// BF16 MFMA contractions for the mixed-precision path: operands are rounded to
// BF16 (round to nearest even; FP64 operands pass through FP32 first), products
// accumulate in FP32 and results are stored in FP64.
//   * gemm_lx_bf16 : D(P x N) = L(P x K) X(K x N), X an FP32 matrix read through
//                    an optional column map (the sketch Omega A and Y2^T A P);
//   * gemm_nn_bf16 : C(M x N) = Y(M x K) Z(K x N), Y FP32 (Z1 = A V of TUXV).
// v_mfma_f32_16x16x32_bf16: lane l supplies A[l % 16][8 (l / 16) + e] and
// B[8 (l / 16) + e][l % 16] (e = 0..7) and holds D[4 (l / 16) + i][l % 16].
#include "device_common.hpp"
#include "kernels.hpp"

namespace rq {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float fx4 __attribute__((ext_vector_type(4)));

RQ_DEV fx4 mfma_bf16(bf16x8 a, bf16x8 b, fx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <int PB>
__global__ __launch_bounds__(256) void gemm_lx_bf16_kernel(GemmArgsF g) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + wave * 16 + (lane & 15);
  const int kq = lane >> 4;
  const int kb = blockIdx.y * g.kchunk;
  const int ke = min(g.K, kb + g.kchunk);
  const bool nok = n < g.N;
  const float* xc = g.X + (nok ? (g.xcol ? g.xcol[n] : (int64_t)n) : 0) * g.ldx;
  fx4 acc[PB];
#pragma unroll
  for (int i = 0; i < PB; ++i) acc[i] = fx4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += 32) {
    const int kk = k0 + 8 * kq;
    bf16x8 xb;
#pragma unroll
    for (int e = 0; e < 8; ++e) xb[e] = (__bf16)((nok && kk + e < ke) ? xc[kk + e] : 0.f);
#pragma unroll
    for (int i = 0; i < PB; ++i) {
      const int p = 16 * i + (lane & 15);
      bf16x8 la;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        la[e] = (__bf16)(float)((p < g.P && kk + e < ke)
                                    ? g.L[(int64_t)p * g.sLp + (int64_t)(kk + e) * g.sLk]
                                    : 0.0);
      acc[i] = mfma_bf16(la, xb, acc[i]);
    }
  }
  if (!nok) return;
  double* o = g.out + (int64_t)blockIdx.y * g.split_stride;
#pragma unroll
  for (int i = 0; i < PB; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int p = 16 * i + 4 * kq + v;
      if (p < g.P) o[p + (int64_t)n * g.ldout] = (double)acc[i][v];
    }
}

hipError_t launch_gemm_lx_bf16(const GemmArgsF& g, hipStream_t s) {
  if (g.N <= 0 || g.P <= 0) return hipSuccess;
  const int pb = (g.P + 15) / 16;
  dim3 grid((g.N + 63) / 64, g.ksplit);
  switch (pb) {
    case 1: hipLaunchKernelGGL(gemm_lx_bf16_kernel<1>, grid, dim3(256), 0, s, g); break;
    case 2: hipLaunchKernelGGL(gemm_lx_bf16_kernel<2>, grid, dim3(256), 0, s, g); break;
    case 3: hipLaunchKernelGGL(gemm_lx_bf16_kernel<3>, grid, dim3(256), 0, s, g); break;
    case 4: hipLaunchKernelGGL(gemm_lx_bf16_kernel<4>, grid, dim3(256), 0, s, g); break;
    case 5: hipLaunchKernelGGL(gemm_lx_bf16_kernel<5>, grid, dim3(256), 0, s, g); break;
    case 6: hipLaunchKernelGGL(gemm_lx_bf16_kernel<6>, grid, dim3(256), 0, s, g); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// C(M x N) = Y(M x K) Z(K x N): 64 x 64 tile per workgroup, wave (wr, wc) owns
// 32 x 32 as 2 x 2 blocks of C^T (so 16 lanes store 16 consecutive rows).
__global__ __launch_bounds__(256) void gemm_nn_bf16_kernel(double* C, int64_t ldc, int M, int N,
                                                          const float* Y, int64_t ldy,
                                                          const double* Z, int64_t ldz, int K) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int rb = blockIdx.x * 64 + (wave & 1) * 32;
  const int cb = blockIdx.y * 64 + (wave >> 1) * 32;
  const int l16 = lane & 15;
  const int kq = lane >> 4;
  fx4 acc[2][2];
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) acc[ib][jb] = fx4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 32) {
    const int kk = k0 + 8 * kq;
    bf16x8 za[2], yb[2];
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
      const int cc = cb + 16 * jb + l16;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        za[jb][e] = (__bf16)(float)((cc < N && kk + e < K) ? Z[(kk + e) + (int64_t)cc * ldz] : 0.0);
    }
#pragma unroll
    for (int ib = 0; ib < 2; ++ib) {
      const int r = rb + 16 * ib + l16;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        yb[ib][e] = (__bf16)((r < M && kk + e < K) ? Y[r + (int64_t)(kk + e) * ldy] : 0.f);
    }
#pragma unroll
    for (int ib = 0; ib < 2; ++ib)
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) acc[ib][jb] = mfma_bf16(za[jb], yb[ib], acc[ib][jb]);
  }
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
      const int r = rb + 16 * ib + l16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int cc = cb + 16 * jb + 4 * kq + v;
        if (r < M && cc < N) C[r + (int64_t)cc * ldc] = (double)acc[ib][jb][v];
      }
    }
}

hipError_t launch_gemm_nn_bf16(double* C, int64_t ldc, int M, int N, const float* Y, int64_t ldy,
                               const double* Z, int64_t ldz, int K, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 grid((M + 63) / 64, (N + 63) / 64);
  hipLaunchKernelGGL(gemm_nn_bf16_kernel, grid, dim3(256), 0, s, C, ldc, M, N, Y, ldy, Z, ldz, K);
  return hipGetLastError();
}

}  // namespace rq
