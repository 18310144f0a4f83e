// BF16 MFMA contractions for the mixed-precision path: operands are rounded to
// BF16 (round to nearest even; FP64 operands pass through FP32 first), products
// accumulate in FP32 and results are stored in FP64.
//   * gemm_lx_bf16 : D(P x N) = L(P x K) X(K x N), X an FP32 matrix read through
//                    an optional column map (the sketch Omega A and Y2^T A P);
//                    L is staged once per launch as BF16 in a workspace;
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

// L (P x K, FP64 with strides) rounded to BF16 (through FP32) into a
// row-major 16 PB x Kpad array with k contiguous, zero-padded, so that a lane's
// 8 consecutive k of one row are one 16-byte load.
__global__ void stage_l_bf16_kernel(const double* L, int64_t sLp, int64_t sLk, int P, int K,
                                    int rows, int kpad, __bf16* out) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)rows * kpad) return;
  const int p = (int)(e / kpad), k = (int)(e % kpad);
  out[e] = (__bf16)(float)((p < P && k < K) ? L[(int64_t)p * sLp + (int64_t)k * sLk] : 0.0);
}

// D(P x N) = L(P x K) X(K x N): a workgroup owns 16 NB columns and all P rows
// over one K chunk; its four waves take interleaved 32-row groups of the chunk
// (wave w: groups w, w + 4, ...) and each holds the PB x NB block of FP32
// accumulators.  The waves' sums are combined in LDS as (w0 + w2) + (w1 + w3).
template <int PB, int NB, bool X16>
__global__ __launch_bounds__(256, 2) void gemm_lx_bf16_kernel(GemmArgsF g) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int l16 = lane & 15;
  const int kq = lane >> 4;
  const int kb = blockIdx.y * g.kchunk;
  const int ke = min(g.K, kb + g.kchunk);
  const float* xc[NB];
  bool nok[NB];
#pragma unroll
  for (int jb = 0; jb < NB; ++jb) {
    const int n = blockIdx.x * 16 * NB + 16 * jb + l16;
    nok[jb] = n < g.N;
    xc[jb] = g.X + (nok[jb] ? (g.xcol ? g.xcol[n] : (int64_t)n) : 0) * g.ldx;
  }
  fx4 acc[PB][NB];
#pragma unroll
  for (int i = 0; i < PB; ++i)
#pragma unroll
    for (int jb = 0; jb < NB; ++jb) acc[i][jb] = fx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
  for (int k0 = kb + 32 * wave; k0 < ke; k0 += 128) {
    const int kk = k0 + 8 * kq;
    bf16x8 xb[NB], la[PB];
    const bool full = kk + 8 <= ke;
#pragma unroll
    for (int jb = 0; jb < NB; ++jb) {
      if (X16 && full && nok[jb]) {
        const float4 u = *reinterpret_cast<const float4*>(xc[jb] + kk);
        const float4 v = *reinterpret_cast<const float4*>(xc[jb] + kk + 4);
        xb[jb][0] = (__bf16)u.x; xb[jb][1] = (__bf16)u.y; xb[jb][2] = (__bf16)u.z; xb[jb][3] = (__bf16)u.w;
        xb[jb][4] = (__bf16)v.x; xb[jb][5] = (__bf16)v.y; xb[jb][6] = (__bf16)v.z; xb[jb][7] = (__bf16)v.w;
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) xb[jb][e] = (__bf16)((nok[jb] && kk + e < ke) ? xc[jb][kk + e] : 0.f);
      }
    }
#pragma unroll
    for (int i = 0; i < PB; ++i)
      la[i] = *reinterpret_cast<const bf16x8*>(g.lbf + (int64_t)(16 * i + l16) * g.kpad + kk);
#pragma unroll
    for (int i = 0; i < PB; ++i)
#pragma unroll
      for (int jb = 0; jb < NB; ++jb) acc[i][jb] = mfma_bf16(la[i], xb[jb], acc[i][jb]);
  }
  constexpr int E = PB * NB * 4;
  __shared__ float s_red[2][E][64];
  if (wave >= 2) {
#pragma unroll
    for (int i = 0; i < PB; ++i)
#pragma unroll
      for (int jb = 0; jb < NB; ++jb)
#pragma unroll
        for (int v = 0; v < 4; ++v) s_red[wave - 2][(i * NB + jb) * 4 + v][lane] = acc[i][jb][v];
  }
  __syncthreads();
  if (wave < 2) {
#pragma unroll
    for (int i = 0; i < PB; ++i)
#pragma unroll
      for (int jb = 0; jb < NB; ++jb)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[i][jb][v] += s_red[wave][(i * NB + jb) * 4 + v][lane];
  }
  __syncthreads();
  if (wave == 1) {
#pragma unroll
    for (int i = 0; i < PB; ++i)
#pragma unroll
      for (int jb = 0; jb < NB; ++jb)
#pragma unroll
        for (int v = 0; v < 4; ++v) s_red[0][(i * NB + jb) * 4 + v][lane] = acc[i][jb][v];
  }
  __syncthreads();
  if (wave != 0) return;
  double* o = g.out + (int64_t)blockIdx.y * g.split_stride;
#pragma unroll
  for (int jb = 0; jb < NB; ++jb) {
    if (!nok[jb]) continue;
    const int64_t n = blockIdx.x * 16 * NB + 16 * jb + l16;
#pragma unroll
    for (int i = 0; i < PB; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int p = 16 * i + 4 * kq + v;
        if (p < g.P) o[p + n * g.ldout] = (double)(acc[i][jb][v] + s_red[0][(i * NB + jb) * 4 + v][lane]);
      }
  }
}

int bf16_stage_kpad(int K) { return ((K + 31) / 32) * 32 + 32; }

hipError_t launch_gemm_lx_bf16(const GemmArgsF& g, hipStream_t s) {
  if (g.N <= 0 || g.P <= 0) return hipSuccess;
  if (!g.lbf || g.kchunk <= 0 || g.kchunk % 32 != 0) return hipErrorInvalidValue;
  const int pb = (g.P + 15) / 16;
  if (pb > 6) return hipErrorInvalidValue;
  GemmArgsF h = g;
  h.kpad = bf16_stage_kpad(g.K);
  const int64_t total = (int64_t)16 * pb * h.kpad;
  hipLaunchKernelGGL(stage_l_bf16_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     g.L, g.sLp, g.sLk, g.P, g.K, 16 * pb, h.kpad, h.lbf);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int cols = pb <= 4 ? 64 : 32;
  dim3 grid((g.N + cols - 1) / cols, g.ksplit);
  const bool x16 = (reinterpret_cast<uintptr_t>(g.X) % 16 == 0) && (g.ldx % 4 == 0);
#define RQ_LXB(pb_, nb_)                                                                    \
  case pb_:                                                                                 \
    if (x16)                                                                                \
      hipLaunchKernelGGL((gemm_lx_bf16_kernel<pb_, nb_, true>), grid, dim3(256), 0, s, h);  \
    else                                                                                    \
      hipLaunchKernelGGL((gemm_lx_bf16_kernel<pb_, nb_, false>), grid, dim3(256), 0, s, h); \
    break;
  switch (pb) {
    RQ_LXB(1, 4)
    RQ_LXB(2, 4)
    RQ_LXB(3, 4)
    RQ_LXB(4, 4)
    RQ_LXB(5, 2)
    RQ_LXB(6, 2)
#undef RQ_LXB
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
