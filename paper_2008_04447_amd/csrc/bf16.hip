// BF16 MFMA contractions for the mixed-precision path: operands are rounded to
// BF16 (round to nearest even; FP64 operands pass through FP32 first), products
// accumulate in FP32 and results are stored in FP64.
//   * gemm_lx_bf16 : D(P x N) = L(P x K) X(K x N), X an FP32 matrix read through
//                    an optional column map (the sketch Omega A and Y2^T A P);
//                    L is staged once per launch as BF16 in a workspace;
//   * gemm_nn_bf16 : C(M x N) = Y(M x K) Z(K x N), Y FP32 (Z1 = A V of TUXV);
//                    Z is staged once as BF16 in a workspace.
// v_mfma_f32_16x16x32_bf16: lane l supplies A[l % 16][8 (l / 16) + e] and
// B[8 (l / 16) + e][l % 16] (e = 0..7) and holds D[4 (l / 16) + i][l % 16].
#include "device_common.hpp"
#include "kernels.hpp"

namespace rq {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
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

// ---- C(M x N) = Y(M x K) Z(K x N) ----------------------------------------
// The one extra pass over A in TUXV (Z1 = A V): Y is the FP32 input, column-major,
// so its rows are contiguous and a 64-row tile of one column is 256 bytes.
//   * Z is staged once as BF16, step-major: the 64 k of step s for all ncp
//     padded columns form one contiguous block, so the slab every workgroup
//     needs at step s is 64 ncp consecutive values (cache- and TLB-friendly).
//   * A workgroup owns 64 rows of C and 64 NBW columns (all of N when N <= 256),
//     so Y is read once.  Per 64-k step its 256 threads load the 64 x 64 Y tile
//     with float4 loads along rows (4 rows x 4 columns per thread), round it to
//     BF16 and store it to LDS row-major (k contiguous), from which each lane
//     reads the 8 consecutive k of one row an MFMA operand needs.
//   * Wave w owns columns 16 NBW w ..; its Z fragments come straight from the
//     staged array.  Loads run ahead of use: the Y tile of step s + 2 is issued
//     during step s (two register sets), and each half-step's Z fragments are
//     replaced by the next step's as soon as they are consumed, Z before Y so
//     that waiting for Z never waits for the later Y tile.
//   * Rows at or past M in the last tile are clamped to valid rows and their
//     results dropped; columns past K (the K tail) are zero.
// Products run in the same order as a plain k-ordered loop of 16x16x32 MFMAs.
constexpr int kNnK = 64;      // k per pipeline step
constexpr int kNnLd = 72;     // LDS row stride of the BF16 Y tile (elements; 144 bytes)

static int nn_nbw(int N) { return N > 192 ? 4 : N > 128 ? 3 : N > 64 ? 2 : 1; }
static int nn_ncp(int N) {
  const int cols = 64 * nn_nbw(N);
  return ((N + cols - 1) / cols) * cols;
}
int64_t gemm_nn_bf16_stage_elems(int N, int K) {
  return (int64_t)nn_ncp(N) * (((K + kNnK - 1) / kNnK) * kNnK);
}

// Z (K x N, FP64) through FP32 to BF16: element (k, c) at
// ((k / 64) ncp + c) 64 + k % 64, zero for c >= N or k >= K.
__global__ void stage_z_bf16_kernel(const double* Z, int64_t ldz, int N, int K, int ncp, int64_t total,
                                    __bf16* zt) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int kk = (int)(e & 63);
  const int64_t sc = e >> 6;
  const int c = (int)(sc % ncp);
  const int k = (int)(sc / ncp) * kNnK + kk;
  zt[e] = (__bf16)(float)((c < N && k < K) ? Z[k + (int64_t)c * ldz] : 0.0);
}

// The K loop of one workgroup of 64 RB rows.  VEC: Y 16-byte aligned, ldy and
// M multiples of 4 and ldy < 2^26 (32-bit lane offsets); otherwise element loads.
template <int NBW, int RB, bool VEC>
RQ_DEV void nn_tile(fx4 (&acc)[4 * RB][NBW], __bf16 (*s_y)[64 * RB * kNnLd], int M, const float* Y,
                    int64_t ldy, const __bf16* zt, int ncp, int K, int r0, int cw) {
  constexpr int CPT = 4 * RB;           // columns of the step each loader thread reads
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int l16 = lane & 15, kq = lane >> 4;
  const int rg = t % (16 * RB), kc = t / (16 * RB);   // rows 4 rg .. 4 rg + 3, columns CPT kc ..
  // wave-uniform bases plus per-lane offsets
  const float* yw = Y + r0;
  const uint32_t yoff = (uint32_t)min(4 * rg, M - 4 - r0) + (uint32_t)(CPT * kc) * (uint32_t)ldy;
  int64_t yoq[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) yoq[q] = min(4 * rg + q, M - 1 - r0) + (int64_t)(CPT * kc) * ldy;
  const __bf16* zw = zt + (int64_t)cw * kNnK;
  const uint32_t zoff = (uint32_t)(l16 * kNnK + 8 * kq);
  const int nsteps = (K + kNnK - 1) / kNnK;
  const int nfull = K / kNnK;   // steps whose 64 columns are all below K

  auto load_y = [&](fx4 (&u)[CPT], int s) {
    const float* p = yw + (int64_t)(s * kNnK) * ldy;
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
      const float* pe = p + (int64_t)e * ldy;
      if (VEC) {
        u[e] = __builtin_nontemporal_load(reinterpret_cast<const fx4*>(pe + yoff));
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) u[e][q] = __builtin_nontemporal_load(pe + yoq[q]);
      }
    }
  };
  auto load_y_tail = [&](fx4 (&u)[CPT], int s) {
    const int k0 = s * kNnK;
#pragma unroll
    for (int e = 0; e < CPT; ++e) {
      const float* pe = yw + (int64_t)(k0 + e) * ldy;
      const bool ok = k0 + CPT * kc + e < K;
      if (VEC) {
        u[e] = ok ? *reinterpret_cast<const fx4*>(pe + yoff) : fx4{0.f, 0.f, 0.f, 0.f};
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) u[e][q] = ok ? pe[yoq[q]] : 0.f;
      }
    }
  };
  auto zfrag = [&](int s, int h, int jb) {
    return *reinterpret_cast<const bf16x8*>((zw + ((int64_t)s * ncp + 16 * jb) * kNnK + 32 * h) + zoff);
  };
  auto store_y = [&](__bf16* buf, const fx4 (&u)[CPT]) {
    __bf16* p = buf + (4 * rg) * kNnLd + CPT * kc;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
#pragma unroll
      for (int e0 = 0; e0 < CPT; e0 += 4)
        *reinterpret_cast<bf16x4*>(p + q * kNnLd + e0) =
            bf16x4{(__bf16)u[e0][q], (__bf16)u[e0 + 1][q], (__bf16)u[e0 + 2][q], (__bf16)u[e0 + 3][q]};
    }
  };
  // MFMAs of one step from the LDS tile and the fragments in z; each half's
  // fragments are then replaced by those of step snext (always a valid step).
  auto compute = [&](const __bf16* buf, bf16x8 (&z)[2][NBW], int snext) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int ib = 0; ib < 4 * RB; ++ib) {
        const bf16x8 yf =
            *reinterpret_cast<const bf16x8*>(buf + (16 * ib + l16) * kNnLd + 32 * h + 8 * kq);
#pragma unroll
        for (int jb = 0; jb < NBW; ++jb) acc[ib][jb] = mfma_bf16(z[h][jb], yf, acc[ib][jb]);
      }
#pragma unroll
      for (int jb = 0; jb < NBW; ++jb) z[h][jb] = zfrag(snext, h, jb);
    }
  };
  if (nsteps == 0) return;
  const int last = nsteps - 1;
  fx4 ya[CPT], yb[CPT];
  bf16x8 z[2][NBW];
  auto load_z0 = [&]() {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int jb = 0; jb < NBW; ++jb) z[h][jb] = zfrag(0, h, jb);
  };
  if (nfull > 0) {
    // Full steps without branches around loads: a prefetch past the last full
    // step reloads that step (in range, unused), so the compiler's waits are
    // plain in-order counts.  The prologue issues loads in the loop's order.
    const int lf = nfull - 1;
    load_y(ya, 0);
    load_z0();
    load_y(yb, min(1, lf));
    int s = 0;
#pragma unroll 1
    for (; s + 1 < nfull; s += 2) {
      store_y(s_y[0], ya);
      __syncthreads();
      compute(s_y[0], z, s + 1);
      __builtin_amdgcn_sched_barrier(0);
      load_y(ya, min(s + 2, lf));
      store_y(s_y[1], yb);
      __syncthreads();
      compute(s_y[1], z, min(s + 2, last));
      __builtin_amdgcn_sched_barrier(0);
      load_y(yb, min(s + 3, lf));
    }
    if (s < nfull) {   // odd number of full steps: the last one is in ya
      store_y(s_y[0], ya);
      __syncthreads();
      compute(s_y[0], z, min(s + 1, last));
    }
  } else {
    load_z0();
  }
  if (nfull < nsteps) {   // K tail (z already holds this step)
    load_y_tail(ya, nfull);
    __syncthreads();
    store_y(s_y[0], ya);
    __syncthreads();
    compute(s_y[0], z, last);
  }
}

template <int NBW, int RB>
__global__ __launch_bounds__(256, 3 - RB) void gemm_nn_bf16_kernel(double* C, int64_t ldc, int M, int N,
                                                              const float* Y, int64_t ldy,
                                                              const __bf16* zt, int ncp, int K,
                                                              int vec) {
  __shared__ __align__(16) __bf16 s_y[2][64 * RB * kNnLd];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l16 = lane & 15, kq = lane >> 4;
  const int r0 = blockIdx.x * 64 * RB;
  const int cw = blockIdx.y * 64 * NBW + 16 * NBW * wave;
  fx4 acc[4 * RB][NBW];
#pragma unroll
  for (int ib = 0; ib < 4 * RB; ++ib)
#pragma unroll
    for (int jb = 0; jb < NBW; ++jb) acc[ib][jb] = fx4{0.f, 0.f, 0.f, 0.f};
  if (vec)
    nn_tile<NBW, RB, true>(acc, s_y, M, Y, ldy, zt, ncp, K, r0, cw);
  else
    nn_tile<NBW, RB, false>(acc, s_y, M, Y, ldy, zt, ncp, K, r0, cw);
  // lane holds C(r0 + 16 ib + l16, cw + 16 jb + 4 kq + v)
#pragma unroll
  for (int ib = 0; ib < 4 * RB; ++ib) {
    const int r = r0 + 16 * ib + l16;
#pragma unroll
    for (int jb = 0; jb < NBW; ++jb)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int cc = cw + 16 * jb + 4 * kq + v;
        if (r < M && cc < N) C[r + (int64_t)cc * ldc] = (double)acc[ib][jb][v];
      }
  }
}

hipError_t launch_gemm_nn_bf16(double* C, int64_t ldc, int M, int N, const float* Y, int64_t ldy,
                               const double* Z, int64_t ldz, int K, __bf16* zbf, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (ldy < M || ldc < M || (K > 0 && !zbf)) return hipErrorInvalidValue;
  const int nbw = nn_nbw(N), ncp = nn_ncp(N);
  const int64_t total = gemm_nn_bf16_stage_elems(N, K);
  if (total > 0) {
    hipLaunchKernelGGL(stage_z_bf16_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, Z,
                       ldz, N, K, ncp, total, zbf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int vec = (reinterpret_cast<uintptr_t>(Y) % 16 == 0) && (ldy % 4 == 0) && (M % 4 == 0) &&
                  ldy < (1 << 26);
  // 128 rows per workgroup when there are enough rows to fill the device that
  // way (V, read by every workgroup, then costs half as much per row)
  const int rb = ((int64_t)M >= 128 * 256) ? 2 : 1;
  dim3 grid((M + 64 * rb - 1) / (64 * rb), ncp / (64 * nbw));
#define RQ_NN(nbw_, rb_) \
  hipLaunchKernelGGL((gemm_nn_bf16_kernel<nbw_, rb_>), grid, dim3(256), 0, s, C, ldc, M, N, Y, ldy, zbf, ncp, K, vec)
  if (rb == 2) {
    switch (nbw) {
      case 1: RQ_NN(1, 2); break;
      case 2: RQ_NN(2, 2); break;
      case 3: RQ_NN(3, 2); break;
      default: RQ_NN(4, 2); break;
    }
  } else {
    switch (nbw) {
      case 1: RQ_NN(1, 1); break;
      case 2: RQ_NN(2, 1); break;
      case 3: RQ_NN(3, 1); break;
      default: RQ_NN(4, 1); break;
    }
  }
#undef RQ_NN
  return hipGetLastError();
}

}  // namespace rq
