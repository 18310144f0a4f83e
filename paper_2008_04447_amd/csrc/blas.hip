// FP64 MFMA contractions and the small kernels of the block loop:
//   * gemm_lx  : D(P x N) = L(P x K) X(K x N) with short P (the sketch Omega A,
//                the inner products Y^T A, and the sample update S12 - M R12);
//   * reduce   : fixed-order sum of split-K partials, optionally Z = T^T W;
//   * update   : trailing update C -= Y Z (the block reflection of Algorithm 4);
//   * omega11  : Omega_hat_11 = S11 R11^{-1} (eq. update1);
//   * permute  : column permutation of a block of pivots.
#include "device_common.hpp"
#include "kernels.hpp"

#include <algorithm>

namespace rq {

// ---------------------------------------------------------------------------
// gemm_lx for short K (at most 64 per chunk): each workgroup owns 64 output
// columns (16 per wave) and all P rows (PB blocks of 16), over one K chunk.  The K index of MFMA step s in lane l is
// k0 + 4 * (l / 16) + s, so each lane reads 4 consecutive rows of X per group of
// 16 k values (both operands use the same ordering of k).
template <int PB>
__global__ __launch_bounds__(256) void gemm_lx_narrow_kernel(GemmArgs g) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + wave * 16 + (lane & 15);
  const int kq = lane >> 4;
  const int kb = blockIdx.y * g.kchunk;
  const int ke = min(g.K, kb + g.kchunk);
  const bool nok = n < g.N;
  const double* xc = g.X + (nok ? (g.xcol ? g.xcol[n] : (int64_t)n) : 0) * g.ldx;
  dx4 acc[PB];
#pragma unroll
  for (int i = 0; i < PB; ++i) acc[i] = dx4{0.0, 0.0, 0.0, 0.0};

  // the chunk has at most 64 rows of K (four groups of 16): every operand, and
  // the C values of the epilogue, is requested before the first product
  double xb[4][4];
  double la[4][PB][4];
#pragma unroll
  for (int c4 = 0; c4 < 4; ++c4) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = kb + 16 * c4 + 4 * kq + s;
      xb[c4][s] = (nok && k < ke) ? xc[k] : 0.0;
#pragma unroll
      for (int i = 0; i < PB; ++i) {
        const int p = 16 * i + (lane & 15);
        la[c4][i][s] = (p < g.P && k < ke) ? g.L[(int64_t)p * g.sLp + (int64_t)k * g.sLk] : 0.0;
      }
    }
  }
  const bool epi_c = g.ksplit == 1 && g.beta != 0.0 && nok;
  double cv[PB][4];
#pragma unroll
  for (int i = 0; i < PB; ++i)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int p = 16 * i + kq + 4 * v;
      cv[i][v] = (epi_c && p < g.P) ? g.C[p + (int64_t)n * g.ldc] : 0.0;
    }
  // the skip flag is read after the operands are requested (they are in bounds
  // either way), so its round trip overlaps theirs; nothing is stored before it
  if (g.skip_if && __hip_atomic_load(g.skip_if, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
    return;
#pragma unroll
  for (int c4 = 0; c4 < 4; ++c4) {
    if (kb + 16 * c4 >= ke) break;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < PB; ++i) acc[i] = mfma_f64(la[c4][i][s], xb[c4][s], acc[i]);
  }
  if (!nok) return;
  if (g.ksplit > 1) {
    double* o = g.out + (int64_t)blockIdx.y * g.split_stride;
#pragma unroll
    for (int i = 0; i < PB; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int p = 16 * i + kq + 4 * v;
        if (p < g.P) o[p + (int64_t)n * g.ldout] = acc[i][v];
      }
  } else {
#pragma unroll
    for (int i = 0; i < PB; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int p = 16 * i + kq + 4 * v;
        if (p < g.P) {
          double r = g.alpha * acc[i][v];
          if (g.beta != 0.0) r += g.beta * cv[i][v];
          g.out[p + (int64_t)n * g.ldout] = r;
        }
      }
  }
}

// ---------------------------------------------------------------------------
// gemm_lx: a workgroup owns 16 * NB output columns and all P rows (PB blocks of
// 16) over one K chunk; its four waves take interleaved 16-row groups of the
// chunk (wave w: groups w, w + 4, ...) and each holds the whole PB x NB block of
// accumulators, so every loaded operand feeds PB or NB matrix-core products.
// The K index of MFMA step s in lane l is k0 + 4 * (l / 16) + s: each lane reads
// 4 consecutive rows of X (and of L when its k stride is 1) per group of 16 k.
// The four waves' sums are combined in LDS in a fixed order, (w0 + w2) + (w1 + w3).
template <int PB, int NB, bool LK1>
__global__ __launch_bounds__(256, 2) void gemm_lx_kernel(GemmArgs g) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int l16 = lane & 15;
  const int kq = lane >> 4;
  const int kb = blockIdx.y * g.kchunk;
  const int ke = min(g.K, kb + g.kchunk);
  const double* xc[NB];
  bool nok[NB];
#pragma unroll
  for (int jb = 0; jb < NB; ++jb) {
    const int n = blockIdx.x * 16 * NB + 16 * jb + l16;
    nok[jb] = n < g.N;
    xc[jb] = g.X + (nok[jb] ? (g.xcol ? g.xcol[n] : (int64_t)n) : 0) * g.ldx + 4 * kq;
  }
  // row 16 i + l16 of L (clamped: rows p >= P are never used), at k = 4 kq
  const double* lr[PB];
#pragma unroll
  for (int i = 0; i < PB; ++i)
    lr[i] = g.L + (int64_t)min(16 * i + l16, g.P - 1) * g.sLp + (int64_t)(4 * kq) * g.sLk;
  dx4 acc[PB][NB];
#pragma unroll
  for (int i = 0; i < PB; ++i)
#pragma unroll
    for (int jb = 0; jb < NB; ++jb) acc[i][jb] = dx4{0.0, 0.0, 0.0, 0.0};

#pragma unroll 1
  for (int k0 = kb + 16 * wave; k0 < ke; k0 += 64) {
    double la[PB][4], xb[NB][4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const bool kok = k0 + 4 * kq + s < ke;
#pragma unroll
      for (int jb = 0; jb < NB; ++jb) xb[jb][s] = (nok[jb] && kok) ? xc[jb][k0 + s] : 0.0;
#pragma unroll
      for (int i = 0; i < PB; ++i) {
        const bool ok = 16 * i + l16 < g.P && kok;
        if (LK1)
          la[i][s] = ok ? lr[i][k0 + s] : 0.0;
        else
          la[i][s] = ok ? lr[i][(int64_t)(k0 + s) * g.sLk] : 0.0;
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < PB; ++i)
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) acc[i][jb] = mfma_f64(la[i][s], xb[jb][s], acc[i][jb]);
  }
  // ---- combine the four waves: (w0 + w2) + (w1 + w3) ---------------------------
  constexpr int E = PB * NB * 4;
  __shared__ double s_red[2][E][64];
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
#pragma unroll
  for (int i = 0; i < PB; ++i)
#pragma unroll
    for (int jb = 0; jb < NB; ++jb)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][jb][v] += s_red[0][(i * NB + jb) * 4 + v][lane];
  // lane holds D[16 i + kq + 4 v][column 16 jb + l16]
  double* o = g.out + (g.ksplit > 1 ? (int64_t)blockIdx.y * g.split_stride : 0);
#pragma unroll
  for (int jb = 0; jb < NB; ++jb) {
    if (!nok[jb]) continue;
    const int64_t n = blockIdx.x * 16 * NB + 16 * jb + l16;
#pragma unroll
    for (int i = 0; i < PB; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int p = 16 * i + kq + 4 * v;
        if (p >= g.P) continue;
        if (g.ksplit > 1) {
          o[p + n * g.ldout] = acc[i][jb][v];
        } else {
          double r = g.alpha * acc[i][jb][v];
          if (g.beta != 0.0) r += g.beta * g.C[p + n * g.ldc];
          o[p + n * g.ldout] = r;
        }
      }
  }
}

// ---------------------------------------------------------------------------
// gemm_lx for L with unit k stride and P <= 64 (the W = Y^T A of every block):
// the same split of the work as gemm_lx_kernel with 32 output columns per
// workgroup, one wave per SIMD and the operands of the next two 16-row groups
// in flight while the matrix cores work on the current one (a ring of three
// register sets, so no set is ever copied).  Rows of full groups are read
// without masks; only a final partial group is masked.  Rows p >= P of L are
// clamped to row P - 1: they only feed output rows that are not stored.
template <int PB>
__global__ __launch_bounds__(256, 1) void gemm_lx_ring_kernel(GemmArgs g) {
  constexpr int NB = 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  const int kb = blockIdx.y * g.kchunk;
  const int ke = min(g.K, kb + g.kchunk);
  const int first = kb + 16 * wave;               // this wave's groups: first + 64 i
  const double* const Lb = (g.alt_if && *g.alt_if) ? g.L_alt : g.L;
  bool nok[NB];
  const double* xp[NB];
  const double* lp[PB];
#pragma unroll
  for (int jb = 0; jb < NB; ++jb) {
    const int n = blockIdx.x * 16 * NB + 16 * jb + l16;
    nok[jb] = n < g.N;
    xp[jb] = g.X + (nok[jb] ? (g.xcol ? g.xcol[n] : (int64_t)n) : 0) * g.ldx + first + 4 * kq;
  }
#pragma unroll
  for (int i = 0; i < PB; ++i)
    lp[i] = Lb + (int64_t)min(16 * i + l16, g.P - 1) * g.sLp + first + 4 * kq;
  dx4 acc[PB][NB];
#pragma unroll
  for (int i = 0; i < PB; ++i)
#pragma unroll
    for (int jb = 0; jb < NB; ++jb) acc[i][jb] = dx4{0.0, 0.0, 0.0, 0.0};
  struct Ops {
    double la[PB][4], xb[NB][4];
  };
  auto load = [&](int grp, Ops& o) {
#pragma unroll
    for (int jb = 0; jb < NB; ++jb)
#pragma unroll
      for (int s = 0; s < 4; ++s) o.xb[jb][s] = xp[jb][64 * grp + s];
#pragma unroll
    for (int i = 0; i < PB; ++i)
#pragma unroll
      for (int s = 0; s < 4; ++s) o.la[i][s] = lp[i][64 * grp + s];
  };
  auto compute = [&](const Ops& o) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int i = 0; i < PB; ++i)
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) acc[i][jb] = mfma_f64(o.la[i][s], o.xb[jb][s], acc[i][jb]);
  };
  const int nfull = (ke >= first + 16) ? (ke - first - 16) / 64 + 1 : 0;
  {
    Ops A, B, Cr;
    if (nfull > 0) load(0, A);
    if (nfull > 1) load(1, B);
    for (int i = 0; i < nfull; i += 3) {
      if (i + 2 < nfull) load(i + 2, Cr);
      compute(A);
      if (i + 1 >= nfull) break;
      if (i + 3 < nfull) load(i + 3, A);
      compute(B);
      if (i + 2 >= nfull) break;
      if (i + 4 < nfull) load(i + 4, B);
      compute(Cr);
    }
  }
  {
    const int k0 = first + 64 * nfull;            // a final partial group
    if (k0 < ke) {
      Ops o;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const bool kok = k0 + 4 * kq + s < ke;
#pragma unroll
        for (int jb = 0; jb < NB; ++jb) o.xb[jb][s] = kok ? xp[jb][64 * nfull + s] : 0.0;
#pragma unroll
        for (int i = 0; i < PB; ++i) o.la[i][s] = kok ? lp[i][64 * nfull + s] : 0.0;
      }
      compute(o);
    }
  }
  // ---- combine the four waves: (w0 + w2) + (w1 + w3) ---------------------------
  constexpr int E = PB * NB * 4;
  __shared__ double s_red[2][E][64];
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
#pragma unroll
  for (int i = 0; i < PB; ++i)
#pragma unroll
    for (int jb = 0; jb < NB; ++jb)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[i][jb][v] += s_red[0][(i * NB + jb) * 4 + v][lane];
  // lane holds D[16 i + kq + 4 v][column 16 jb + l16]
  double* o = g.out + (g.ksplit > 1 ? (int64_t)blockIdx.y * g.split_stride : 0);
#pragma unroll
  for (int jb = 0; jb < NB; ++jb) {
    if (!nok[jb]) continue;
    const int64_t n = blockIdx.x * 16 * NB + 16 * jb + l16;
#pragma unroll
    for (int i = 0; i < PB; ++i)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int p = 16 * i + kq + 4 * v;
        if (p >= g.P) continue;
        if (g.ksplit > 1) {
          o[p + n * g.ldout] = acc[i][jb][v];
        } else {
          double r = g.alpha * acc[i][jb][v];
          if (g.beta != 0.0) r += g.beta * g.C[p + n * g.ldc];
          o[p + n * g.ldout] = r;
        }
      }
  }
}

// Split of K for a product with N output columns: about `target` workgroups
// of `cols` columns each, at least 64 rows per wave, chunks a multiple of 64.
void plan_split_target(int K, int N, int cols, int target, int* ksplit, int* kchunk) {
  const int tiles = (N + cols - 1) / cols;
  int ks = (target + tiles - 1) / tiles;
  const int kmax = (K + 255) / 256;
  if (ks > kmax) ks = kmax;
  if (ks > 32) ks = 32;
  if (ks < 1) ks = 1;
  int kc = (K + ks - 1) / ks;
  kc = ((kc + 63) / 64) * 64;
  if (kc < 64) kc = 64;
  ks = (K + kc - 1) / kc;
  if (ks < 1) ks = 1;
  *ksplit = ks;
  *kchunk = kc;
}

// Split for the ring kernel (P <= 64) by resident rounds: with `slots`
// workgroups resident at once, the ks (at most 8) that minimizes the rounds
// times the rows each workgroup streams, plus a fixed cost of 320 rows per
// workgroup (its start and the combination of its waves).  Ties keep the
// smaller ks (fewer partials to reduce).
void plan_split_rounds(int K, int N, int slots, int* ksplit, int* kchunk) {
  slots = std::max(1, slots);
  const int tiles = (N + 31) / 32;
  const int kmax = std::max(1, std::min((K + 255) / 256, 8));
  int best_ks = 1, best_kc = std::max(64, ((K + 63) / 64) * 64);
  int64_t best = -1;
  for (int ks = 1; ks <= kmax; ++ks) {
    int kc = (K + ks - 1) / ks;
    kc = std::max(64, ((kc + 63) / 64) * 64);
    const int ks2 = (K + kc - 1) / kc;
    const int64_t rounds = ((int64_t)tiles * ks2 + slots - 1) / slots;
    const int64_t cost = rounds * (kc + 320);
    if (best < 0 || cost < best) {
      best = cost;
      best_ks = ks2;
      best_kc = kc;
    }
  }
  *ksplit = best_ks;
  *kchunk = best_kc;
}

// FP64 gemm_lx: 32 output columns per workgroup; one workgroup per CU for the
// ring kernel (P <= 64), two for the general kernel.
void plan_split(int K, int N, int* ksplit, int* kchunk, int P) {
  plan_split_target(K, N, 32, P <= 64 ? 256 : 512, ksplit, kchunk);
}

hipError_t launch_gemm_lx(const GemmArgs& g, hipStream_t s) {
  if (g.N <= 0 || g.P <= 0) return hipSuccess;
  if (g.kchunk <= 0 || g.kchunk % 16 != 0) return hipErrorInvalidValue;
  const int pb = (g.P + 15) / 16;
  const bool lk1 = g.sLk == 1;
  if (g.skip_if && g.kchunk > 64) return hipErrorInvalidValue;   // only the narrow route skips
  if (g.alt_if && !(lk1 && pb <= 4 && g.kchunk > 64)) return hipErrorInvalidValue;   // ring route only
  if (lk1 && pb <= 4 && g.kchunk > 64) {
    dim3 grid((g.N + 31) / 32, g.ksplit);
    switch (pb) {
      case 1: hipLaunchKernelGGL(gemm_lx_ring_kernel<1>, grid, dim3(256), 0, s, g); break;
      case 2: hipLaunchKernelGGL(gemm_lx_ring_kernel<2>, grid, dim3(256), 0, s, g); break;
      case 3: hipLaunchKernelGGL(gemm_lx_ring_kernel<3>, grid, dim3(256), 0, s, g); break;
      default: hipLaunchKernelGGL(gemm_lx_ring_kernel<4>, grid, dim3(256), 0, s, g); break;
    }
    return hipGetLastError();
  }
  if (g.kchunk <= 64) {
    dim3 grid((g.N + 63) / 64, g.ksplit);
    switch (pb) {
      case 1: hipLaunchKernelGGL(gemm_lx_narrow_kernel<1>, grid, dim3(256), 0, s, g); break;
      case 2: hipLaunchKernelGGL(gemm_lx_narrow_kernel<2>, grid, dim3(256), 0, s, g); break;
      case 3: hipLaunchKernelGGL(gemm_lx_narrow_kernel<3>, grid, dim3(256), 0, s, g); break;
      case 4: hipLaunchKernelGGL(gemm_lx_narrow_kernel<4>, grid, dim3(256), 0, s, g); break;
      case 5: hipLaunchKernelGGL(gemm_lx_narrow_kernel<5>, grid, dim3(256), 0, s, g); break;
      case 6: hipLaunchKernelGGL(gemm_lx_narrow_kernel<6>, grid, dim3(256), 0, s, g); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  dim3 grid((g.N + (g.P <= 64 ? 63 : 31)) / (g.P <= 64 ? 64 : 32), g.ksplit);
#define RQ_LX(pb_, nb_)                                                                  \
  case pb_:                                                                              \
    if (lk1)                                                                             \
      hipLaunchKernelGGL((gemm_lx_kernel<pb_, nb_, true>), grid, dim3(256), 0, s, g);    \
    else                                                                                 \
      hipLaunchKernelGGL((gemm_lx_kernel<pb_, nb_, false>), grid, dim3(256), 0, s, g);   \
    break;
  switch (pb) {
    RQ_LX(1, 4)
    RQ_LX(2, 4)
    RQ_LX(3, 4)
    RQ_LX(4, 4)
    RQ_LX(5, 2)
    RQ_LX(6, 2)
#undef RQ_LX
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// reduce: out(p, n) = sum_s part_s(p, n) in order s = 0, 1, ...; with T the
// column is then multiplied by T^T (T upper triangular bj x bj):
// Z(i, n) = sum_{q <= i} T(q, i) W(q, n), rows bj..63 of Z set to zero.
// Split-K partials p[0], p[stride], ..., p[(ks - 1) stride] of one output:
// the first eight are requested together (a loop with a run-time trip count
// waited for each load before issuing the next); kSplitBatch values land in v.
constexpr int kSplitBatch = 8;
RQ_DEV void load_partials(const double* p, int64_t stride, int ks, bool ok,
                          double (&v)[kSplitBatch]) {
#pragma unroll
  for (int r = 0; r < kSplitBatch; ++r) v[r] = (ok && r < ks) ? p[r * stride] : 0.0;
}
// Their sum in the order s = 0, 1, ... (starting from the first partial, not
// from 0.0 + it: that add was folded into the first load's branch, with a
// wait for it before the other loads).
RQ_DEV double sum_partials(const double* p, int64_t stride, int ks, bool ok,
                           const double (&v)[kSplitBatch]) {
  double acc = v[0];
#pragma unroll
  for (int r = 1; r < kSplitBatch; ++r)
    if (r < ks) acc += v[r];
  for (int r = kSplitBatch; ok && r < ks; ++r) acc += p[r * stride];
  return acc;
}

__global__ __launch_bounds__(256) void reduce_plain_kernel(const double* part, int64_t ldp,
                                                           int64_t sstride, int ks, int P, int N,
                                                           double* out, int64_t ldout) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)P * N) return;
  const int p = (int)(e % P);
  const int64_t n = e / P;
  const double* src = part + p + n * ldp;
  double v[kSplitBatch];
  load_partials(src, sstride, ks, true, v);
  out[p + n * ldout] = sum_partials(src, sstride, ks, true, v);
}

// Four columns per workgroup, one thread per (row i, column): the split-K
// partials of a column are summed into LDS by 64 threads, then row i of
// Z = T^T W is an inner product of column i of T with that column.
__global__ __launch_bounds__(256) void reduce_t_kernel(const double* part, int64_t ldp,
                                                       int64_t sstride, int ks, int N,
                                                       double* Z, int64_t ldz, bool zero_pad,
                                                       const double* T, int64_t ldt, int bj,
                                                       bool trans) {
  __shared__ double s_T[64][65];
  __shared__ double s_w[4][64];
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int i = e % 64, q = e / 64;
    s_T[i][q] = (i < bj && q < bj && i <= q) ? T[i + (int64_t)q * ldt] : 0.0;
  }
  const int i = threadIdx.x & 63;
  const int cl = threadIdx.x >> 6;
  const int64_t n = (int64_t)blockIdx.x * 4 + cl;
  const bool ok = n < N && i < bj;
  const double* src = part + i + (ok ? n : 0) * ldp;
  double v[kSplitBatch];
  load_partials(src, sstride, ks, ok, v);
  s_w[cl][i] = sum_partials(src, sstride, ks, ok, v);
  __syncthreads();
  if (n >= N) return;
  double z = 0.0;
#pragma unroll 16
  for (int q = 0; q < 64; ++q) z += (trans ? s_T[q][i] : s_T[i][q]) * s_w[cl][q];
  if (i < bj)
    Z[i + n * ldz] = z;
  else if (zero_pad && i < ldz)
    Z[i + n * ldz] = 0.0;
}

// reduce + R12 update of one block (steps 4 and 5 of Algorithm 4 for the rows
// of R12).  A workgroup takes 16 columns (4 per wave), so that the 64 x 64
// operands are staged in LDS once for all of them.  Two forms, chosen on the
// device when `qflag` is given:
//  * from W = Y^T A (qflag null, or *qflag != 0: the column-by-column panel
//    ran): W(:, n) = sum_s part_s(:, n) in order s = 0, 1, ...; Z(:, n) =
//    T^T W(:, n); R12(:, n) -= Y11 Z(:, n), with Y11 the leading bj x bj block
//    of Y;
//  * from P = Q^T A (*qflag == 0: the Cholesky-QR panel, whose Householder
//    block has first b columns Q S and Y11 = L11): P(:, n) = sum_s part_s(:, n);
//    R12(:, n) = S P(:, n), and as R12 = A_top - Y11 Z, Z(:, n) =
//    L11^{-1} (A_top(:, n) - S P(:, n)), with A_top the rows of R12 before.
// Rows bj..63 of Z are zero.
__global__ __launch_bounds__(256) void reduce_t_r12_kernel(const double* part, int64_t sstride,
                                                           int ks, int N, double* Z,
                                                           const double* T, int64_t ldt,
                                                           const double* Y, int64_t ldy,
                                                           double* R12, int64_t ldr, int bj,
                                                           const uint32_t* qflag,
                                                           const double* linv,
                                                           const double* sgn) {
  __shared__ double s_T[64][65];   // s_T[q][i] = T(q, i), upper triangle (or L^{-1}(i, q))
  __shared__ double s_Y[64][65];   // s_Y[r][i] = Y(r, i), r, i < bj
  __shared__ double s_v[4][64][4]; // per wave: the 4 columns' vectors, row-major [q][c]
  const int i = threadIdx.x & 63;
  const int cl = threadIdx.x >> 6;
  // wave cl takes the 4 columns 16 blockIdx + 4 cl + c together, so that every
  // staged entry read from LDS feeds four products; their split-K partials
  // and R12 entries are requested first, with the staging
  const int64_t n0 = (int64_t)blockIdx.x * 16 + 4 * cl;
  double w[4], r12[4];
  double pv[4][kSplitBatch];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int64_t n = n0 + c;
    const bool ok = n < N && i < bj;
    load_partials(part + i + (ok ? n : 0) * 64, sstride, ks, ok, pv[c]);
    r12[c] = ok ? R12[i + n * ldr] : 0.0;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int64_t n = n0 + c;
    const bool ok = n < N && i < bj;
    w[c] = sum_partials(part + i + (ok ? n : 0) * 64, sstride, ks, ok, pv[c]);
  }
  // the route flag is read after the partials are requested (they do not
  // depend on it)
  const bool qr = qflag && *qflag == 0u;
  if (qr) {
    const double sg = (i < bj) ? sgn[i] : 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double rn = sg * w[c];    // R12 = S P
      w[c] = r12[c] - rn;             // A_top - S P, the operand of L^{-1}
      r12[c] = rn;
    }
  }
#pragma unroll
  for (int e0 = 0; e0 < 64 * 64; e0 += 256) {
    const int e = e0 + threadIdx.x;
    const int a = e % 64, b = e / 64;
    const bool in = a < bj && b < bj && a <= b;
    s_T[a][b] = in ? (qr ? linv[b * 64 + a] : T[a + (int64_t)b * ldt]) : 0.0;
    if (!qr) s_Y[a][b] = (a < bj && b < bj) ? Y[a + (int64_t)b * ldy] : 0.0;
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) s_v[cl][i][c] = w[c];
  __syncthreads();
  // Z(:, n) = T^T W(:, n), or L^{-1} (A_top - S P)(:, n)
  double z[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
  for (int q = 0; q < 64; ++q) {
    const double tq = s_T[q][i];
#pragma unroll
    for (int c = 0; c < 4; ++c) z[c] += tq * s_v[cl][q][c];
  }
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    z[c] = (i < bj) ? z[c] : 0.0;
    if (n0 + c < N) Z[i + (n0 + c) * 64] = z[c];
  }
  if (qr) {
#pragma unroll
    for (int c = 0; c < 4; ++c)
      if (n0 + c < N && i < bj) R12[i + (n0 + c) * ldr] = r12[c];
    return;
  }
  // the wave's own LDS accesses complete in order
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
  for (int c = 0; c < 4; ++c) s_v[cl][i][c] = z[c];
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // R12(:, n) -= Y11 Z(:, n)
  double u[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
  for (int q = 0; q < 64; ++q) {
    const double yq = s_Y[i][q];
#pragma unroll
    for (int c = 0; c < 4; ++c) u[c] += yq * s_v[cl][q][c];
  }
#pragma unroll
  for (int c = 0; c < 4; ++c)
    if (n0 + c < N && i < bj) R12[i + (n0 + c) * ldr] = r12[c] - u[c];
}

hipError_t launch_reduce_r12(const double* part, int64_t sstride, int ks, int N, double* Z,
                             const double* T, int64_t ldt, const double* Y, int64_t ldy,
                             double* R12, int64_t ldr, int bj, hipStream_t s,
                             const uint32_t* qflag, const double* linv, const double* sgn) {
  if (N <= 0) return hipSuccess;
  if (bj < 1 || bj > 64) return hipErrorInvalidValue;
  if (qflag && (!linv || !sgn)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(reduce_t_r12_kernel, dim3((N + 15) / 16), dim3(256), 0, s, part, sstride, ks,
                     N, Z, T, ldt, Y, ldy, R12, ldr, bj, qflag, linv, sgn);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* part, int64_t ldp, int64_t sstride, int ks, int P, int N,
                         double* out, int64_t ldout, const double* T, int64_t ldt, int bj,
                         hipStream_t s) {
  if (N <= 0) return hipSuccess;
  if (T) {
    hipLaunchKernelGGL(reduce_t_kernel, dim3((N + 3) / 4), dim3(256), 0, s, part, ldp, sstride,
                       ks, N, out, (int64_t)64, true, T, ldt, bj, true);
  } else {
    const int64_t total = (int64_t)P * N;
    hipLaunchKernelGGL(reduce_plain_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                       s, part, ldp, sstride, ks, P, N, out, ldout);
  }
  return hipGetLastError();
}

hipError_t launch_reduce_t(const double* part, int64_t ldp, int64_t sstride, int ks, int N,
                           double* Z, int64_t ldz, bool zero_pad, const double* T, int64_t ldt,
                           int bj, bool trans, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_t_kernel, dim3((N + 3) / 4), dim3(256), 0, s, part, ldp, sstride, ks,
                     N, Z, ldz, zero_pad, T, ldt, bj, trans);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// update: C(M x N) -= Y(M x K) Z(K x N).  Each workgroup owns a 64 x 64 tile of
// C; wave (wr, wc) owns 32 x 32 as 2 x 2 MFMA blocks computed as blocks of
// C^T, so that for a fixed accumulator element the 16 lanes of a row touch 16
// consecutive rows of one column of C (coalesced loads and stores).
__global__ __launch_bounds__(256) void update_kernel(double* C, int64_t ldc, int M, int N,
                                                     const double* Y, int64_t ldy,
                                                     const double* Z, int64_t ldz, int K,
                                                     double alpha, double beta) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int rb = blockIdx.x * 64 + (wave & 1) * 32;
  const int cb = blockIdx.y * 64 + (wave >> 1) * 32;
  const int l16 = lane & 15;
  const int kq = lane >> 4;
  dx4 acc[2][2];
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
      const int r = rb + 16 * ib + l16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int cc = cb + 16 * jb + kq + 4 * v;
        acc[ib][jb][v] = (beta != 0.0 && r < M && cc < N) ? beta * C[r + (int64_t)cc * ldc] : 0.0;
      }
    }
  for (int k0 = 0; k0 < K; k0 += 16) {
    double za[2][4], yb[2][4];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int k = k0 + 4 * kq + s;
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) {
        const int cc = cb + 16 * jb + l16;
        za[jb][s] = (cc < N && k < K) ? alpha * Z[k + (int64_t)cc * ldz] : 0.0;
      }
#pragma unroll
      for (int ib = 0; ib < 2; ++ib) {
        const int r = rb + 16 * ib + l16;
        yb[ib][s] = (r < M && k < K) ? Y[r + (int64_t)k * ldy] : 0.0;
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int ib = 0; ib < 2; ++ib)
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) acc[ib][jb] = mfma_f64(za[jb][s], yb[ib][s], acc[ib][jb]);
  }
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
      const int r = rb + 16 * ib + l16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int cc = cb + 16 * jb + kq + 4 * v;
        if (r < M && cc < N) C[r + (int64_t)cc * ldc] = acc[ib][jb][v];
      }
    }
}

// ---- C(M x N) = Y(M x K) Z(K x N) for tall Y and N <= 256 (Z1 = A V of TUXV) --
// One pass over Y: a workgroup owns 64 rows of C and 64 NBW columns (all of N
// when N <= 256).  Z is staged once, step-major: element (k, c) at
// ((k / 4) ncp + c) 4 + k % 4, so a wave's Z operands of one 4-k step are 64
// consecutive doubles; Y operands come straight from Y (16 consecutive rows per
// 4 lanes).  Wave w owns columns 16 NBW w ..; the operands of the next two steps
// are in flight (a ring of three register sets).  Rows at or past M are clamped
// to row M - 1 and not stored; Z is zero past K and N.  C = alpha Y Z + beta C.
constexpr int kNf64Rows = 64;

static int nf64_nbw(int N) { return N > 192 ? 4 : N > 128 ? 3 : N > 64 ? 2 : 1; }
static int nf64_ncp(int N) {
  const int cols = 64 * nf64_nbw(N);
  return ((N + cols - 1) / cols) * cols;
}
int64_t gemm_nn_tall_stage_doubles(int N, int K) {
  return (int64_t)nf64_ncp(N) * (((K + 3) / 4) * 4);
}

__global__ void stage_z_f64_kernel(const double* Z, int64_t ldz, int N, int K, int ncp, int64_t total,
                                   double* zt) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int kk = (int)(e & 3);
  const int64_t sc = e >> 2;
  const int c = (int)(sc % ncp);
  const int k = (int)(sc / ncp) * 4 + kk;
  zt[e] = (c < N && k < K) ? Z[k + (int64_t)c * ldz] : 0.0;
}

template <int NBW>
__global__ __launch_bounds__(256, 2) void gemm_nn_tall_kernel(double* C, int64_t ldc, int M, int N,
                                                              const double* Y, int64_t ldy,
                                                              const double* zt, int ncp, int K,
                                                              double alpha, double beta) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int l16 = lane & 15, kq = lane >> 4;
  const int r0 = blockIdx.x * kNf64Rows;
  const int cw = blockIdx.y * 64 * NBW + 16 * NBW * wave;
  const double* yp[4];
#pragma unroll
  for (int ib = 0; ib < 4; ++ib) yp[ib] = Y + min(r0 + 16 * ib + l16, M - 1) + (int64_t)kq * ldy;
  const double* zp = zt + (int64_t)(cw + l16) * 4 + kq;
  dx4 acc[4][NBW];
#pragma unroll
  for (int ib = 0; ib < 4; ++ib)
#pragma unroll
    for (int jb = 0; jb < NBW; ++jb) acc[ib][jb] = dx4{0.0, 0.0, 0.0, 0.0};
  struct Ops {
    double y[4], z[NBW];
  };
  auto load = [&](int st, Ops& o) {
    const int64_t yo = (int64_t)(4 * st) * ldy;
#pragma unroll
    for (int ib = 0; ib < 4; ++ib) o.y[ib] = yp[ib][yo];
#pragma unroll
    for (int jb = 0; jb < NBW; ++jb) o.z[jb] = zp[((int64_t)st * ncp + 16 * jb) * 4];
  };
  auto compute = [&](const Ops& o) {
#pragma unroll
    for (int ib = 0; ib < 4; ++ib)
#pragma unroll
      for (int jb = 0; jb < NBW; ++jb) acc[ib][jb] = mfma_f64(o.y[ib], o.z[jb], acc[ib][jb]);
  };
  const int nfull = K / 4;
  {
    Ops A, B, Cr;
    if (nfull > 0) load(0, A);
    if (nfull > 1) load(1, B);
    for (int i = 0; i < nfull; i += 3) {
      if (i + 2 < nfull) load(i + 2, Cr);
      compute(A);
      if (i + 1 >= nfull) break;
      if (i + 3 < nfull) load(i + 3, A);
      compute(B);
      if (i + 2 >= nfull) break;
      if (i + 4 < nfull) load(i + 4, B);
      compute(Cr);
    }
  }
  if (4 * nfull < K) {                            // a final partial step
    Ops o;
    const bool kok = 4 * nfull + kq < K;
#pragma unroll
    for (int ib = 0; ib < 4; ++ib) o.y[ib] = kok ? yp[ib][(int64_t)(4 * nfull) * ldy] : 0.0;
#pragma unroll
    for (int jb = 0; jb < NBW; ++jb) o.z[jb] = zp[((int64_t)nfull * ncp + 16 * jb) * 4];
    compute(o);
  }
  // lane holds C(r0 + 16 ib + kq + 4 v, cw + 16 jb + l16)
#pragma unroll
  for (int ib = 0; ib < 4; ++ib)
#pragma unroll
    for (int jb = 0; jb < NBW; ++jb) {
      const int c = cw + 16 * jb + l16;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + 16 * ib + kq + 4 * v;
        if (r < M && c < N) {
          double* cp = C + r + (int64_t)c * ldc;
          *cp = (beta != 0.0) ? alpha * acc[ib][jb][v] + beta * *cp : alpha * acc[ib][jb][v];
        }
      }
    }
}

hipError_t launch_gemm_nn_tall(double* C, int64_t ldc, int M, int N, const double* Y, int64_t ldy,
                               const double* Z, int64_t ldz, int K, double alpha, double beta,
                               double* zstage, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (ldy < M || ldc < M || (K > 0 && !zstage)) return hipErrorInvalidValue;
  const int nbw = nf64_nbw(N), ncp = nf64_ncp(N);
  const int64_t total = gemm_nn_tall_stage_doubles(N, K);
  if (total > 0) {
    hipLaunchKernelGGL(stage_z_f64_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       Z, ldz, N, K, ncp, total, zstage);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  dim3 grid((M + kNf64Rows - 1) / kNf64Rows, ncp / (64 * nbw));
  switch (nbw) {
    case 1: hipLaunchKernelGGL(gemm_nn_tall_kernel<1>, grid, dim3(256), 0, s, C, ldc, M, N, Y, ldy, zstage, ncp, K, alpha, beta); break;
    case 2: hipLaunchKernelGGL(gemm_nn_tall_kernel<2>, grid, dim3(256), 0, s, C, ldc, M, N, Y, ldy, zstage, ncp, K, alpha, beta); break;
    case 3: hipLaunchKernelGGL(gemm_nn_tall_kernel<3>, grid, dim3(256), 0, s, C, ldc, M, N, Y, ldy, zstage, ncp, K, alpha, beta); break;
    default: hipLaunchKernelGGL(gemm_nn_tall_kernel<4>, grid, dim3(256), 0, s, C, ldc, M, N, Y, ldy, zstage, ncp, K, alpha, beta); break;
  }
  return hipGetLastError();
}

hipError_t launch_gemm_nn(double* C, int64_t ldc, int M, int N, const double* Y, int64_t ldy,
                          const double* Z, int64_t ldz, int K, double alpha, double beta,
                          hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 grid((M + 63) / 64, (N + 63) / 64);
  hipLaunchKernelGGL(update_kernel, grid, dim3(256), 0, s, C, ldc, M, N, Y, ldy, Z, ldz, K, alpha,
                     beta);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Trailing update of tall blocks, C(M x N) -= Y(M x K) Z(K x N) with K <= 64
// (the rank-b update of Algorithm 4).  A 1024-thread workgroup owns 256 rows
// (wave w: 16 rows, whose Y operands it keeps in registers for the whole
// launch) and walks the 64-column blocks cg, cg + G, cg + 2G, ...: each block's
// Z (64 x 64, negated) is staged once in LDS for all 16 waves, double-buffered,
// and the next block's C and Z are fetched while the current one is on the
// matrix cores.  C is read and written exactly once.  Each workgroup fills one
// compute unit, so the grid (row groups x G) is sized to the units the launch
// may take.
constexpr int kStripRows = 256;
constexpr int kZld = 72;   // LDS row stride of a staged Z block [k][col] (2-way banked reads)

__global__ __launch_bounds__(1024) void update_strip_kernel(double* C, int64_t ldc, int M, int N,
                                                            const double* Y, int64_t ldy,
                                                            const double* Z, int64_t ldz, int K,
                                                            int G) {
  __shared__ double sZ[2][64 * kZld];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  const int rg = blockIdx.x / G, cg = blockIdx.x - rg * G;
  const int row = rg * kStripRows + wave * 16 + l16;
  const bool rok = row < M;
  const int nblk = (N + 63) / 64;
  if (cg >= nblk) return;                       // the whole workgroup
  // B operands of the 16 k-steps: Y(row, 4 s + kq)
  double yv[16];
#pragma unroll
  for (int s = 0; s < 16; ++s) {
    const int k = 4 * s + kq;
    yv[s] = (rok && k < K) ? Y[row + (int64_t)k * ldy] : 0.0;
  }
  // thread t stages Z rows zk..zk+3 of the block's column zc
  const int zc = t >> 4, zk = (t & 15) * 4;
  double zs[4];
  auto fetch_z = [&](int cb) {
    const int col = cb * 64 + zc;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      zs[i] = (col < N && zk + i < K) ? Z[(zk + i) + (int64_t)col * ldz] : 0.0;
  };
  auto put_z = [&](int b) {
#pragma unroll
    for (int i = 0; i < 4; ++i) sZ[b][(zk + i) * kZld + zc] = -zs[i];
  };
  // accumulator layout of the 16 x 16 blocks jb: lane holds column
  // 16 jb + kq + 4 i of the block, row `row`
  auto fetch_c = [&](int cb, dx4(&v)[4]) {
    const double* cp = C + row + (int64_t)(cb * 64 + kq) * ldc;
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int col = cb * 64 + 16 * jb + kq + 4 * i;
        v[jb][i] = (rok && col < N) ? cp[(int64_t)(16 * jb + 4 * i) * ldc] : 0.0;
      }
  };
  auto compute_store = [&](int cb, int b, dx4(&acc)[4]) {
    const double* zb = sZ[b];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int k = 4 * s + kq;
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) acc[jb] = mfma_f64(zb[k * kZld + 16 * jb + l16], yv[s], acc[jb]);
    }
    double* cp = C + row + (int64_t)(cb * 64 + kq) * ldc;
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int col = cb * 64 + 16 * jb + kq + 4 * i;
        if (rok && col < N) cp[(int64_t)(16 * jb + 4 * i) * ldc] = acc[jb][i];
      }
  };
  // two named accumulator sets alternate (the walk is unrolled by two), so the
  // prefetched block never has to be copied
  dx4 accA[4], accB[4];
  int cb = cg;
  fetch_z(cb);
  fetch_c(cb, accA);
  put_z(0);
  __syncthreads();
  while (true) {
    int cn = cb + G;
    if (cn < nblk) {
      fetch_z(cn);
      fetch_c(cn, accB);
    }
    compute_store(cb, 0, accA);
    if (cn >= nblk) break;
    put_z(1);
    __syncthreads();   // buffer 1 complete; every wave is done with buffer 0
    cb = cn;
    cn = cb + G;
    if (cn < nblk) {
      fetch_z(cn);
      fetch_c(cn, accA);
    }
    compute_store(cb, 1, accB);
    if (cn >= nblk) break;
    put_z(0);
    __syncthreads();
    cb = cn;
  }
}

hipError_t launch_update(double* C, int64_t ldc, int M, int N, const double* Y, int64_t ldy,
                         const double* Z, int64_t ldz, int bj, int max_wgs, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (bj < 1 || bj > 64) return hipErrorInvalidValue;
  if (M < kStripRows || max_wgs < 1)
    return launch_gemm_nn(C, ldc, M, N, Y, ldy, Z, ldz, bj, -1.0, 1.0, s);
  const int nrg = (M + kStripRows - 1) / kStripRows, nblk = (N + 63) / 64;
  const int G = std::max(1, std::min(nblk, max_wgs / nrg));
  hipLaunchKernelGGL(update_strip_kernel, dim3(nrg * G), dim3(1024), 0, s, C, ldc, M, N, Y, ldy, Z,
                     ldz, bj, G);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fresh sample of the updated trailing matrix for one tile of kFreshCols
// columns (64 threads): B(:, c) = Omega(:, 0:M2) (C(:, c) - Y Z(:, c)).
RQ_DEV void fresh_sample_tile(const RankCheck& rk, int tile) {
  __shared__ double s_z[64][kFreshCols];
  __shared__ double s_u[kFreshRows][kFreshCols + 1];
  __shared__ double s_om[kFreshRows][kFreshMaxEll + 1];
  const int t = threadIdx.x;
  const int c0 = tile * kFreshCols;
#pragma unroll
  for (int q = 0; q < kFreshCols; ++q) {
    const int c = c0 + q;
    s_z[t][q] = (t < rk.bj && c < rk.N) ? rk.Z[t + (int64_t)c * rk.ldz] : 0.0;
  }
  const int cc = t & (kFreshCols - 1), rg = t / kFreshCols;   // accumulation: column, row phase
  const int rr = t & (kFreshRows - 1), hf = t / kFreshRows;   // staging: chunk row, half
  constexpr int kAcc = kFreshMaxEll / 4;
  double acc[kAcc];
#pragma unroll
  for (int q = 0; q < kAcc; ++q) acc[q] = 0.0;
  for (int r0 = 0; r0 < rk.M2; r0 += kFreshRows) {
    __syncthreads();   // s_z is staged and the previous chunk consumed
    const int r = r0 + rr;
    const bool rok = r < rk.M2;
    double u[kFreshCols / 2];
#pragma unroll
    for (int q = 0; q < kFreshCols / 2; ++q) {
      const int c = c0 + hf * (kFreshCols / 2) + q;
      u[q] = (rok && c < rk.N) ? rk.C[r + (int64_t)c * rk.ldc] : 0.0;
    }
    for (int j = 0; j < rk.bj; ++j) {
      const double y = rok ? rk.Y[r + (int64_t)j * rk.ldy] : 0.0;
#pragma unroll
      for (int q = 0; q < kFreshCols / 2; ++q) u[q] = fma(-y, s_z[j][hf * (kFreshCols / 2) + q], u[q]);
    }
#pragma unroll
    for (int q = 0; q < kFreshCols / 2; ++q) s_u[rr][hf * (kFreshCols / 2) + q] = u[q];
#pragma unroll
    for (int q = 0; q < kFreshMaxEll / 2; ++q) {
      const int e = hf + 2 * q;
      if (e < rk.ell) s_om[rr][e] = rok ? rk.Om[e + (int64_t)r * rk.ldo] : 0.0;
    }
    __syncthreads();
    for (int x = 0; x < kFreshRows; ++x) {
      const double uv = s_u[x][cc];
#pragma unroll
      for (int q = 0; q < kAcc; ++q) acc[q] = fma(s_om[x][rg + 4 * q], uv, acc[q]);
    }
  }
  const int c = c0 + cc;
  if (c < rk.N) {
#pragma unroll
    for (int q = 0; q < kAcc; ++q) {
      const int e = rg + 4 * q;
      if (e < rk.ell) rk.B[e + (int64_t)c * rk.ldb] = acc[q];
    }
  }
}

// ---------------------------------------------------------------------------
// omega11: Mhat = S11 R11^{-1} (both bj x bj upper triangular, so Mhat is too),
// M[i + c ldm] = Mhat(i, c).  One single-wave workgroup per row
// i (rows on different compute units); lane c holds column c of R11 in
// registers and the reciprocal of R11(c, c).  Step c: m_c = s_c / R(c, c), then
// s_c' -= m_c R(c, c') for c' > c, with s_c and 1 / R(c, c) read from lane c by
// v_readlane.
//
// With a rank check (rk.info set), eq. (update1) is used only while R11 is
// numerically nonsingular (Section 3.2 needs R11^{-1}): every workgroup tests
// |R11(c, c)| <= rk.thresh |R_00| itself, so all take the same decision without
// waiting for each other.  The first time the test fires, workgroup 0 records
// the 1-based column in *rk.info; from then on (*rk.info != 0) the rows of
// Mhat are not formed, the sample update product that follows skips itself,
// and the extra workgroups bj.. of the launch write a fresh sample of the
// updated trailing matrix instead (repeated sampling, Section 3.4):
//   B = Omega(:, 0:M2) (C - Y Z),  C = the M2 x N rows below R12 before their
// update, Y (M2 x bj) and Z = T^T W (bj x N) the block's reflection, so
// C - Y Z is the trailing matrix A^[J] the next block factors.  Each extra
// workgroup owns 16 columns of B: per chunk of 64 rows, thread t forms row t
// of C - Y Z for those columns into LDS and stages column t of the Omega chunk,
// then each thread accumulates ell / 4 rows of its column of B.
//
// Workgroups past those (nprep of them) set the next block's record areas to
// the sentinel, which saves the launch of exchange_prep2 before its sample QRCP.
__global__ __launch_bounds__(64) void omega11_kernel(const double* S11, int64_t lds,
                                                     const double* R11, int64_t ldr, int bj,
                                                     double* M, int64_t ldm, RankCheck rk,
                                                     RecordPrep rp, int nprep) {
  const int lane = threadIdx.x;
  const int i = blockIdx.x;
  const int first_prep = (int)gridDim.x - nprep;
  if (i >= first_prep) {
    const int p = i - first_prep;
    if (p == 0 && lane < 3) rp.sync[lane] = 0u;
    unsigned long long* const r1 = reinterpret_cast<unsigned long long*>(rp.rec1);
    unsigned long long* const r2 = reinterpret_cast<unsigned long long*>(rp.rec2);
    for (int64_t e = (int64_t)p * 64 + lane; e < rp.n1 + rp.n2; e += (int64_t)nprep * 64) {
      if (e < rp.n1)
        r1[e] = kUnpublished;
      else
        r2[e - rp.n1] = kUnpublished;
    }
    return;
  }
  // every load that does not depend on the rank check goes out first: R11's
  // column of this lane (its diagonal entry among them), S11's entry and R_00
  // (rows i >= bj, the fresh-sample tiles, skip the ones they never use)
  const bool row = i < bj;
  double rc[64];
#pragma unroll
  for (int q = 0; q < 64; ++q)
    rc[q] = (row && lane < bj && q <= lane) ? R11[q + (int64_t)lane * ldr] : 0.0;
  double sv = (row && lane < bj && lane >= i) ? S11[i + (int64_t)lane * lds] : 0.0;
  const double diag = (lane < bj) ? R11[lane + (int64_t)lane * ldr] : 0.0;
  if (rk.info) {
    bool resample = __hip_atomic_load(rk.info, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    const double r00 = *rk.r00;
    if (!resample) {
      const double lim = rk.thresh * fabs(r00);
      const bool small = lane < bj && fabs(diag) <= lim;
      const unsigned long long hit = __builtin_amdgcn_ballot_w64(small);
      if (hit) {
        resample = true;
        if (i == 0 && lane == 0)
          __hip_atomic_store(rk.info, rk.col0 + (int64_t)__builtin_ctzll(hit) + 1, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    if (!row) {
      if (resample) fresh_sample_tile(rk, i - bj);
      return;
    }
    if (resample) return;
  }
  const double rinv = (lane < bj) ? 1.0 / diag : 0.0;
  double mine = 0.0;
#pragma unroll
  for (int c = 0; c < 64; ++c) {
    if (c < bj) {
      const double mc = readlane_f64(sv, c) * readlane_f64(rinv, c);
      if (lane == c) mine = mc;
      if (lane > c) sv = fma(-mc, rc[c], sv);   // rc[c] = R11(c, lane)
    }
  }
  if (lane < bj) M[i + (int64_t)lane * ldm] = mine;
}

hipError_t launch_omega11(const double* S11, int64_t lds, const double* R11, int64_t ldr, int bj,
                          double* M, int64_t ldm, const RankCheck* rk, const RecordPrep* prep,
                          hipStream_t s) {
  if (bj < 1 || bj > 64) return hipErrorInvalidValue;
  RankCheck r{};
  int extra = 0;
  if (rk) {
    r = *rk;
    if (!r.info || !r.r00 || r.ell < 1 || r.ell > kFreshMaxEll || r.N < 0 || r.M2 < 0)
      return hipErrorInvalidValue;
    extra = (r.N + kFreshCols - 1) / kFreshCols;
  }
  RecordPrep rp{};
  int nprep = 0;
  if (prep) {
    rp = *prep;
    if (!rp.sync || rp.n1 < 0 || rp.n2 < 0 || (rp.n1 > 0 && !rp.rec1) || (rp.n2 > 0 && !rp.rec2))
      return hipErrorInvalidValue;
    // about 32 words per thread, at least one workgroup (it clears the flags)
    nprep = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (rp.n1 + rp.n2 + 2047) / 2048));
  }
  hipLaunchKernelGGL(omega11_kernel, dim3(bj + extra + nprep), dim3(64), 0, s, S11, lds, R11, ldr,
                     bj, M, ldm, r, rp, nprep);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// permute: new X(:, q) = X(:, src_top[q]) for q < bj and
// new X(:, dst_low[o]) = X(:, o) for o < bj with dst_low[o] >= 0 (positions
// relative to the block start).  Each thread owns one row of a 64-row slab and
// reads every moved value of that row into registers (all loads in flight at
// once), then, after the workgroup's barrier, writes them: the only reads a
// write could clobber are those of the same slab, and slabs are disjoint.
//
// The block has ncols columns.  A sample QRCP that stopped early (non-finite
// norms, an expired wait: both leave a status bit) does not write the maps, so
// entries are checked here: a source outside 0..ncols-1 leaves its column in
// place and a destination outside bj..ncols-1 moves nothing.  Every access
// stays inside the block whatever the maps hold.
__global__ __launch_bounds__(256) void permute_kernel(double* X, int64_t ldx, int rows, int bj,
                                                      int ncols, const int* src_top,
                                                      const int* dst_low, int64_t* jpvt) {
  __shared__ int s_src[64], s_dst[64];
  const int t = threadIdx.x;
  if (t < 64) {
    int sv = -1, dv = -1;
    if (t < bj) {
      sv = src_top[t];
      dv = dst_low[t];
      if (sv < 0 || sv >= ncols) sv = t;
      if (dv < bj || dv >= ncols) dv = -1;
    }
    s_src[t] = sv;
    s_dst[t] = dv;
  }
  __syncthreads();
  const int r = blockIdx.x * 64 + (t & 63);
  const bool rok = r < rows;
  double top[16], low[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int q = (t >> 6) + 4 * i;
    const bool qok = rok && q < bj;
    top[i] = qok ? X[r + (int64_t)s_src[q] * ldx] : 0.0;
    low[i] = (qok && s_dst[q] >= 0) ? X[r + (int64_t)q * ldx] : 0.0;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int q = (t >> 6) + 4 * i;
    if (rok && q < bj) {
      X[r + (int64_t)q * ldx] = top[i];
      if (s_dst[q] >= 0) X[r + (int64_t)s_dst[q] * ldx] = low[i];
    }
  }
  if (jpvt && blockIdx.x == 0) {
    __shared__ int64_t s_jt[64], s_jl[64];
    if (t < bj) {
      s_jt[t] = jpvt[s_src[t]];
      s_jl[t] = jpvt[t];
    }
    __syncthreads();
    if (t < bj) {
      jpvt[t] = s_jt[t];
      if (s_dst[t] >= 0) jpvt[s_dst[t]] = s_jl[t];
    }
  }
}

hipError_t launch_permute(double* X, int64_t ldx, int rows, int bj, int64_t ncols,
                          const int* src_top, const int* dst_low, int64_t* jpvt, hipStream_t s) {
  if (bj < 0 || bj > 64 || ncols < bj || ncols > INT_MAX) return hipErrorInvalidValue;
  const int blocks = rows > 0 ? (rows + 63) / 64 : 1;
  hipLaunchKernelGGL(permute_kernel, dim3(blocks), dim3(256), 0, s, X, ldx, rows, bj, (int)ncols,
                     src_top, dst_low, jpvt);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ void iota_kernel(int64_t* v, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) v[i] = i;
}
hipError_t launch_iota(int64_t* v, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(iota_kernel, dim3((n + 255) / 256), dim3(256), 0, s, v, n);
  return hipGetLastError();
}

__global__ void cast_f32_f64_kernel(const float* src, double* dst, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = (double)src[i];
}
hipError_t launch_cast_f32_f64(const float* src, double* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(cast_f32_f64_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src,
                     dst, n);
  return hipGetLastError();
}

__global__ void set_i64_kernel(int64_t* p, int64_t v) {
  if (threadIdx.x == 0) *p = v;
}
hipError_t launch_set_i64(int64_t* p, int64_t v, hipStream_t s) {
  hipLaunchKernelGGL(set_i64_kernel, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

__global__ void exchange_prep_kernel(uint32_t* sync, unsigned long long* rec, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < 3) sync[e] = 0u;
  if (e < n) rec[e] = kUnpublished;
}
hipError_t launch_exchange_prep(uint32_t* sync, double* rec, int64_t n, hipStream_t s) {
  const int64_t total = n > 3 ? n : 3;
  hipLaunchKernelGGL(exchange_prep_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                     sync, reinterpret_cast<unsigned long long*>(rec), n);
  return hipGetLastError();
}

// The same for two record areas in one launch (words [0, n1) of rec1, then
// [0, n2) of rec2).
__global__ void exchange_prep2_kernel(uint32_t* sync, unsigned long long* rec1, int64_t n1,
                                      unsigned long long* rec2, int64_t n2) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e < 3) sync[e] = 0u;
  if (e < n1)
    rec1[e] = kUnpublished;
  else if (e - n1 < n2)
    rec2[e - n1] = kUnpublished;
}
hipError_t launch_exchange_prep2(uint32_t* sync, double* rec1, int64_t n1, double* rec2,
                                 int64_t n2, hipStream_t s) {
  const int64_t total = std::max<int64_t>(n1 + n2, 3);
  hipLaunchKernelGGL(exchange_prep2_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                     s, sync, reinterpret_cast<unsigned long long*>(rec1), n1,
                     reinterpret_cast<unsigned long long*>(rec2), n2);
  return hipGetLastError();
}

__global__ void copy2d_kernel(const double* src, int64_t lds, double* dst, int64_t ldd, int rows,
                              int cols) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)rows * cols) return;
  const int r = (int)(e % rows);
  const int64_t c = e / rows;
  dst[r + c * ldd] = src[r + c * lds];
}
hipError_t launch_copy2d(const double* src, int64_t lds, double* dst, int64_t ldd, int rows,
                         int cols, hipStream_t s) {
  const int64_t total = (int64_t)rows * cols;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy2d_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, src,
                     lds, dst, ldd, rows, cols);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
template <class TS>
__global__ void gather_cols_kernel(const TS* src, int64_t lds, int r0, const int64_t* col,
                                   double* dst, int64_t ldd, int rows, int cols) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  if (r >= rows || c >= cols) return;
  dst[r + (int64_t)c * ldd] = (double)src[(r0 + r) + col[c] * lds];
}
hipError_t launch_gather_cols(const void* src, bool src_f32, int64_t lds, int r0, const int64_t* col,
                              double* dst, int64_t ldd, int rows, int cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  dim3 grid((rows + 255) / 256, cols);
  if (src_f32)
    hipLaunchKernelGGL(gather_cols_kernel<float>, grid, dim3(256), 0, s,
                       static_cast<const float*>(src), lds, r0, col, dst, ldd, rows, cols);
  else
    hipLaunchKernelGGL(gather_cols_kernel<double>, grid, dim3(256), 0, s,
                       static_cast<const double*>(src), lds, r0, col, dst, ldd, rows, cols);
  return hipGetLastError();
}

__global__ void fill_kernel(double* X, int64_t ldx, int rows, int cols, double value,
                            bool unit_diag) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)rows * cols) return;
  const int r = (int)(e % rows);
  const int64_t c = e / rows;
  X[r + c * ldx] = (unit_diag && r == c) ? 1.0 : value;
}
hipError_t launch_fill(double* X, int64_t ldx, int rows, int cols, double value, bool unit_diag,
                       hipStream_t s) {
  const int64_t total = (int64_t)rows * cols;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, X, ldx,
                     rows, cols, value, unit_diag);
  return hipGetLastError();
}

__global__ void explicit_y_kernel(const double* A, int64_t lda, int M, int bj, double* Y,
                                  int64_t ldy) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  if (r >= M) return;
  Y[r + (int64_t)c * ldy] = (c >= bj) ? 0.0 : (r < c ? 0.0 : (r == c ? 1.0 : A[r + (int64_t)c * lda]));
}
hipError_t launch_explicit_y(const double* A, int64_t lda, int M, int bj, double* Y, int64_t ldy,
                             hipStream_t s) {
  if (M <= 0) return hipSuccess;
  hipLaunchKernelGGL(explicit_y_kernel, dim3((M + 255) / 256, 64), dim3(256), 0, s, A, lda, M, bj,
                     Y, ldy);
  return hipGetLastError();
}

__global__ void copy_upper_kernel(const double* A, int64_t lda, int rows, int cols, double* R,
                                  int64_t ldr) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  if (r >= rows || c >= cols) return;
  R[r + (int64_t)c * ldr] = (r <= c) ? A[r + (int64_t)c * lda] : 0.0;
}
hipError_t launch_copy_upper(const double* A, int64_t lda, int rows, int cols, double* R,
                             int64_t ldr, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_upper_kernel, dim3((rows + 255) / 256, cols), dim3(256), 0, s, A, lda,
                     rows, cols, R, ldr);
  return hipGetLastError();
}

// X1(i, c) = sum_{q <= c} G(q, i) T2(q, c)   (i < c0, c < bj)
__global__ void tcomp1_kernel(const double* G, const double* T2, int64_t ldt2, int c0, int bj,
                              double* X1) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= c0 || c >= bj) return;
  double acc = 0.0;
  for (int q = 0; q <= c; ++q) acc += G[q + (int64_t)i * 64] * T2[q + (int64_t)c * ldt2];
  X1[i + (int64_t)c * c0] = acc;
}
// T12 = -T11 X1 with X1 = G^T T2 (c0 x bj): T11 is upper triangular with exact
// zeros below the diagonal, so the product runs as a plain matrix product on
// the matrix cores, straight into T(0:c0, c0:c0+bj).
hipError_t launch_tcompose(double* T, int64_t ldt, int c0, int bj, const double* G,
                           const double* T2, int64_t ldt2, double* X1, hipStream_t s) {
  if (c0 <= 0 || bj <= 0) return hipSuccess;
  dim3 grid((c0 + 255) / 256, bj);
  hipLaunchKernelGGL(tcomp1_kernel, grid, dim3(256), 0, s, G, T2, ldt2, c0, bj, X1);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_gemm_nn(T + (int64_t)c0 * ldt, ldt, c0, bj, T, ldt, X1, c0, c0, -1.0, 0.0, s);
}

__global__ void scatter_t_kernel(const double* R, int64_t ldr, int k, int n, const int64_t* col,
                                 double* Z0T, int64_t ldz) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= k || c >= n) return;
  Z0T[col[c] + (int64_t)i * ldz] = R[i + (int64_t)c * ldr];
}
hipError_t launch_scatter_t(const double* R, int64_t ldr, int k, int n, const int64_t* col,
                            double* Z0T, int64_t ldz, hipStream_t s) {
  if (k <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scatter_t_kernel, dim3((k + 255) / 256, n), dim3(256), 0, s, R, ldr, k, n, col,
                     Z0T, ldz);
  return hipGetLastError();
}

}  // namespace rq
