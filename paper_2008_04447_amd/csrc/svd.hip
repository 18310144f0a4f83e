// Singular values of a small square matrix on the device: the SVD of TUXV's
// k x k connection matrix X (Algorithm 6, Section 4.2), whose singular values
// estimate the leading singular values of A more closely than the diagonal of
// X does.
//
// Two kernels:
//   * bidiag_kernel: Householder bidiagonalization W = U^T B V with B upper
//     bidiagonal (diagonal d, superdiagonal e), in one workgroup of 16 waves.
//     Step i forms the left reflector of column i (rows i..), applies it to the
//     columns on its right (each wave owns whole columns, so its inner products
//     are wave sums), then the right reflector of row i (columns i+1..) and its
//     application to the rows below (row sums over the columns: per-wave
//     partials combined in LDS).  W lives in the workspace (k^2 doubles, held
//     in the caller's L2); d and e go to the workspace too.  Backward stable:
//     the singular values of B are those of X + dX with ||dX|| = O(k eps ||X||),
//     the same bound as LAPACK's bidiagonalization.
//   * bidiag_sv_kernel: the singular values of B as the nonnegative eigenvalues
//     of the 2k x 2k Golub-Kahan tridiagonal with zero diagonal and
//     off-diagonal (d0, e0, d1, e1, ..., d_{k-1}), found by bisection with
//     Sturm counts, which resolves every singular value of a bidiagonal matrix
//     to high relative accuracy.  One wave per singular value runs a 64-way
//     multisection: each lane counts the eigenvalues below one of 64 points of
//     the current bracket (the LDL^T recurrence q = -x - t^2 / q), and the
//     bracket shrinks 65-fold per round until it is 2 eps wide.
#include <algorithm>
#include <cfloat>

#include "host.hpp"
#include "device_common.hpp"

namespace rq {

constexpr int kSvdWaves = 16;
constexpr int kSvdChunk = 256;   // rows per pass of the row sums

// Reflector of x = (alpha, tail) with tail 2-norm^2 s2 (Section 2):
// beta = -sign(alpha) ||x||, v = (1, tail / (alpha - beta)), tau = (beta - alpha) / beta;
// a zero column gives tau = 0 and beta = 0.
RQ_DEV void svd_reflector(double alpha, double s2, double& beta, double& scale, double& tau) {
  const double nrm = sqrt(alpha * alpha + s2);
  if (nrm == 0.0) {
    beta = 0.0;
    scale = 0.0;
    tau = 0.0;
    return;
  }
  beta = (alpha >= 0.0) ? -nrm : nrm;
  scale = 1.0 / (alpha - beta);
  tau = (beta - alpha) / beta;
}

__global__ __launch_bounds__(1024) void bidiag_kernel(double* W, int64_t ldw, int k, double* d,
                                                      double* e) {
  __shared__ double s_v[RQ_MAX_SVD];              // the current reflector
  __shared__ double s_z[RQ_MAX_SVD];              // tau_R (W u) of the right step
  __shared__ double s_zp[kSvdWaves][kSvdChunk];   // per-wave partial row sums
  __shared__ double s_tau;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  for (int i = 0; i < k; ++i) {
    const int s = k - i;                           // rows (and columns) of the trailing block
    double* Wi = W + i + (int64_t)i * ldw;         // W(i, i)
    // ---- left reflector of column i, rows i..k-1 ----------------------------------
    if (wave == 0) {
      double s2 = 0.0;
      for (int r = 1 + lane; r < s; r += 64) s2 += Wi[r] * Wi[r];
      s2 = wave_sum(s2);
      double beta, scale, tau;
      svd_reflector(Wi[0], s2, beta, scale, tau);
      for (int r = lane; r < s; r += 64) s_v[r] = (r == 0) ? 1.0 : Wi[r] * scale;
      if (lane == 0) {
        s_tau = tau;
        d[i] = beta;
      }
    }
    __syncthreads();
    const double tl = s_tau;
    if (tl != 0.0) {
      for (int c = 1 + wave; c < s; c += kSvdWaves) {
        double* col = Wi + (int64_t)c * ldw;
        double dot = 0.0;
        for (int r = lane; r < s; r += 64) dot += s_v[r] * col[r];
        dot = wave_sum(dot) * tl;
        for (int r = lane; r < s; r += 64) col[r] -= dot * s_v[r];
      }
    }
    __syncthreads();
    if (s == 1) break;
    // ---- right reflector of row i, columns i+1..k-1 -----------------------------------
    const int sr = s - 1;                          // columns right of the diagonal
    double* Wr = Wi + ldw;                         // W(i, i + 1)
    if (wave == 0) {
      double s2 = 0.0;
      for (int c = 1 + lane; c < sr; c += 64) {
        const double x = Wr[(int64_t)c * ldw];
        s2 += x * x;
      }
      s2 = wave_sum(s2);
      double beta, scale, tau;
      svd_reflector(Wr[0], s2, beta, scale, tau);
      for (int c = lane; c < sr; c += 64) s_v[c] = (c == 0) ? 1.0 : Wr[(int64_t)c * ldw] * scale;
      if (lane == 0) {
        s_tau = tau;
        e[i] = beta;
      }
    }
    __syncthreads();
    const double tr = s_tau;
    double* Wb = Wr + 1;                           // W(i + 1, i + 1): sr x sr block
    // (tr is uniform; with tr = 0 there is nothing to apply)
    for (int r0 = 0; tr != 0.0 && r0 < sr; r0 += kSvdChunk) {
      double zp[kSvdChunk / 64];
#pragma unroll
      for (int q = 0; q < kSvdChunk / 64; ++q) zp[q] = 0.0;
      for (int c = wave; c < sr; c += kSvdWaves) {
        const double uc = s_v[c];
        const double* col = Wb + (int64_t)c * ldw;
#pragma unroll
        for (int q = 0; q < kSvdChunk / 64; ++q) {
          const int r = r0 + lane + 64 * q;
          if (r < sr) zp[q] += col[r] * uc;
        }
      }
#pragma unroll
      for (int q = 0; q < kSvdChunk / 64; ++q) s_zp[wave][lane + 64 * q] = zp[q];
      __syncthreads();
      if (t < kSvdChunk && r0 + t < sr) {
        double z = 0.0;
#pragma unroll
        for (int w = 0; w < kSvdWaves; ++w) z += s_zp[w][t];
        s_z[r0 + t] = z * tr;
      }
      __syncthreads();
    }
    for (int c = wave; tr != 0.0 && c < sr; c += kSvdWaves) {
      const double uc = s_v[c];
      double* col = Wb + (int64_t)c * ldw;
      for (int r = lane; r < sr; r += 64) col[r] -= s_z[r] * uc;
    }
    __syncthreads();   // before wave 0 rewrites s_v and s_tau
  }
}

__global__ __launch_bounds__(64) void bidiag_sv_kernel(const double* d, const double* e, int k,
                                                       double* sigma) {
  __shared__ double s_t2[2 * RQ_MAX_SVD];
  const int lane = threadIdx.x;
  const int j = blockIdx.x;                        // sigma[j] is the j-th largest
  const int nt = 2 * k - 1;                        // off-diagonal entries of the tridiagonal
  double fro = 0.0, big = 0.0;
  for (int q = lane; q < nt; q += 64) {
    const double tv = (q & 1) ? e[q >> 1] : d[q >> 1];
    const double t2 = tv * tv;
    s_t2[q] = t2;
    fro += t2;
    big = fmax(big, t2);
  }
  fro = wave_sum(fro);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) big = fmax(big, __shfl_xor(big, o));
  __syncthreads();
  // ||B||_F bounds every singular value
  double lo = 0.0, hi = sqrt(fro) * (1.0 + 8.0 * DBL_EPSILON);
  if (hi == 0.0) {
    if (lane == 0) sigma[j] = 0.0;
    return;
  }
  const double pivmin = DBL_MIN * fmax(1.0, big);
  const int target = k - 1 - j;                    // its index in ascending order
  for (int it = 0; it < 64 && hi - lo > 2.0 * DBL_EPSILON * hi; ++it) {
    const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
    // eigenvalues of the tridiagonal below x: negative pivots of LDL^T of T - x I
    int neg = 0;
    double qv = -x;
    neg += qv < 0.0;
    for (int q = 0; q < nt; ++q) {
      if (qv == 0.0) qv = -pivmin;
      qv = -x - s_t2[q] / qv;
      neg += qv < 0.0;
    }
    // the eigenvalues below x > 0 are the k negative ones and the singular
    // values below x
    const bool past = neg - k > target;
    const unsigned long long m = __builtin_amdgcn_ballot_w64(past);
    const int f = m ? __builtin_ctzll(m) : 64;     // first point past sigma_j
    const double nlo = (f == 0) ? lo : lo + (hi - lo) * (double)f / 65.0;
    const double nhi = (f == 64) ? hi : lo + (hi - lo) * (double)(f + 1) / 65.0;
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) sigma[j] = 0.5 * (lo + hi);
}

size_t singular_values_workspace_bytes(int64_t k) {
  return padded_bytes((size_t)k * k) + 2 * padded_bytes((size_t)k);
}

// Singular values of the k x k matrix X (ld ldx) into sigma[k], largest first.
// Needs singular_values_workspace_bytes(k) of workspace at `work`.
rq_status run_singular_values(rq_handle h, int64_t k, const double* X, int64_t ldx, double* sigma,
                              double* work) {
  if (k <= 0) return RQ_OK;
  Carve cv(reinterpret_cast<char*>(work));
  double* Wk = cv.take<double>((size_t)k * k);
  double* d = cv.take<double>((size_t)k);
  double* e = cv.take<double>((size_t)k);
  hipStream_t s = h->stream;
  {
    KTimer kt(h, K_SVD, 8.0 * k * k * k / 3.0, 8.0 * (2.0 * k * k + 2.0 * k));
    RQ_CHECK(h, launch_copy2d(X, ldx, Wk, k, (int)k, (int)k, s));
    hipLaunchKernelGGL(bidiag_kernel, dim3(1), dim3(64 * kSvdWaves), 0, s, Wk, k, (int)k, d, e);
    RQ_CHECK(h, hipGetLastError());
    hipLaunchKernelGGL(bidiag_sv_kernel, dim3((unsigned)k), dim3(64), 0, s, d, e, (int)k, sigma);
    RQ_CHECK(h, hipGetLastError());
  }
  return RQ_OK;
}

}  // namespace rq

using namespace rq;

extern "C" rq_status rq_singular_values(rq_handle h, int64_t k, const double* X, int64_t ldx,
                                        double* sigma) {
  if (!h) return -1;
  if (k < 0) return -2;
  if (!valid_ptr(X, k * k)) return -3;
  if (ldx < std::max<int64_t>(1, k)) return -4;
  if (!valid_ptr(sigma, k)) return -5;
  if (k == 0) return RQ_OK;
  if (k > RQ_MAX_SVD) return RQ_E_UNSUPPORTED;
  DeviceGuard guard(h->device);
  RQ_TRY(reserve(h, singular_values_workspace_bytes(k)));
  return run_singular_values(h, k, X, ldx, sigma, reinterpret_cast<double*>(h->ws));
}
