// Host side of the C ABI declared in include/rqrcp.h: handle, argument
// validation, workspace and the block loops that enqueue the gfx950 kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>

#include "../../include/rqrcp.h"
#include "kernels.hpp"

struct rq_handle_s {
  int device = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;          // grow-only workspace
  size_t ws_bytes = 0;
  int64_t* status = nullptr;   // device int64[4]
  uint32_t* sync = nullptr;    // device u32[64]: [0] barrier counter, [1] abort flag
  std::string last_error;
};

namespace {

using rq::launch_zero_u32;

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

rq_status fail(rq_handle h, hipError_t e, const char* where) {
  if (h) {
    h->last_error = std::string(where) + ": " + hipGetErrorString(e);
  }
  return RQ_E_HIP;
}

#define RQ_CHECK(h, expr)                              \
  do {                                                 \
    hipError_t _e = (expr);                            \
    if (_e != hipSuccess) return fail((h), _e, #expr); \
  } while (0)

// Bump allocator over the handle's workspace.  reserve() is called once with
// the total size before carving, so pointers stay valid for the whole call.
struct Carve {
  char* base;
  size_t off = 0;
  explicit Carve(char* b) : base(b) {}
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base + off);
    off += count * sizeof(T);
    return p;
  }
};

rq_status reserve(rq_handle h, size_t bytes) {
  if (bytes <= h->ws_bytes) return RQ_OK;
  if (h->ws) {
    RQ_CHECK(h, hipStreamSynchronize(h->stream));
    RQ_CHECK(h, hipFree(h->ws));
    h->ws = nullptr;
    h->ws_bytes = 0;
  }
  size_t want = bytes + (bytes >> 3);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&h->ws), want);
  if (e != hipSuccess) {
    h->ws = nullptr;
    h->last_error = "workspace allocation failed";
    return RQ_E_NOMEM;
  }
  h->ws_bytes = want;
  return RQ_OK;
}

size_t bytes_of_doubles(size_t n) { return n * sizeof(double) + 256; }

int panel_groups(int64_t M) { return (int)((M + rq::kPanelRows - 1) / rq::kPanelRows); }

// Sketch B = Omega A (ell x n) through split-K partials in `part`.
rq_status sketch_fp64(rq_handle h, int ell, int64_t m, int64_t n, const double* Omega,
                      int64_t ldo, const double* A, int64_t lda, double* B, int64_t ldb,
                      double* part) {
  int ks, kc;
  rq::plan_split((int)m, (int)n, &ks, &kc);
  rq::GemmArgs g{};
  g.L = Omega;
  g.sLp = 1;
  g.sLk = ldo;
  g.X = A;
  g.ldx = lda;
  g.P = ell;
  g.K = (int)m;
  g.N = (int)n;
  g.ksplit = ks;
  g.kchunk = kc;
  g.alpha = 1.0;
  g.beta = 0.0;
  if (ks == 1) {
    g.out = B;
    g.ldout = ldb;
    RQ_CHECK(h, rq::launch_gemm_lx(g, h->stream));
    return RQ_OK;
  }
  g.out = part;
  g.ldout = ell;
  g.split_stride = (int64_t)ell * n;
  RQ_CHECK(h, rq::launch_gemm_lx(g, h->stream));
  RQ_CHECK(h, rq::launch_reduce(part, ell, g.split_stride, ks, ell, (int)n, B, ldb, nullptr, 0,
                                0, h->stream));
  return RQ_OK;
}

size_t sketch_part_doubles(int ell, int64_t m, int64_t n) {
  int ks, kc;
  rq::plan_split((int)m, (int)n, &ks, &kc);
  return ks > 1 ? (size_t)ks * ell * n : 0;
}

struct SqWork {
  double* rec;
  int* src_top;
  int* dst_low;
};

rq_status run_sample_qrcp(rq_handle h, double* B, int64_t ldb, int ell, int64_t N, int steps,
                          SqWork w, int64_t* perm) {
  const int lm = rq::sq_lm(ell);
  rq::SqArgs a{};
  a.B = B;
  a.ldb = ldb;
  a.ell = ell;
  a.N = (int)N;
  a.steps = steps;
  a.nwg = (int)((N + 255) / 256);
  a.rec = w.rec;
  a.rs = rq::sq_record_stride(lm);
  a.counter = h->sync;
  a.abort_flag = h->sync + 1;
  a.status = h->status;
  a.src_top = w.src_top;
  a.dst_low = w.dst_low;
  a.perm = perm;
  RQ_CHECK(h, launch_zero_u32(h->sync, 2, h->stream));
  RQ_CHECK(h, rq::launch_sample_qrcp(a, lm, h->stream));
  return RQ_OK;
}

size_t sq_rec_doubles(int ell, int64_t N) {
  const int lm = rq::sq_lm(ell);
  return (size_t)2 * ((N + 255) / 256) * rq::sq_record_stride(lm);
}

rq_status run_panel(rq_handle h, double* A, int64_t lda, int64_t M, int bj, double* rec,
                    double* tau, double* Y, int64_t ldy, double* T, int64_t ldt) {
  rq::PanelArgs a{};
  a.A = A;
  a.lda = lda;
  a.M = (int)M;
  a.bj = bj;
  a.nwg = panel_groups(M);
  a.rec = rec;
  a.counter = h->sync;
  a.abort_flag = h->sync + 1;
  a.status = h->status;
  a.tau = tau;
  a.Y = Y;
  a.ldy = ldy;
  a.T = T;
  a.ldt = ldt;
  RQ_CHECK(h, launch_zero_u32(h->sync, 2, h->stream));
  RQ_CHECK(h, rq::launch_panel(a, h->stream));
  return RQ_OK;
}

size_t panel_rec_doubles(int64_t M) { return (size_t)2 * panel_groups(M) * 3 * 64; }

bool valid_ptr(const void* p, int64_t count) { return count <= 0 || p != nullptr; }

}  // namespace

extern "C" {

rq_status rq_create(rq_handle* out, int device, void* hip_stream) {
  if (!out) return -1;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return -2;
  DeviceGuard guard(device);
  rq_handle h = new rq_handle_s();
  h->device = device;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&h->status), 4 * sizeof(int64_t));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&h->sync), 64 * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemsetAsync(h->status, 0, 4 * sizeof(int64_t), h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->sync, 0, 64 * sizeof(uint32_t), h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) {
    if (h->status) (void)hipFree(h->status);
    if (h->sync) (void)hipFree(h->sync);
    delete h;
    return RQ_E_HIP;
  }
  *out = h;
  return RQ_OK;
}

rq_status rq_destroy(rq_handle h) {
  if (!h) return -1;
  DeviceGuard guard(h->device);
  (void)hipStreamSynchronize(h->stream);
  if (h->ws) (void)hipFree(h->ws);
  if (h->status) (void)hipFree(h->status);
  if (h->sync) (void)hipFree(h->sync);
  delete h;
  return RQ_OK;
}

rq_status rq_set_stream(rq_handle h, void* hip_stream) {
  if (!h) return -1;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return RQ_OK;
}

const char* rq_last_error(rq_handle h) { return h ? h->last_error.c_str() : "null handle"; }

rq_status rq_sync_status(rq_handle h, int64_t* device_error) {
  if (!h) return -1;
  DeviceGuard guard(h->device);
  RQ_CHECK(h, hipStreamSynchronize(h->stream));
  int64_t st[4] = {0, 0, 0, 0};
  RQ_CHECK(h, hipMemcpy(st, h->status, sizeof(st), hipMemcpyDeviceToHost));
  if (st[0]) {
    RQ_CHECK(h, hipMemset(h->status, 0, 4 * sizeof(int64_t)));
  }
  if (device_error) *device_error = st[0];
  return st[0] ? RQ_E_DEVICE : RQ_OK;
}

rq_status rq_sketch(rq_handle h, rq_prec prec, int64_t ell, int64_t m, int64_t n,
                    const double* Omega, int64_t ldo, const void* A, int64_t lda, double* B,
                    int64_t ldb) {
  if (!h) return -1;
  if (prec != RQ_FP64 && prec != RQ_MIXED_BF16) return -2;
  if (ell < 1 || ell > RQ_MAX_ELL) return -3;
  if (m < 0) return -4;
  if (n < 0 || n > RQ_MAX_N) return -5;
  if (!valid_ptr(Omega, ell * m)) return -6;
  if (ldo < std::max<int64_t>(1, ell)) return -7;
  if (!valid_ptr(A, m * n)) return -8;
  if (lda < std::max<int64_t>(1, m)) return -9;
  if (!valid_ptr(B, ell * n)) return -10;
  if (ldb < ell) return -11;
  if (prec != RQ_FP64) return RQ_E_UNSUPPORTED;
  if (n == 0) return RQ_OK;
  DeviceGuard guard(h->device);
  size_t need = bytes_of_doubles(sketch_part_doubles((int)ell, m, n));
  rq_status st = reserve(h, need);
  if (st) return st;
  Carve cv(h->ws);
  double* part = cv.take<double>(sketch_part_doubles((int)ell, m, n));
  return sketch_fp64(h, (int)ell, m, n, Omega, ldo, static_cast<const double*>(A), lda, B, ldb,
                     part);
}

rq_status rq_sample_qrcp(rq_handle h, int64_t ell, int64_t n, int64_t steps, double* B,
                         int64_t ldb, int64_t* perm) {
  if (!h) return -1;
  if (ell < 1 || ell > RQ_MAX_ELL) return -2;
  if (n < 0 || n > RQ_MAX_N) return -3;
  if (steps < 0 || steps > std::min(ell, n) || steps > RQ_MAX_B) return -4;
  if (!valid_ptr(B, ell * n)) return -5;
  if (ldb < ell) return -6;
  if (!valid_ptr(perm, n)) return -7;
  if (n == 0) return RQ_OK;
  DeviceGuard guard(h->device);
  size_t need = bytes_of_doubles(sq_rec_doubles((int)ell, n)) + 2 * 64 * sizeof(int) + 512;
  rq_status st = reserve(h, need);
  if (st) return st;
  Carve cv(h->ws);
  SqWork w;
  w.rec = cv.take<double>(sq_rec_doubles((int)ell, n));
  w.src_top = cv.take<int>(64);
  w.dst_low = cv.take<int>(64);
  if (steps == 0) {
    RQ_CHECK(h, rq::launch_iota(perm, (int)n, h->stream));
    return RQ_OK;
  }
  return run_sample_qrcp(h, B, ldb, (int)ell, n, (int)steps, w, perm);
}

rq_status rqrcp_factor(rq_handle h, int64_t m, int64_t n, int64_t k, int64_t b, int64_t p,
                       double* A, int64_t lda, const double* Omega, int64_t ldo, int64_t* jpvt,
                       double* tau, double* T, int64_t ldt) {
  if (!h) return -1;
  if (m < 0) return -2;
  if (n < 0 || n > RQ_MAX_N) return -3;
  if (k < 0 || k > std::min(m, n)) return -4;
  if (b < 1 || b > RQ_MAX_B) return -5;
  if (p < 0 || b + p > RQ_MAX_ELL) return -6;
  if (!valid_ptr(A, m * n)) return -7;
  if (lda < std::max<int64_t>(1, m)) return -8;
  const int64_t ell = b + p;
  if (k > 0 && ell > m) return -6;
  if (!valid_ptr(Omega, k > 0 ? ell * m : 0)) return -9;
  if (ldo < ell) return -10;
  if (!valid_ptr(jpvt, n)) return -11;
  if (!valid_ptr(tau, k)) return -12;
  if (T && ldt < b) return -14;
  if (n == 0) return RQ_OK;
  DeviceGuard guard(h->device);
  if (k == 0) {
    RQ_CHECK(h, rq::launch_iota(jpvt, (int)n, h->stream));
    return RQ_OK;
  }

  // ---- workspace -------------------------------------------------------------
  size_t w_part = 0;                                 // largest split-K buffer of any block
  for (int64_t c0 = 0; c0 < k; c0 += b) {
    const int64_t nt = n - c0 - std::min<int64_t>(b, k - c0);
    if (nt <= 0) continue;
    int ks_b, kc_b;
    rq::plan_split((int)(m - c0), (int)nt, &ks_b, &kc_b);
    w_part = std::max(w_part, (size_t)ks_b * 64 * nt);
  }
  const size_t n_sample = (size_t)ell * n;
  const size_t n_part = std::max(w_part, sketch_part_doubles((int)ell, m, n));
  const size_t n_sqrec = sq_rec_doubles((int)ell, n);
  const size_t n_prec = panel_rec_doubles(m);
  const size_t n_y = (size_t)m * 64;
  const size_t need = bytes_of_doubles(n_sample) + bytes_of_doubles(n_part) +
                      bytes_of_doubles(n_sqrec) + bytes_of_doubles(n_prec) +
                      bytes_of_doubles(n_y) + bytes_of_doubles(64 * 64) * 2 +
                      bytes_of_doubles((size_t)64 * n) + 4 * 64 * sizeof(int) + 1024;
  rq_status st = reserve(h, need);
  if (st) return st;
  Carve cv(h->ws);
  double* sample = cv.take<double>(n_sample);
  double* part = cv.take<double>(n_part);
  SqWork sw;
  sw.rec = cv.take<double>(n_sqrec);
  double* prec = cv.take<double>(n_prec);
  double* ybuf = cv.take<double>(n_y);
  double* tblk = cv.take<double>(64 * 64);
  double* mhat = cv.take<double>(64 * 64);
  double* zbuf = cv.take<double>((size_t)64 * n);
  sw.src_top = cv.take<int>(64);
  sw.dst_low = cv.take<int>(64);
  hipStream_t s = h->stream;

  // ---- B = Omega A -------------------------------------------------------------
  st = sketch_fp64(h, (int)ell, m, n, Omega, ldo, A, lda, sample, ell, part);
  if (st) return st;
  RQ_CHECK(h, rq::launch_iota(jpvt, (int)n, s));

  for (int64_t col0 = 0; col0 < k; col0 += b) {
    const int bj = (int)std::min<int64_t>(b, k - col0);
    const int64_t N = n - col0;
    const int64_t M = m - col0;
    double* Ablk = A + col0 + col0 * lda;            // trailing block A(col0:, col0:)
    // 1. sample pivots (QRCP(B, b)); the sample is rewritten in pivoted order
    st = run_sample_qrcp(h, sample + col0 * ell, ell, (int)ell, N, bj, sw, nullptr);
    if (st) return st;
    // 2. permute all m rows of A's columns col0.. (finished R rows included) and jpvt
    RQ_CHECK(h, rq::launch_permute(A + col0 * lda, lda, (int)m, bj, sw.src_top, sw.dst_low,
                                   jpvt + col0, s));
    // 3. panel QR of the b selected columns, T of the block
    st = run_panel(h, Ablk, lda, M, bj, prec, tau + col0, ybuf, m, tblk, 64);
    if (st) return st;
    if (T) RQ_CHECK(h, rq::launch_copy2d(tblk, 64, T + col0 * ldt, ldt, bj, bj, s));
    const int64_t Nt = N - bj;
    if (Nt <= 0) continue;
    double* Ctr = Ablk + bj * lda;                   // A(col0:, col0+bj:)
    // 4. W = Y^T A_trailing (split-K), Z = T^T W
    int ks, kc;
    rq::plan_split((int)M, (int)Nt, &ks, &kc);
    rq::GemmArgs g{};
    g.L = ybuf;
    g.sLp = m;
    g.sLk = 1;
    g.X = Ctr;
    g.ldx = lda;
    g.P = bj;
    g.K = (int)M;
    g.N = (int)Nt;
    g.ksplit = ks;
    g.kchunk = kc;
    g.out = part;
    g.ldout = 64;
    g.split_stride = (int64_t)64 * Nt;
    g.alpha = 1.0;
    g.beta = 0.0;
    // with ksplit == 1 the single product lands in `part` too (alpha=1, beta=0)
    RQ_CHECK(h, rq::launch_gemm_lx(g, s));
    RQ_CHECK(h, rq::launch_reduce(part, 64, g.split_stride, ks, bj, (int)Nt, zbuf, 64, tblk, 64,
                                  bj, s));
    // 5. A_trailing -= Y Z  (rows 0..bj-1 become R12)
    RQ_CHECK(h, rq::launch_update(Ctr, lda, (int)M, (int)Nt, ybuf, m, zbuf, 64, bj, s));
    // 6. sample update B1 = S12 - S11 R11^{-1} R12, B2 = S22 (in place)
    if (col0 + bj < k) {
      double* sblk = sample + col0 * ell;
      RQ_CHECK(h, rq::launch_omega11(sblk, ell, Ablk, lda, bj, mhat, 64, s));
      rq::GemmArgs u{};
      u.L = mhat;
      u.sLp = 1;
      u.sLk = 64;
      u.X = Ctr;
      u.ldx = lda;
      u.P = bj;
      u.K = bj;
      u.N = (int)Nt;
      u.ksplit = 1;
      u.kchunk = ((bj + 15) / 16) * 16;
      u.out = sblk + bj * ell;
      u.ldout = ell;
      u.alpha = -1.0;
      u.beta = 1.0;
      u.C = sblk + bj * ell;
      u.ldc = ell;
      RQ_CHECK(h, rq::launch_gemm_lx(u, s));
    }
  }
  return RQ_OK;
}

rq_status qrcp_factor(rq_handle h, int64_t m, int64_t n, int64_t k, int64_t nb, double* A,
                      int64_t lda, int64_t* jpvt, double* tau) {
  if (!h) return -1;
  (void)m; (void)n; (void)k; (void)nb; (void)A; (void)lda; (void)jpvt; (void)tau;
  return RQ_E_UNSUPPORTED;
}

rq_status trqrcp_truncate(rq_handle h, rq_prec prec, int64_t m, int64_t n, int64_t k, int64_t b,
                          int64_t p, const void* A, int64_t lda, const double* Omega, int64_t ldo,
                          int64_t* jpvt, double* Y, int64_t ldy, double* T, int64_t ldt,
                          double* R, int64_t ldr) {
  if (!h) return -1;
  (void)prec; (void)m; (void)n; (void)k; (void)b; (void)p; (void)A; (void)lda; (void)Omega;
  (void)ldo; (void)jpvt; (void)Y; (void)ldy; (void)T; (void)ldt; (void)R; (void)ldr;
  return RQ_E_UNSUPPORTED;
}

rq_status tuxv_svd(rq_handle h, rq_prec prec, int64_t m, int64_t n, int64_t k, int64_t b,
                   int64_t p, const void* A, int64_t lda, const double* Omega, int64_t ldo,
                   double* U, int64_t ldu, double* X, int64_t ldx, double* V, int64_t ldv,
                   int64_t* jpvt) {
  if (!h) return -1;
  (void)prec; (void)m; (void)n; (void)k; (void)b; (void)p; (void)A; (void)lda; (void)Omega;
  (void)ldo; (void)U; (void)ldu; (void)X; (void)ldx; (void)V; (void)ldv; (void)jpvt;
  return RQ_E_UNSUPPORTED;
}

}  // extern "C"
