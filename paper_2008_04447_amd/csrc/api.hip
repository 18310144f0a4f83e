// Host side of the C ABI declared in include/rqrcp.h: handle, argument
// validation, workspace, kernel timing and the RQRCP block loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cstring>
#include <string>

#include "device_common.hpp"
#include "host.hpp"

namespace rq {

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

static hipEvent_t next_event(rq_handle h) {
  if (h->pool_used < h->pool.size()) return h->pool[h->pool_used++];
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  h->pool.push_back(e);
  h->pool_used++;
  return e;
}

KTimer::KTimer(rq_handle h_, int cls_, double f_, double b_, hipStream_t s_)
    : h(h_), cls(cls_), f(f_), b(b_), s(s_) {
  if (h->prof && ((h->prof_mask >> cls) & 1u)) {
    e0 = next_event(h);
    if (e0) (void)hipEventRecord(e0, s);
  }
}

KTimer::~KTimer() {
  if (!e0) return;
  hipEvent_t e1 = next_event(h);
  if (!e1) return;
  (void)hipEventRecord(e1, s);
  h->recs.push_back(ProfRec{cls, e0, e1, f, b});
}

size_t sketch_part_doubles(int ell, int64_t m, int64_t n) {
  int ks, kc;
  plan_split((int)m, (int)n, &ks, &kc, ell);
  return ks > 1 ? (size_t)ks * ell * n : 0;
}

rq_status sketch_fp64(rq_handle h, int ell, int64_t m, int64_t n, const double* Omega, int64_t ldo,
                      const double* A, int64_t lda, double* B, int64_t ldb, double* part) {
  int ks, kc;
  plan_split((int)m, (int)n, &ks, &kc, ell);
  GemmArgs g{};
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
  const double fl = 2.0 * ell * m * n;
  const double by = 8.0 * ((double)m * n + (double)ell * m + (double)ell * n);
  if (ks == 1) {
    g.out = B;
    g.ldout = ldb;
    KTimer kt(h, K_SKETCH, fl, by);
    RQ_CHECK(h, launch_gemm_lx(g, h->stream));
    return RQ_OK;
  }
  g.out = part;
  g.ldout = ell;
  g.split_stride = (int64_t)ell * n;
  {
    KTimer kt(h, K_SKETCH, fl, by + 8.0 * ks * ell * n);
    RQ_CHECK(h, launch_gemm_lx(g, h->stream));
  }
  {
    KTimer kt(h, K_REDUCE, (double)(ks - 1) * ell * n, 8.0 * (ks + 1) * ell * n);
    RQ_CHECK(h, launch_reduce(part, ell, g.split_stride, ks, ell, (int)n, B, ldb, nullptr, 0, 0,
                              h->stream));
  }
  return RQ_OK;
}

static void plan_split32(int K, int N, int* ks, int* kc) {
  plan_split_target(K, N, 64, 512, ks, kc);
  *kc = ((*kc + 31) / 32) * 32;
  *ks = (K + *kc - 1) / *kc;
  if (*ks < 1) *ks = 1;
}

size_t sketch_part_doubles_bf16(int ell, int64_t m, int64_t n) {
  int ks, kc;
  plan_split32((int)m, (int)n, &ks, &kc);
  return (size_t)ks * ell * n;
}

rq_status gemm_lx_bf16_reduced(rq_handle h, int cls, GemmArgsF g, double* part, double* out,
                               int64_t ldout, __bf16* lbf) {
  int ks, kc;
  plan_split32(g.K, g.N, &ks, &kc);
  g.lbf = lbf;
  g.ksplit = ks;
  g.kchunk = kc;
  const double fl = 2.0 * g.P * (double)g.K * g.N;
  const double by = 4.0 * (double)g.K * g.N + 8.0 * ((double)g.P * g.K + (double)ks * g.P * g.N);
  if (ks == 1) {
    g.out = out;
    g.ldout = ldout;
    g.split_stride = 0;
    KTimer kt(h, cls, fl, by);
    RQ_CHECK(h, launch_gemm_lx_bf16(g, h->stream));
    return RQ_OK;
  }
  g.out = part;
  g.ldout = g.P;
  g.split_stride = (int64_t)g.P * g.N;
  {
    KTimer kt(h, cls, fl, by);
    RQ_CHECK(h, launch_gemm_lx_bf16(g, h->stream));
  }
  KTimer kt(h, K_REDUCE, (double)(ks - 1) * g.P * g.N, 8.0 * (ks + 1.0) * g.P * g.N);
  RQ_CHECK(h, launch_reduce(part, g.P, g.split_stride, ks, g.P, g.N, out, ldout, nullptr, 0, 0,
                            h->stream));
  return RQ_OK;
}

rq_status sketch_bf16(rq_handle h, int ell, int64_t m, int64_t n, const double* Omega, int64_t ldo,
                      const float* A, int64_t lda, double* B, int64_t ldb, double* part,
                      __bf16* lbf) {
  GemmArgsF g{};
  g.L = Omega;
  g.sLp = 1;
  g.sLk = ldo;
  g.X = A;
  g.ldx = lda;
  g.P = ell;
  g.K = (int)m;
  g.N = (int)n;
  return gemm_lx_bf16_reduced(h, K_SKETCH_BF16, g, part, B, ldb, lbf);
}

size_t sq_rec_doubles(int ell, int64_t N) {
  const int lm = sq_lm(ell);
  return (size_t)RQ_MAX_B * sq_max_groups(N) * sq_record_stride(lm);   // one slot per step
}

static int panel_groups(int64_t M);
static int64_t panel_prep_words(int64_t M, int bj);

// Cross-stream ordering in the RQRCP block loop.  Each link (one direction of
// one hand-over between the caller's stream and the side stream) has a 64-bit
// word in the handle's sync area, zero since the handle was created, and a
// running count on the host: the signalling side writes the next count once
// its earlier work has finished, and the waiting stream runs a one-wave
// kernel (wait_word_kernel) that holds its later work until the word has
// reached the count last written; the hand-over then takes a few
// microseconds, where an event took about 10 (7 without the system-scope
// fence).  A wait always names a count whose write is already enqueued (the
// count only advances once its write is), and the waiting kernel's spin is
// bounded besides.  The writes: the side stream's work done (U, P) and the
// product's start (Q) are stream memory operations; the update's release (Z)
// is written by the sample QRCP kernel itself once all its workgroups hold
// their compute units, so the caller's stream needs no operation before it.
// A call whose panels need every compute unit at once uses events (a pending
// wait holds part of a compute unit; a 65300-row factorization on 256 units
// timed out with the words), and so does every call where kernels of two
// streams do not run at the same time (a profiler's counter collection,
// kernel serialization): there a waiting kernel would wait for a kernel that
// cannot start.  h->link_values holds the choice for the current call.
enum { kLinkZ = 0, kLinkU, kLinkQ, kLinkP, kCallStart };
static bool link_on_words(rq_handle h, int /*link*/) { return h->link_values; }
// Each of two one-wave kernels, one per stream, sets its own flag and waits
// (at most `ticks` of the wall clock) for the other's: both see each other only
// when the two streams' kernels run at the same time.  words: u32[4], zero
// before; [0], [1] the flags, [2], [3] what each kernel saw.
__global__ void concurrency_probe_kernel(uint32_t* words, int me, uint64_t ticks) {
  if (threadIdx.x != 0) return;
  __hip_atomic_store(words + me, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  const uint64_t t0 = wall_clock64();
  uint32_t seen = 0u;
  while (wall_clock64() - t0 < ticks) {
    if (__hip_atomic_load(words + (1 - me), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
      seen = 1u;
      break;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  __hip_atomic_store(words + 2 + me, seen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Run once per handle, on the side stream and a stream of its own (never the
// caller's, whose queued work it does not wait for); blocks the host for the
// two kernels only, about 2 ms at most each.
static bool streams_run_concurrently(rq_handle h) {
  uint32_t* w = h->sync + 8;     // zero since the handle was created
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, h->device) != hipSuccess ||
      khz <= 0)
    return false;
  const uint64_t ticks = 2ull * (uint64_t)khz;   // 2 ms
  hipStream_t other = nullptr;
  if (hipStreamCreateWithFlags(&other, hipStreamNonBlocking) != hipSuccess) return false;
  hipLaunchKernelGGL(concurrency_probe_kernel, dim3(1), dim3(64), 0, h->side, w, 0, ticks);
  hipLaunchKernelGGL(concurrency_probe_kernel, dim3(1), dim3(64), 0, other, w, 1, ticks);
  bool ok = hipGetLastError() == hipSuccess;
  ok = (hipStreamSynchronize(other) == hipSuccess) && ok;
  (void)hipStreamDestroy(other);
  uint32_t seen[2] = {0u, 0u};
  ok = ok && hipMemcpyAsync(seen, w + 2, sizeof(seen), hipMemcpyDeviceToHost, h->side) == hipSuccess;
  ok = (hipStreamSynchronize(h->side) == hipSuccess) && ok;
  (void)hipGetLastError();
  return ok && seen[0] == 1u && seen[1] == 1u;
}

static uint64_t* link_word(rq_handle h, int l) {
  return reinterpret_cast<uint64_t*>(h->sync + 32) + 4 * l;   // 32 bytes apart
}
static hipError_t link_signal(rq_handle h, int l, hipStream_t s) {
  if (!link_on_words(h, l)) return hipEventRecord(h->link_ev[l], s);
  const hipError_t e = hipStreamWriteValue64(s, link_word(h, l), h->link_count[l] + 1, 0);
  if (e == hipSuccess) ++h->link_count[l];
  return e;
}
// Holds its stream until *word >= value: one wave that sleeps between its
// polls (about one device-coherent load per microsecond), so a workgroup that
// shares a compute unit with it loses few issue slots.  A wait that does not
// end within the bounded spin sets the timeout bit and the abort flag.
__global__ void wait_word_kernel(const uint64_t* word, uint64_t value, uint32_t* abort_flag,
                                 int64_t* status) {
  if (threadIdx.x != 0) return;
  uint32_t it = 0;
  while (__hip_atomic_load(word, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < value)
    if (!keep_waiting(it, abort_flag, status)) return;
}

static hipError_t link_wait(rq_handle h, int l, hipStream_t s) {
  if (!link_on_words(h, l)) return hipStreamWaitEvent(s, h->link_ev[l], 0);
  hipLaunchKernelGGL(wait_word_kernel, dim3(1), dim3(64), 0, s, link_word(h, l),
                     h->link_count[l], h->sync + 1, h->status);
  return hipGetLastError();
}

rq_status run_sample_qrcp(rq_handle h, double* B, int64_t ldb, int ell, int64_t N, int steps,
                          SqWork w, int64_t* perm, bool signal_side, double* panel_rec,
                          int64_t panel_m, int panel_bj, int groups, bool prepared) {
  const int lm = sq_lm(ell);
  SqArgs a{};
  a.B = B;
  a.ldb = ldb;
  a.ell = ell;
  a.N = (int)N;
  a.steps = steps;
  a.nwg = sq_groups(N, groups > 0 ? groups : h->max_groups);
  a.rec = w.rec;
  a.rs = sq_record_stride(lm);
  a.counter = h->sync;
  a.abort_flag = h->sync + 1;
  a.status = h->status;
  a.src_top = w.src_top;
  a.dst_low = w.dst_low;
  a.perm = perm;
  if (!prepared) {
    if (panel_rec)
      RQ_CHECK(h, launch_exchange_prep2(h->sync, w.rec, (int64_t)steps * a.nwg * a.rs, panel_rec,
                                        panel_prep_words(panel_m, panel_bj), h->stream));
    else
      RQ_CHECK(h, launch_exchange_prep(h->sync, w.rec, (int64_t)steps * a.nwg * a.rs, h->stream));
  }
  KTimer kt(h, K_SAMPLE_QRCP, 6.0 * ell * (double)N * steps, 16.0 * ell * (double)N);
  if (signal_side) {
    if (link_on_words(h, kLinkZ)) {   // the kernel writes the word
      a.release = link_word(h, kLinkZ);
      a.release_value = h->link_count[kLinkZ] + 1;
    } else {
      RQ_CHECK(h, link_signal(h, kLinkZ, h->stream));
    }
  }
  RQ_CHECK(h, launch_sample_qrcp(a, lm, h->stream));
  if (a.release) ++h->link_count[kLinkZ];
  return RQ_OK;
}

static int panel_groups(int64_t M) { return (int)((M + kPanelRows - 1) / kPanelRows); }

// Record words a panel of M rows and bj columns uses: the column-by-column
// route's, then (bj >= 2) the Cholesky-QR route's.
static int64_t panel_prep_words(int64_t M, int bj) {
  const int nwg = panel_groups(M);
  const int64_t hh = (int64_t)(bj + 1) * nwg * 3 * 64;
  return hh + (bj >= 2 ? panel_cholqr_doubles(nwg) : 0);
}

// Buffers of the Cholesky-QR route after a panel's record words: Q (M x 64,
// or ldq x 64 for an ldq up to the M the area is sized for), R = R2 R1,
// L11^{-1} (64 x 64 each) and S (64).
static int64_t panel_extra_doubles(int64_t M) { return M * 64 + 2 * 4096 + 64; }

size_t panel_rec_doubles(int64_t M) {
  return (size_t)(RQ_MAX_B + 1) * panel_groups(M) * 3 * 64 +
         (size_t)panel_cholqr_doubles(panel_groups(M)) + (size_t)panel_extra_doubles(M);
}

static PanelArgs panel_args(rq_handle h, double* A, int64_t lda, int64_t M, int bj, double* rec,
                            double* tau, double* Y, int64_t ldy, double* T, int64_t ldt,
                            int64_t ldq = 0) {
  PanelArgs a{};
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
  // the Cholesky-QR route is tried for panels of two or more columns
  const int64_t hh = (int64_t)(bj + 1) * a.nwg * 3 * 64;
  a.crec = bj >= 2 ? rec + hh : nullptr;
  a.fallback = a.crec ? h->sync + 2 : nullptr;
  double* const extra = rec + panel_prep_words(M, bj);
  a.ldq = std::max<int64_t>(ldq > 0 ? ldq : M, 1);   // ldq >= M; the area holds ldq x 64
  a.qbuf = extra;
  a.rbuf = extra + a.ldq * 64;
  a.linv = a.rbuf + 4096;
  a.sgnb = a.linv + 4096;
  return a;
}

rq_status run_panel(rq_handle h, double* A, int64_t lda, int64_t M, int bj, double* rec,
                    double* tau, double* Y, int64_t ldy, double* T, int64_t ldt, bool prepared) {
  const PanelArgs a = panel_args(h, A, lda, M, bj, rec, tau, Y, ldy, T, ldt);
  if (!prepared) RQ_CHECK(h, launch_exchange_prep(h->sync, rec, panel_prep_words(M, bj), h->stream));
  KTimer kt(h, K_PANEL, 2.0 * (double)M * bj * bj, 8.0 * (double)M * (2.0 * bj + 64));
  RQ_CHECK(h, launch_panel(a, h->stream));
  return RQ_OK;
}

// B1 = S12 - (S11 R11^{-1}) R12 in place on rows 0..bj-1 of the sample block
// (columns bj..), B2 = S22 untouched (eq. update1).
rq_status run_sample_update(rq_handle h, double* sblk, int ell, const double* R11, int64_t ldr,
                            const double* R12, int64_t ldr12, int bj, int64_t Nt, double* mhat,
                            const RankCheck* rk, const RecordPrep* prep) {
  {
    KTimer kt(h, K_OMEGA11, (double)bj * bj * bj / 3.0, 8.0 * 2 * bj * bj);
    RQ_CHECK(h, launch_omega11(sblk, ell, R11, ldr, bj, mhat, 64, rk, prep, h->stream));
  }
  GemmArgs u{};
  u.L = mhat;
  u.sLp = 1;
  u.sLk = 64;
  u.X = R12;
  u.ldx = ldr12;
  u.P = bj;
  u.K = bj;
  u.N = (int)Nt;
  u.ksplit = 1;
  u.kchunk = ((bj + 15) / 16) * 16;
  u.out = sblk + (int64_t)bj * ell;
  u.ldout = ell;
  u.alpha = -1.0;
  u.beta = 1.0;
  u.C = sblk + (int64_t)bj * ell;
  u.ldc = ell;
  u.skip_if = rk ? rk->info : nullptr;
  KTimer kt(h, K_SAMPLE_UPDATE, 2.0 * bj * bj * (double)Nt, 8.0 * 3.0 * bj * (double)Nt);
  RQ_CHECK(h, launch_gemm_lx(u, h->stream));
  return RQ_OK;
}

}  // namespace rq

using namespace rq;

// Scratch memory of rq_sample_qrcp_noalloc, which allocates nothing: the
// exchange records of one sample-QRCP launch of up to RQ_NOALLOC_MAX_N columns
// (64 steps x 128 workgroups x a 100-word record) and the two column maps.
// Each device holds its own copy until the process ends; calls that overlap on
// one device share it and race.
namespace {
constexpr size_t kScratchRec = (size_t)RQ_MAX_B * 128 * (RQ_MAX_ELL + 4);
constexpr size_t kScratchDoubles = kScratchRec + 2 * 64;
static_assert(kScratchRec >= (size_t)RQ_MAX_B * ((RQ_NOALLOC_MAX_N + 127) / 128) * (RQ_MAX_ELL + 4),
              "records of the widest sample fit");
}  // namespace
static __device__ __align__(256) double scratch[kScratchDoubles];

extern "C" {

rq_status rq_create(rq_handle* out, int device, void* hip_stream) {
  if (!out) return -1;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return -2;
  DeviceGuard guard(device);
  rq_handle h = new rq_handle_s();
  h->device = device;
  h->stream = reinterpret_cast<hipStream_t>(hip_stream);
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
      cus > 0) {
    h->update_wgs = cus;
    h->cus = cus;
  }
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&h->status), 4 * sizeof(int64_t));
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&h->sync), 64 * sizeof(uint32_t));
  if (e == hipSuccess) e = hipMemsetAsync(h->status, 0, 4 * sizeof(int64_t), h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->sync, 0, 64 * sizeof(uint32_t), h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e == hipSuccess) {
    // the device address of this device's copy of the static scratch array
    // (the array's name is only a host-side stand-in)
    void* p = nullptr;
    const hipError_t es = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (es == hipSuccess) {
      h->scratch = static_cast<double*>(p);
    } else {
      h->last_error = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(es);
      (void)hipGetLastError();
    }
  }
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
  if (h->side) {
    (void)hipStreamSynchronize(h->side);
    (void)hipStreamDestroy(h->side);
  }
  for (hipEvent_t e : h->link_ev)
    if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->pool) (void)hipEventDestroy(e);
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
  if (st[0]) RQ_CHECK(h, hipMemset(h->status, 0, 4 * sizeof(int64_t)));
  if (device_error) *device_error = st[0];
  return st[0] ? RQ_E_DEVICE : RQ_OK;
}

rq_status rq_workspace_query(rq_handle h, int32_t op, rq_prec prec, int64_t m, int64_t n, int64_t k,
                             int64_t b, int64_t p, size_t* bytes) {
  if (!h) return -1;
  if (op < RQ_OP_TRQRCP || op > RQ_OP_SAMPLE_QRCP) return -2;
  if (prec != RQ_FP64 && prec != RQ_MIXED_BF16) return -3;
  if (m < 0) return -4;
  if (n < 0 || n > RQ_MAX_N) return -5;
  if (!bytes) return -9;
  const int64_t ell = b + p;
  switch (op) {
    case RQ_OP_QRCP:
      if (k < 0 || k > std::min(m, n)) return -6;
      if (b < 1 || b > 64) return -7;
      *bytes = qrcp_workspace_bytes(m, n, k);
      return RQ_OK;
    case RQ_OP_SKETCH:
      if (ell < 1 || ell > RQ_MAX_ELL) return -7;
      *bytes = sketch_workspace_bytes(ell, m, n);
      return RQ_OK;
    case RQ_OP_SAMPLE_QRCP:
      if (ell < 1 || ell > RQ_MAX_ELL) return -7;
      if (k < 0 || k > std::min(ell, n) || k > RQ_MAX_B) return -6;
      *bytes = (k > 0) ? sample_qrcp_workspace_bytes(ell, n) : 0;
      return RQ_OK;
    default:
      break;
  }
  if (k < 0 || k > std::min(m, n)) return -6;
  if (b < 1 || b > RQ_MAX_B) return -7;
  if (p < 0 || ell > RQ_MAX_ELL || (k > 0 && ell > m)) return -8;
  if (op == RQ_OP_RQRCP || op == RQ_OP_RSRQRCP)
    *bytes = rqrcp_workspace_bytes(m, n, k, b, p, op == RQ_OP_RSRQRCP);
  else
    *bytes = (k > 0 && n > 0) ? truncated_workspace_bytes(m, n, k, (int)ell, op == RQ_OP_TUXV) : 0;
  return RQ_OK;
}

rq_status rq_workspace_reserve(rq_handle h, size_t bytes) {
  if (!h) return -1;
  DeviceGuard guard(h->device);
  return reserve(h, bytes);
}

rq_status rq_workspace_size(rq_handle h, size_t* bytes) {
  if (!h) return -1;
  if (!bytes) return -2;
  *bytes = h->ws_bytes;
  return RQ_OK;
}

rq_status rq_profile_classes(rq_handle h, uint32_t mask) {
  if (!h) return -1;
  h->prof_mask = mask;
  return RQ_OK;
}

rq_status rq_profile_start(rq_handle h) {
  if (!h) return -1;
  h->prof = true;
  h->recs.clear();
  h->pool_used = 0;
  for (auto& t : h->tot) t = ProfTot{};
  return RQ_OK;
}

rq_status rq_profile_stop(rq_handle h) {
  if (!h) return -1;
  DeviceGuard guard(h->device);
  RQ_CHECK(h, hipStreamSynchronize(h->stream));
  for (const ProfRec& r : h->recs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, r.e0, r.e1) != hipSuccess) continue;
    ProfTot& t = h->tot[r.cls];
    t.launches += 1;
    t.ms += ms;
    t.flops += r.flops;
    t.bytes += r.bytes;
  }
  h->recs.clear();
  h->pool_used = 0;
  h->prof = false;
  return RQ_OK;
}

int32_t rq_profile_count(rq_handle h) { return h ? (int32_t)K_NUM_CLASSES : 0; }

rq_status rq_profile_get(rq_handle h, int32_t index, const char** name, int64_t* launches,
                         double* total_ms, double* flops, double* bytes) {
  if (!h) return -1;
  if (index < 0 || index >= K_NUM_CLASSES) return -2;
  const ProfTot& t = h->tot[index];
  if (name) *name = kclass_name(index);
  if (launches) *launches = t.launches;
  if (total_ms) *total_ms = t.ms;
  if (flops) *flops = t.flops;
  if (bytes) *bytes = t.bytes;
  return RQ_OK;
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
  if (n == 0) return RQ_OK;
  if (m > INT_MAX) return RQ_E_UNSUPPORTED;   // the products index rows with 32-bit ints
  DeviceGuard guard(h->device);
  const size_t np = std::max(sketch_part_doubles((int)ell, m, n),
                             sketch_part_doubles_bf16((int)ell, m, n));
  const size_t nl = bf16_stage_doubles(m);
  RQ_TRY(reserve(h, sketch_workspace_bytes(ell, m, n)));
  Carve cv(h->ws);
  double* part = cv.take<double>(np);
  __bf16* lbf = reinterpret_cast<__bf16*>(cv.take<double>(nl));
  if (prec == RQ_MIXED_BF16)
    return sketch_bf16(h, (int)ell, m, n, Omega, ldo, static_cast<const float*>(A), lda, B, ldb,
                       part, lbf);
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
  if (steps > 0 && !rows_fit(h, n)) return RQ_E_UNSUPPORTED;
  DeviceGuard guard(h->device);
  RQ_TRY(reserve(h, sample_qrcp_workspace_bytes(ell, n)));
  Carve cv(h->ws);
  SqWork w;
  w.rec = cv.take<double>(sq_rec_doubles((int)ell, n));
  w.src_top = cv.take<int>(64);
  w.dst_low = cv.take<int>(64);
  // identity first: a pivoting that stops early (no admissible column) leaves it
  RQ_CHECK(h, launch_iota(perm, (int)n, h->stream));
  if (steps == 0) return RQ_OK;
  return run_sample_qrcp(h, B, ldb, (int)ell, n, (int)steps, w, perm);
}

rq_status rq_sample_qrcp_noalloc(rq_handle h, int64_t ell, int64_t n, int64_t steps, double* B,
                                 int64_t ldb, int64_t* perm) {
  if (!h) return -1;
  if (ell < 1 || ell > RQ_MAX_ELL) return -2;
  if (n < 0 || n > RQ_MAX_N) return -3;
  if (steps < 0 || steps > std::min(ell, n) || steps > RQ_MAX_B) return -4;
  if (!valid_ptr(B, ell * n)) return -5;
  if (ldb < ell) return -6;
  if (!valid_ptr(perm, n)) return -7;
  if (n > RQ_NOALLOC_MAX_N) return RQ_E_UNSUPPORTED;   // beyond the static scratch
  if (n == 0) return RQ_OK;
  if (steps > 0 && !rows_fit(h, n)) return RQ_E_UNSUPPORTED;
  if (!h->scratch) return RQ_E_HIP;     // the address lookup at rq_create failed
  DeviceGuard guard(h->device);
  SqArgs a{};
  a.B = B;
  a.ldb = ldb;
  a.ell = (int)ell;
  a.N = (int)n;
  a.steps = (int)steps;
  a.nwg = sq_groups(n, h->max_groups);
  a.rs = sq_record_stride(sq_lm((int)ell));
  a.rec = h->scratch;
  a.counter = h->sync;
  a.abort_flag = h->sync + 1;
  a.status = h->status;
  a.src_top = reinterpret_cast<int*>(h->scratch + kScratchRec);
  a.dst_low = reinterpret_cast<int*>(h->scratch + kScratchRec + 64);
  a.perm = perm;
  const int64_t words = steps * (int64_t)a.nwg * a.rs;
  if ((size_t)words > kScratchRec) return RQ_E_UNSUPPORTED;
  RQ_CHECK(h, launch_iota(perm, (int)n, h->stream));
  if (steps == 0) return RQ_OK;
  // a fill kernel (not a memset) marks the records unpublished and clears the flags
  RQ_CHECK(h, launch_exchange_prep(h->sync, h->scratch, words, h->stream));
  RQ_CHECK(h, launch_sample_qrcp(a, sq_lm((int)ell), h->stream));
  return RQ_OK;
}

}  // extern "C"

// Largest split-K buffer of any block of the RQRCP loop (and of the sketches).
// Workgroup slots the inner products of a block of M rows plan their split of
// K for: beside the panel's second half (the usual route) its workgroups hold
// whole compute units, so they are left out -- down to a floor, since a panel
// of up to 65536 rows can hold every unit (the product then mostly runs after it).
static int inner_slots(int64_t M, bool resample) {
  return resample ? 256 : std::max(64, 256 - panel_groups(M));
}

static size_t rqrcp_part_doubles(int64_t m, int64_t n, int64_t k, int64_t b, int64_t p,
                                 bool resample) {
  const int64_t ell = b + p;
  size_t w_part = 0;
  for (int64_t c0 = 0; c0 < k; c0 += b) {
    const int64_t nt = n - c0 - std::min<int64_t>(b, k - c0);
    if (nt <= 0) continue;
    int ks_b, kc_b;
    plan_split_rounds((int)(m - c0), (int)nt, inner_slots(m - c0, resample), &ks_b, &kc_b);
    w_part = std::max(w_part, (size_t)ks_b * 64 * nt);
    const int64_t c1 = c0 + std::min<int64_t>(b, k - c0);     // next block's sketch
    if (resample && c1 < k) w_part = std::max(w_part, sketch_part_doubles((int)ell, m - c1, n - c1));
  }
  return std::max(w_part, sketch_part_doubles((int)ell, m, n));
}

namespace rq {
size_t rqrcp_workspace_bytes(int64_t m, int64_t n, int64_t k, int64_t b, int64_t p, bool resample) {
  if (k <= 0 || n <= 0) return 0;
  const int64_t ell = b + p;
  return padded_bytes((size_t)ell * n) + padded_bytes(rqrcp_part_doubles(m, n, k, b, p, resample)) +
         padded_bytes(sq_rec_doubles((int)ell, n)) + padded_bytes(panel_rec_doubles(m)) +
         padded_bytes((size_t)m * 64) + 2 * padded_bytes(64 * 64) + padded_bytes((size_t)64 * n) +
         4 * 64 * sizeof(int) + 1024;
}

size_t sketch_workspace_bytes(int64_t ell, int64_t m, int64_t n) {
  if (n <= 0) return 0;
  const size_t np = std::max(sketch_part_doubles((int)ell, m, n), sketch_part_doubles_bf16((int)ell, m, n));
  return padded_bytes(np) + padded_bytes(bf16_stage_doubles(m));
}

size_t sample_qrcp_workspace_bytes(int64_t ell, int64_t n) {
  if (n <= 0) return 0;
  return padded_bytes(sq_rec_doubles((int)ell, n)) + 2 * 64 * sizeof(int) + 512;
}
}  // namespace rq

// The block loop of Algorithm 4.  With `resample` (repeated sampling, Section
// 3.4) the sample of block J is a fresh sketch of the updated trailing matrix,
// B = Omega^[J] A^[J], with Omega^[J] the first m - Jb columns of the ell x m
// slice Omega + J ostride, instead of the sample update (eq. update1).
static rq_status rqrcp_core(rq_handle h, int64_t m, int64_t n, int64_t k, int64_t b, int64_t p,
                            double* A, int64_t lda, const double* Omega, int64_t ldo,
                            int64_t ostride, bool resample, int64_t* jpvt, double* tau, double* T,
                            int64_t ldt, int64_t* info) {
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
  const int64_t nblk = (k + b - 1) / b;
  if (!valid_ptr(Omega, k > 0 ? (resample ? ostride * (nblk - 1) + ldo * m : ell * m) : 0)) return -9;
  if (ldo < ell) return -10;
  if (!valid_ptr(jpvt, n)) return -11;
  if (!valid_ptr(tau, k)) return -12;
  if (T && ldt < b) return -14;
  if (n == 0) return RQ_OK;
  if (k > 0 && !rows_fit(h, std::max(m, n))) return RQ_E_UNSUPPORTED;
  DeviceGuard guard(h->device);
  hipStream_t s = h->stream;
  // the rank check's record: the caller's, else a spare word of the status area
  int64_t* info_p = info ? info : h->status + 2;
  if (k == 0 || resample) {
    if (info) RQ_CHECK(h, launch_set_i64(info, 0, s));
    if (k == 0) {
      RQ_CHECK(h, launch_iota(jpvt, (int)n, s));
      return RQ_OK;
    }
  } else {
    RQ_CHECK(h, launch_set_i64(info_p, 0, s));
  }

  // ---- workspace -------------------------------------------------------------
  const size_t need = rqrcp_workspace_bytes(m, n, k, b, p, resample);
  const size_t n_sample = (size_t)ell * n;
  const size_t n_part = rqrcp_part_doubles(m, n, k, b, p, resample);
  const size_t n_sqrec = sq_rec_doubles((int)ell, n);
  const size_t n_prec = panel_rec_doubles(m);
  const size_t n_y = (size_t)m * 64;
  RQ_TRY(reserve(h, need));
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

  if (!h->side) {
    RQ_CHECK(h, hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
    for (hipEvent_t& e : h->link_ev)
      RQ_CHECK(h, hipEventCreateWithFlags(&e, hipEventDisableTiming | hipEventDisableSystemFence));
    h->words_ok = streams_run_concurrently(h);
  }
  // the panels, the widest persistent kernels of the loop, take panel_groups(m)
  // compute units at most; a pending wait on the words may hold one more
  h->link_values = h->words_ok && panel_groups(m) < h->cus;
  // A word wait's spin is bounded, so the second stream must not start its
  // first wait of this call before the caller's stream gets here: the caller's
  // earlier work may take longer than that bound.  One event orders the two.
  if (h->link_values) {
    RQ_CHECK(h, hipEventRecord(h->link_ev[kCallStart], s));
    RQ_CHECK(h, hipStreamWaitEvent(h->side, h->link_ev[kCallStart], 0));
  }
  // The update of the rows below R12 runs on the side stream.  It is handed to
  // that stream only after the next block's sample QRCP is queued and waits on
  // a link signalled right before that launch: the persistent kernel needs
  // whole compute units, and reaching the dispatcher first it gets them before
  // the update's many workgroups fill the device.
  struct SideUpdate {
    double* C;
    int64_t M, N;
    const double* Y;
    int bj;
  } side{};
  bool side_queued = false;   // `side` is waiting to be handed to the side stream
  bool pending_rows = false;  // the side stream holds an update the main stream must wait for
  // `beside`: workgroups of the sample QRCP the update runs next to
  auto release_side = [&](int beside) -> rq_status {
    RQ_CHECK(h, link_wait(h, kLinkZ, h->side));
    {
      const double Mr = (double)side.M, Nr = (double)side.N;
      KTimer kt(h, K_UPDATE, 2.0 * side.bj * Mr * Nr,
                8.0 * (2.0 * Mr * Nr + Mr * side.bj + (double)side.bj * Nr), h->side);
      RQ_CHECK(h, launch_update(side.C, lda, (int)side.M, (int)side.N, side.Y, m, zbuf, 64,
                                side.bj, std::max(1, h->update_wgs - beside), h->side));
    }
    RQ_CHECK(h, link_signal(h, kLinkU, h->side));
    side_queued = false;
    pending_rows = true;
    return RQ_OK;
  };

  // ---- B = Omega A -------------------------------------------------------------
  RQ_TRY(sketch_fp64(h, (int)ell, m, n, Omega, ldo, A, lda, sample, ell, part));
  RQ_CHECK(h, launch_iota(jpvt, (int)n, s));

  // the records of the next block's sample QRCP and panel were prepared by
  // this block's sample-update launch
  bool prepared = false;
  for (int64_t col0 = 0; col0 < k; col0 += b) {
    const int bj = (int)std::min<int64_t>(b, k - col0);
    const int64_t N = n - col0;
    const int64_t M = m - col0;
    double* Ablk = A + col0 + col0 * lda;            // trailing block A(col0:, col0:)
    // 1. sample pivots, QRCP(B, b); the sample is rewritten in pivoted order
    RQ_TRY(run_sample_qrcp(h, sample + col0 * ell, ell, (int)ell, N, bj, sw, nullptr,
                           side_queued, prec, M, bj, /*groups=*/0, prepared));
    prepared = false;
    if (side_queued) RQ_TRY(release_side(sq_groups(N, h->max_groups)));
    // the previous block's update of rows below its R12 must be complete
    if (pending_rows) {
      RQ_CHECK(h, link_wait(h, kLinkU, s));
      pending_rows = false;
    }
    // 2. permute all m rows of A's columns col0.. (finished R rows included), jpvt
    {
      KTimer kt(h, K_PERMUTE, 0.0, 32.0 * bj * (double)m);
      RQ_CHECK(h, launch_permute(A + col0 * lda, lda, (int)m, bj, n - col0, sw.src_top,
                                 sw.dst_low, jpvt + col0, s));
    }
    // 3. panel QR of the b selected columns and T of the block (written straight
    // into the caller's T when there is one: only its bj x bj block is touched)
    double* tj = T ? T + col0 * ldt : tblk;
    const int64_t ldtj = T ? ldt : 64;
    const int64_t Nt = N - bj;
    double* Ctr = Ablk + bj * lda;                   // A(col0:, col0+bj:)
    const PanelArgs pa = panel_args(h, Ablk, lda, M, bj, prec, tau + col0, ybuf, m, tj, ldtj, m);
    int ks = 1, kc = 64;
    if (Nt > 0) plan_split_rounds((int)M, (int)Nt, inner_slots(M, resample), &ks, &kc);   // as sized in rqrcp_part_doubles
    // The inner products of step 4 need only Q of the Cholesky-QR route
    // (P = Q^T A_trailing; the reduce forms R12 = S P and Z from it), so they
    // run on the side stream beside the panel's second half (the LU of Q11 - S
    // and the reflectors).  The side stream's launch waits on a link
    // signalled right before the second half's launch, which thus reaches the
    // dispatcher first and gets its compute units.  When the column-by-column
    // route runs instead, the same launch reads its Y (the panel's fallback
    // flag selects the operand) and the reduce takes the W = Y^T A form.
    const bool overlap = !resample && Nt > 0 && pa.crec && kc > 64;
    GemmArgs g{};
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
    g.out = part;                                    // ksplit == 1 lands here too
    g.ldout = 64;
    g.split_stride = (int64_t)64 * Nt;
    g.alpha = 1.0;
    g.beta = 0.0;
    const double inner_flops = 2.0 * bj * (double)M * Nt;
    const double inner_bytes = 8.0 * ((double)M * Nt + (double)M * bj + (double)ks * bj * Nt);
    {
      KTimer kt(h, K_PANEL, 2.0 * (double)M * bj * bj, 8.0 * (double)M * (2.0 * bj + 64));
      RQ_CHECK(h, launch_panel_first(pa, s));
    }
    if (overlap) {
      RQ_CHECK(h, link_signal(h, kLinkQ, s));
      RQ_CHECK(h, link_wait(h, kLinkQ, h->side));
      g.L = pa.qbuf;                                 // ldq = m, the strides of Y
      g.L_alt = ybuf;
      g.alt_if = pa.fallback;
      {
        KTimer kt(h, K_INNER, inner_flops, inner_bytes, h->side);
        RQ_CHECK(h, launch_gemm_lx(g, h->side));
      }
      RQ_CHECK(h, link_signal(h, kLinkP, h->side));
    }
    {
      KTimer kt(h, K_PANEL, 0.0, 0.0);
      RQ_CHECK(h, launch_panel_second(pa, s));
    }
    if (Nt <= 0) continue;
    // 4. W = Y^T A_trailing (split-K partials), Z = T^T W -- or, overlapped,
    // P = Q^T A_trailing, R12 = S P, Z = L11^{-1} (A_top - S P)
    if (overlap) {
      RQ_CHECK(h, link_wait(h, kLinkP, s));
    } else {
      KTimer kt(h, K_INNER, inner_flops, inner_bytes);
      RQ_CHECK(h, launch_gemm_lx(g, s));
    }
    {
      // with step 5 for rows 0..bj-1 (R12): the sample update and the next
      // block's sample QRCP need only them
      KTimer kt(h, K_REDUCE,
                (double)bj * bj * Nt + (double)(ks - 1) * bj * Nt + 2.0 * bj * (double)bj * Nt,
                8.0 * ((double)ks * bj * Nt + 64.0 * Nt + 2.0 * bj * (double)Nt));
      RQ_CHECK(h, launch_reduce_r12(part, g.split_stride, ks, (int)Nt, zbuf, tj, ldtj, ybuf, m,
                                    Ctr, lda, bj, s, overlap ? pa.fallback : nullptr, pa.linv,
                                    pa.sgnb));
    }
    if (resample) {
      // 5. A_trailing -= Y Z for the rows below R12, then 6'. the next sample,
      // Omega^[J+1] times the updated trailing matrix
      if (M > bj) {
        const double Mr = (double)(M - bj), Nr = (double)Nt;
        KTimer kt(h, K_UPDATE, 2.0 * bj * Mr * Nr, 8.0 * (2.0 * Mr * Nr + Mr * bj + (double)bj * Nr));
        RQ_CHECK(h, launch_update(Ctr + bj, lda, (int)(M - bj), (int)Nt, ybuf + bj, m, zbuf, 64, bj,
                                  h->update_wgs, s));
      }
      if (col0 + bj < k)
        RQ_TRY(sketch_fp64(h, (int)ell, M - bj, Nt, Omega + (col0 / b + 1) * ostride, ldo,
                           Ctr + bj, lda, sample + (col0 + bj) * ell, ell, part));
      continue;
    }
    // 5. A_trailing -= Y Z for the rows below R12: on the side stream alongside
    // the next sample QRCP (see release_side); the next block waits for them
    // before it permutes and factors its panel.
    // 6. sample update B1 = S12 - S11 R11^{-1} R12, B2 = S22 (in place)
    // (or, once R11 has been numerically singular, a fresh sample of the updated
    // trailing matrix with Omega's first M - bj columns; see launch_omega11)
    if (col0 + bj < k) {
      RankCheck rk{};
      rk.info = info_p;
      rk.r00 = A;                     // R_00, the first diagonal entry of R
      rk.thresh = DBL_EPSILON * (double)std::max(m, n);
      rk.col0 = col0;
      rk.Om = Omega;
      rk.ldo = ldo;
      rk.C = Ctr + bj;                // rows below R12, before their update
      rk.ldc = lda;
      rk.M2 = (int)(M - bj);
      rk.Y = ybuf + bj;
      rk.ldy = m;
      rk.Z = zbuf;
      rk.ldz = 64;
      rk.bj = bj;
      rk.ell = (int)ell;
      rk.N = (int)Nt;
      rk.B = sample + (col0 + bj) * ell;
      rk.ldb = ell;
      // the next block's records: its sample QRCP (bjn steps over Nn columns)
      // and its panel (Mn rows), as run_sample_qrcp would prepare them
      const int64_t col1 = col0 + bj;
      const int bjn = (int)std::min<int64_t>(b, k - col1);
      RecordPrep rp{};
      rp.sync = h->sync;
      rp.rec1 = sw.rec;
      rp.n1 = (int64_t)bjn * sq_groups(n - col1, h->max_groups) * sq_record_stride(sq_lm((int)ell));
      rp.rec2 = prec;
      rp.n2 = panel_prep_words(m - col1, bjn);
      RQ_TRY(run_sample_update(h, sample + col0 * ell, (int)ell, Ablk, lda, Ctr, lda, bj, Nt,
                               mhat, &rk, &rp));
      prepared = true;
    }
    if (M > bj) {
      side = SideUpdate{Ctr + bj, M - bj, Nt, ybuf + bj, bj};
      side_queued = true;
    }
  }
  if (side_queued) {                // no sample QRCP follows: release it now
    RQ_CHECK(h, link_signal(h, kLinkZ, s));
    RQ_TRY(release_side(0));
  }
  if (pending_rows) RQ_CHECK(h, link_wait(h, kLinkU, s));
  return RQ_OK;
}

extern "C" {

rq_status rqrcp_factor(rq_handle h, int64_t m, int64_t n, int64_t k, int64_t b, int64_t p,
                       double* A, int64_t lda, const double* Omega, int64_t ldo, int64_t* jpvt,
                       double* tau, double* T, int64_t ldt, int64_t* info) {
  return rqrcp_core(h, m, n, k, b, p, A, lda, Omega, ldo, 0, false, jpvt, tau, T, ldt, info);
}

rq_status rsrqrcp_factor(rq_handle h, int64_t m, int64_t n, int64_t k, int64_t b, int64_t p,
                         double* A, int64_t lda, const double* Omegas, int64_t ldo,
                         int64_t ostride, int64_t* jpvt, double* tau, double* T, int64_t ldt) {
  if (h && k > 0 && b >= 1 && ldo >= b + p && m > 0 && ostride < ldo * m) return -11;
  rq_status r =
      rqrcp_core(h, m, n, k, b, p, A, lda, Omegas, ldo, ostride, true, jpvt, tau, T, ldt, nullptr);
  if (r <= -11 && r >= -14) r -= 1;   // jpvt, tau, T, ldt come after ostride here
  return r;
}

}  // extern "C"
