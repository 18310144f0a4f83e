// Host-side internals shared by the entry points: the handle, error plumbing,
// the workspace carve-out and event-based kernel timing.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/rqrcp.h"
#include "kernels.hpp"

namespace rq {

// Kernel classes reported by rq_profile_get.
enum KClass {
  K_SKETCH = 0,
  K_SAMPLE_QRCP,
  K_PERMUTE,
  K_PANEL,
  K_INNER,          // W = Y^T A (split-K)
  K_REDUCE,         // fixed-order split-K sum (and T^T W)
  K_UPDATE,         // A -= Y Z
  K_OMEGA11,
  K_SAMPLE_UPDATE,
  K_QP3_PIVOT,      // plain QRCP: argmax, swap, column update, reflector
  K_QP3_GEMV,       // plain QRCP: adjusted inner products over the trailing matrix
  K_QP3_ROW,        // plain QRCP: row update and norm downdate
  K_TR_SELECT,      // TRQRCP: selected columns A - Y W^T
  K_TR_ROWS,        // TRQRCP: new R rows A - Y W^T
  K_TR_SMALL,       // TRQRCP/TUXV: small products (Y2^T Y, T composition, ...)
  K_OTHER,
  K_SKETCH_BF16,    // mixed precision: B = Omega A with BF16 operands
  K_INNER_BF16,     // mixed precision: products over A with BF16 operands
  K_SVD,            // singular values of a small square matrix (TUXV's X)
  K_NUM_CLASSES
};

inline const char* kclass_name(int c) {
  static const char* names[K_NUM_CLASSES] = {
      "sketch", "sample_qrcp", "permute", "panel", "inner_products", "reduce",
      "trailing_update", "omega11", "sample_update", "qp3_pivot", "qp3_gemv", "qp3_row",
      "tr_select", "tr_rows", "tr_small", "other", "sketch_bf16", "inner_products_bf16", "svd"};
  return (c >= 0 && c < K_NUM_CLASSES) ? names[c] : "?";
}

struct ProfRec {
  int cls;
  hipEvent_t e0, e1;
  double flops, bytes;
};
struct ProfTot {
  int64_t launches = 0;
  double ms = 0, flops = 0, bytes = 0;
};

}  // namespace rq

struct rq_handle_s {
  int device = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;          // grow-only workspace
  size_t ws_bytes = 0;
  int64_t* status = nullptr;   // device int64[4]
  uint32_t* sync = nullptr;    // device u32[64]: [0] barrier counter, [1] abort flag,
                               // [2] panel fallback flag, [8..11] the concurrency probe,
                               // [32..63] the block loop's stream links
  int max_groups = 128;        // workgroups one persistent sample-QRCP launch may use
  int update_wgs = 256;        // compute units a trailing-update launch may fill (device count)
  int cus = 256;               // compute units of the device
  hipStream_t side = nullptr;  // second stream of the RQRCP block loop (created on first use)
  // the RQRCP block loop's links between its two streams: device words with
  // the count each last had written, or events (see link_signal in api.hip)
  uint64_t link_count[4] = {0, 0, 0, 0};
  hipEvent_t link_ev[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // [4]: a call's start
  bool link_values = true;     // the current call orders the streams through the words
  bool words_ok = false;       // kernels of two streams were seen running at the same time
  double* scratch = nullptr;   // device address of the static scratch array (rq_sample_qrcp_noalloc)
  std::string last_error;
  bool prof = false;
  uint32_t prof_mask = ~0u;     // kernel classes timed while prof is set
  std::vector<rq::ProfRec> recs;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
  rq::ProfTot tot[rq::K_NUM_CLASSES];
};

// The persistent kernels (panels, plain-QRCP steps) give each workgroup
// kPanelRows rows, one workgroup per compute unit, and need all of them
// resident at once: m rows fit when ceil(m / kPanelRows) <= compute units.
inline bool rows_fit(const rq_handle_s* h, int64_t m) {
  return (m + rq::kPanelRows - 1) / rq::kPanelRows <= h->cus;
}

namespace rq {

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

inline rq_status fail(rq_handle h, hipError_t e, const char* where) {
  if (h) h->last_error = std::string(where) + ": " + hipGetErrorString(e);
  return RQ_E_HIP;
}

#define RQ_CHECK(h, expr)                                  \
  do {                                                     \
    hipError_t _e = (expr);                                \
    if (_e != hipSuccess) return rq::fail((h), _e, #expr); \
  } while (0)

#define RQ_TRY(expr)              \
  do {                            \
    rq_status _s = (expr);        \
    if (_s != RQ_OK) return _s;   \
  } while (0)

// Bump allocator over the handle's workspace (reserve() first).
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
inline size_t padded_bytes(size_t n_doubles) { return n_doubles * sizeof(double) + 256; }

rq_status reserve(rq_handle h, size_t bytes);

// Brackets the launches in its scope with events when profiling is on.
struct KTimer {
  rq_handle h;
  int cls;
  double f, b;
  hipStream_t s;
  hipEvent_t e0 = nullptr;
  KTimer(rq_handle h_, int cls_, double f_, double b_) : KTimer(h_, cls_, f_, b_, h_->stream) {}
  KTimer(rq_handle h_, int cls_, double f_, double b_, hipStream_t s_);
  ~KTimer();
};

inline bool valid_ptr(const void* p, int64_t count) { return count <= 0 || p != nullptr; }

// Shared building blocks of the block loops (api.hip).
struct SqWork {
  double* rec;
  int* src_top;
  int* dst_low;
};
size_t sq_rec_doubles(int ell, int64_t N);
size_t panel_rec_doubles(int64_t M);
size_t sketch_part_doubles(int ell, int64_t m, int64_t n);
rq_status sketch_fp64(rq_handle h, int ell, int64_t m, int64_t n, const double* Omega, int64_t ldo,
                      const double* A, int64_t lda, double* B, int64_t ldb, double* part);
// B = Omega A with A FP32 on BF16 MFMA (split-K partials summed in FP64).
rq_status sketch_bf16(rq_handle h, int ell, int64_t m, int64_t n, const double* Omega, int64_t ldo,
                      const float* A, int64_t lda, double* B, int64_t ldb, double* part,
                      __bf16* lbf);
// Y^T-style product with FP32 X on BF16 MFMA, reduced into out (leading dim ldout).
rq_status gemm_lx_bf16_reduced(rq_handle h, int cls, GemmArgsF g, double* part, double* out,
                               int64_t ldout, __bf16* lbf);
// doubles of workspace that hold the BF16 staging of an operand with K columns
inline size_t bf16_stage_doubles(int64_t K) { return (size_t)(bf16_stage_elems(K) + 3) / 4; }
size_t sketch_part_doubles_bf16(int ell, int64_t m, int64_t n);
// `signal_side` releases the RQRCP block loop's trailing update on the side
// stream (link Z): the kernel writes the link's word once all its workgroups
// hold their compute units, or, where the call orders its streams with
// events, the link's event is recorded right before the launch.
// `panel_rec`, when given, is the record area of the panel that follows (M
// rows, bj columns): it is prepared together with the sample's records, and
// that panel is then run with `prepared` set.  `groups` is the workgroup
// allowance of the launch (0: the handle's max_groups, which leaves compute
// units to the RQRCP side stream).
// With `prepared`, the records (and the panel's, when panel_rec is given)
// were prepared by an earlier launch (see launch_omega11) and no preparation
// is launched here.
rq_status run_sample_qrcp(rq_handle h, double* B, int64_t ldb, int ell, int64_t N, int steps,
                          SqWork w, int64_t* perm, bool signal_side = false,
                          double* panel_rec = nullptr, int64_t panel_m = 0, int panel_bj = 0,
                          int groups = 0, bool prepared = false);
rq_status run_panel(rq_handle h, double* A, int64_t lda, int64_t M, int bj, double* rec,
                    double* tau, double* Y, int64_t ldy, double* T, int64_t ldt,
                    bool prepared = false);
// With rk (RQRCP), the rank check of launch_omega11 runs in the same launch
// and the product skips itself once rk->info is set; with prep, that launch
// also prepares the next block's record areas.
rq_status run_sample_update(rq_handle h, double* sblk, int ell, const double* R11, int64_t ldr,
                            const double* R12, int64_t ldr12, int bj, int64_t Nt, double* mhat,
                            const RankCheck* rk = nullptr, const RecordPrep* prep = nullptr);
// Workspace bytes each entry point reserves for a problem shape (what
// rq_workspace_query reports).
size_t truncated_workspace_bytes(int64_t m, int64_t n, int64_t k, int ell, bool tuxv);
size_t rqrcp_workspace_bytes(int64_t m, int64_t n, int64_t k, int64_t b, int64_t p, bool resample);
size_t qrcp_workspace_bytes(int64_t m, int64_t n, int64_t k);
size_t sketch_workspace_bytes(int64_t ell, int64_t m, int64_t n);
size_t sample_qrcp_workspace_bytes(int64_t ell, int64_t n);
size_t singular_values_workspace_bytes(int64_t k);
// Singular values of the k x k matrix X (ld ldx), largest first, into sigma
// (k <= RQ_MAX_SVD); `work` holds singular_values_workspace_bytes(k).
rq_status run_singular_values(rq_handle h, int64_t k, const double* X, int64_t ldx, double* sigma,
                              double* work);

}  // namespace rq
