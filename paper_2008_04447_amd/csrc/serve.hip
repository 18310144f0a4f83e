// Serving loop: continuous batching of TRQRCP / TUXV requests (see the
// rq_serve_* comment in include/rqrcp.h).  One scheduler thread owns every HIP
// call of the server: it notices completed slots, frees their arena blocks and
// admits queued requests (serve_sched.hpp) onto free slots, each slot being a
// library handle on its own stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "host.hpp"
#include "serve_sched.hpp"

namespace {

using Clock = std::chrono::steady_clock;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

struct Req {
  rq_request r;
  int32_t route = RQ_FP64;     // the arithmetic it runs in
  Clock::time_point t_submit, t_admit;
  rq_result res{};
  size_t off = 0, footprint = 0;
  int slot = -1;
};

// host element size of A
size_t elem_bytes(int32_t prec) { return prec == RQ_FP64 ? 8 : 4; }

// RQ_AUTO requests that run in FP64 hold A twice on the device: as copied in
// (float) and widened to double.
size_t a_bytes(const rq_request& r, int32_t route) {
  const size_t mn = (size_t)r.m * r.n;
  size_t b = rq::Arena::round(mn * elem_bytes(r.prec));
  if (r.prec == RQ_AUTO && route == RQ_FP64) b += rq::Arena::round(mn * 8);
  return b;
}

size_t footprint_of(const rq_request& r, int32_t route) {
  const size_t ell = (size_t)(r.b + r.p);
  size_t b = a_bytes(r, route);
  b += rq::Arena::round(ell * r.m * 8);
  b += rq::Arena::round((size_t)r.n * 8);                  // jpvt
  if (r.op == RQ_OP_TRQRCP)
    b += rq::Arena::round((size_t)r.m * r.k * 8) + rq::Arena::round((size_t)r.k * r.k * 8) +
         rq::Arena::round((size_t)r.k * r.n * 8);
  else
    b += rq::Arena::round((size_t)r.m * r.k * 8) + rq::Arena::round((size_t)r.k * r.k * 8) +
         rq::Arena::round((size_t)r.n * r.k * 8) +
         (r.sigma ? rq::Arena::round((size_t)r.k * 8) : 0);
  return b;
}

double flops_of(const rq_request& r) {
  // sketch + k/b blocks of (Y2^T A, R rows, selected columns, panel) + TUXV extras
  const double m = (double)r.m, n = (double)r.n, k = (double)r.k, ell = (double)(r.b + r.p);
  double f = 2.0 * ell * m * n + 2.0 * k * m * n + 2.0 * k * k * n + 2.0 * m * k * k;
  if (r.op == RQ_OP_TUXV) f += 2.0 * m * n * k + 4.0 * (m + n) * k * k;
  return f;
}

}  // namespace

struct rq_server_s {
  int device = 0;
  int slots = 0;
  int64_t max_m = 0, max_n = 0, max_k = 0, max_ell = 0;
  std::vector<hipStream_t> streams;
  std::vector<rq_handle> handles;
  std::vector<hipEvent_t> done;
  std::vector<int64_t> slot_req;      // request id or -1
  char* arena = nullptr;
  rq::Admitter* adm = nullptr;
  std::mutex mu;
  std::condition_variable cv;        // wakes the scheduler (new work / stop)
  std::condition_variable cv_done;   // wakes waiters
  std::thread th;
  bool stopping = false;
  uint64_t next_id = 1;
  std::unordered_map<uint64_t, Req> reqs;
  int64_t completed = 0;
  size_t peak_bytes = 0;
  int peak_running = 0;
};

namespace {

// Enqueue one admitted request on its slot (scheduler thread, lock held).
rq_status launch(rq_server s, Req& q) {
  const rq_request& r = q.r;
  rq_handle h = s->handles[q.slot];
  hipStream_t st = s->streams[q.slot];
  char* base = s->arena + q.off;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    char* p = base + o;
    o += rq::Arena::round(bytes);
    return p;
  };
  const int64_t ell = r.b + r.p;
  const size_t mn = (size_t)r.m * r.n;
  void* A = take(mn * elem_bytes(r.prec));
  const bool widen = r.prec == RQ_AUTO && q.route == RQ_FP64;
  double* A64 = widen ? reinterpret_cast<double*>(take(mn * 8)) : nullptr;
  double* Om = reinterpret_cast<double*>(take((size_t)ell * r.m * 8));
  int64_t* jp = reinterpret_cast<int64_t*>(take((size_t)r.n * 8));
  double* o0 = reinterpret_cast<double*>(take((size_t)r.m * r.k * 8));
  double* o1 = reinterpret_cast<double*>(take((size_t)r.k * r.k * 8));
  double* o2 = reinterpret_cast<double*>(take((size_t)std::max(r.k * r.n, r.n * r.k) * 8));
  double* sv = (r.op == RQ_OP_TUXV && r.sigma) ? reinterpret_cast<double*>(take((size_t)r.k * 8))
                                               : nullptr;
  RQ_CHECK(h, hipMemcpyAsync(A, r.A, mn * elem_bytes(r.prec), hipMemcpyHostToDevice, st));
  RQ_CHECK(h, hipMemcpyAsync(Om, r.Omega, (size_t)ell * r.m * 8, hipMemcpyHostToDevice, st));
  if (widen) RQ_CHECK(h, rq::launch_cast_f32_f64(static_cast<const float*>(A), A64, (int64_t)mn, st));
  const void* Arun = widen ? A64 : A;
  const rq_prec prun = (rq_prec)q.route;
  rq_status rc;
  if (r.op == RQ_OP_TRQRCP)
    rc = trqrcp_truncate(h, prun, r.m, r.n, r.k, r.b, r.p, Arun, r.m, Om, ell, jp, o0, r.m, o1,
                         r.k, o2, r.k);
  else
    rc = tuxv_svd(h, prun, r.m, r.n, r.k, r.b, r.p, Arun, r.m, Om, ell, o0, r.m, o1, r.k, o2, r.n,
                  jp, sv);
  if (rc != RQ_OK) return rc;
  if (sv) RQ_CHECK(h, hipMemcpyAsync(r.sigma, sv, (size_t)r.k * 8, hipMemcpyDeviceToHost, st));
  if (r.jpvt) RQ_CHECK(h, hipMemcpyAsync(r.jpvt, jp, (size_t)r.n * 8, hipMemcpyDeviceToHost, st));
  if (r.out0) RQ_CHECK(h, hipMemcpyAsync(r.out0, o0, (size_t)r.m * r.k * 8, hipMemcpyDeviceToHost, st));
  if (r.out1) RQ_CHECK(h, hipMemcpyAsync(r.out1, o1, (size_t)r.k * r.k * 8, hipMemcpyDeviceToHost, st));
  if (r.out2) RQ_CHECK(h, hipMemcpyAsync(r.out2, o2, (size_t)r.k * r.n * 8, hipMemcpyDeviceToHost, st));
  RQ_CHECK(h, hipEventRecord(s->done[q.slot], st));
  return RQ_OK;
}

void finish(rq_server s, int slot, Req& q, rq_status st) {
  q.res.state = st == RQ_OK ? RQ_REQ_DONE : RQ_REQ_FAILED;
  q.res.status = st;
  q.res.latency_ms = ms_between(q.t_submit, Clock::now());
  s->adm->finish(q.off, q.footprint);
  s->slot_req[slot] = -1;
  s->completed++;
}

void scheduler(rq_server s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    bool progress = false;
    int running = 0;
    // completions
    for (int i = 0; i < s->slots; ++i) {
      if (s->slot_req[i] < 0) continue;
      hipError_t e = hipEventQuery(s->done[i]);
      if (e == hipErrorNotReady) {
        ++running;
        continue;
      }
      Req& q = s->reqs[(uint64_t)s->slot_req[i]];
      int64_t derr = 0;
      rq_status st = (e == hipSuccess) ? rq_sync_status(s->handles[i], &derr) : RQ_E_HIP;
      q.res.device_error = derr;
      finish(s, i, q, st);
      progress = true;
    }
    // admissions, in arrival order
    std::vector<int> free_slots;
    for (int i = 0; i < s->slots; ++i)
      if (s->slot_req[i] < 0) free_slots.push_back(i);
    auto adm = s->adm->admit((int)free_slots.size());
    for (size_t a = 0; a < adm.size(); ++a) {
      Req& q = s->reqs[adm[a].id];
      q.off = adm[a].offset;
      q.slot = free_slots[a];
      q.t_admit = Clock::now();
      q.res.queue_ms = ms_between(q.t_submit, q.t_admit);
      q.res.state = RQ_REQ_RUNNING;
      s->slot_req[q.slot] = (int64_t)adm[a].id;
      rq_status st = launch(s, q);
      if (st != RQ_OK) {
        (void)hipStreamSynchronize(s->streams[q.slot]);
        finish(s, q.slot, q, st);
      } else {
        ++running;
      }
      progress = true;
    }
    s->peak_bytes = std::max(s->peak_bytes, s->adm->used());
    s->peak_running = std::max(s->peak_running, running);
    if (progress) s->cv_done.notify_all();
    if (s->stopping && running == 0 && s->adm->queued() == 0) break;
    if (!progress) s->cv.wait_for(lk, std::chrono::microseconds(running ? 20 : 2000));
  }
  s->cv_done.notify_all();
}

}  // namespace

using namespace rq;

extern "C" {

int32_t rq_serve_route(int32_t prec, int64_t m, int64_t n, int64_t k, double tol) {
  if (prec == RQ_FP64 || prec == RQ_MIXED_BF16) return prec;
  if (prec != RQ_AUTO || !(tol > 0.0) || !(tol < HUGE_VAL) || m < 1 || n < 1 || k < 1) return -1;
  // BF16 rounding noise of A seen through k of min(m, n) directions
  const double floor_bf16 = 1.5 * std::ldexp(1.0, -9) * std::sqrt((double)k / (double)std::min(m, n));
  return floor_bf16 <= 0.3 * tol ? RQ_MIXED_BF16 : RQ_FP64;
}

rq_status rq_serve_start(int device, size_t budget_bytes, int32_t slots, int64_t max_m,
                         int64_t max_n, int64_t max_k, int64_t max_ell, rq_server* out) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return -1;
  if (budget_bytes < 4096) return -2;
  if (slots < 1 || slots > 16) return -3;
  if (max_m < 1) return -4;
  if (max_n < 1 || max_n > RQ_MAX_N) return -5;
  if (max_k < 1 || max_k > std::min(max_m, max_n)) return -6;
  if (max_ell < 1 || max_ell > RQ_MAX_ELL) return -7;
  if (!out) return -8;
  // persistent kernels of all slots must be able to be resident together
  const int cap = 192 / slots;
  if (sq_groups(max_n, cap) > cap || (std::max(max_m, max_n) + kPanelRows - 1) / kPanelRows > cap)
    return RQ_E_UNSUPPORTED;
  DeviceGuard guard(device);
  rq_server s = new rq_server_s();
  s->device = device;
  s->slots = slots;
  s->max_m = max_m;
  s->max_n = max_n;
  s->max_k = max_k;
  s->max_ell = max_ell;
  rq_status st = RQ_OK;
  const size_t ws = truncated_workspace_bytes(max_m, max_n, max_k, (int)max_ell, true);
  for (int i = 0; i < slots && st == RQ_OK; ++i) {
    hipStream_t str = nullptr;
    hipEvent_t ev = nullptr;
    if (hipStreamCreateWithFlags(&str, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      st = RQ_E_HIP;
      break;
    }
    s->streams.push_back(str);
    s->done.push_back(ev);
    rq_handle h = nullptr;
    st = rq_create(&h, device, str);
    if (st != RQ_OK) break;
    h->max_groups = cap;
    h->update_wgs = cap;
    s->handles.push_back(h);
    st = reserve(h, ws);
  }
  if (st == RQ_OK && hipMalloc(reinterpret_cast<void**>(&s->arena), budget_bytes) != hipSuccess)
    st = RQ_E_NOMEM;
  if (st != RQ_OK) {
    for (rq_handle h : s->handles) rq_destroy(h);
    for (hipEvent_t e : s->done) (void)hipEventDestroy(e);
    for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
    if (s->arena) (void)hipFree(s->arena);
    delete s;
    return st;
  }
  s->adm = new Admitter(budget_bytes);
  s->slot_req.assign(slots, -1);
  s->th = std::thread(scheduler, s);
  *out = s;
  return RQ_OK;
}

rq_status rq_serve_submit(rq_server s, const rq_request* r, uint64_t* id) {
  if (!s) return -1;
  if (!r || (r->op != RQ_OP_TRQRCP && r->op != RQ_OP_TUXV) ||
      rq_serve_route(r->prec, r->m, r->n, r->k, r->tol) < 0 || r->m < 1 || r->n < 1 || r->k < 1 ||
      r->k > std::min(r->m, r->n) || r->b < 1 || r->b > RQ_MAX_B || r->p < 0 ||
      r->b + r->p > RQ_MAX_ELL || r->b + r->p > r->m || !r->A || !r->Omega)
    return -2;
  if (!id) return -3;
  if (r->m > s->max_m || r->n > s->max_n || r->k > s->max_k || r->b + r->p > s->max_ell)
    return RQ_E_UNSUPPORTED;
  if (r->op == RQ_OP_TUXV && r->sigma && r->k > RQ_MAX_SVD) return RQ_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stopping) return RQ_E_UNSUPPORTED;
  const uint64_t nid = s->next_id++;
  Req q;
  q.r = *r;
  q.route = rq_serve_route(r->prec, r->m, r->n, r->k, r->tol);
  q.t_submit = Clock::now();
  q.footprint = footprint_of(*r, q.route);
  q.res.state = RQ_REQ_QUEUED;
  q.res.prec_used = q.route;
  q.res.flops = flops_of(*r);
  if (!s->adm->enqueue(nid, q.footprint)) return RQ_E_UNSUPPORTED;
  s->reqs.emplace(nid, q);
  *id = nid;
  s->cv.notify_one();
  return RQ_OK;
}

rq_status rq_serve_poll(rq_server s, uint64_t id, rq_result* res) {
  if (!s) return -1;
  if (!res) return -3;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return -2;
  *res = it->second.res;
  return RQ_OK;
}

rq_status rq_serve_wait(rq_server s, uint64_t id, rq_result* res) {
  if (!s) return -1;
  if (!res) return -3;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return -2;
  s->cv_done.wait(lk, [&] {
    const int32_t st = s->reqs[id].res.state;
    return st == RQ_REQ_DONE || st == RQ_REQ_FAILED;
  });
  *res = s->reqs[id].res;
  return RQ_OK;
}

rq_status rq_serve_stats(rq_server s, int64_t* completed, int64_t* peak_bytes,
                         int32_t* peak_running) {
  if (!s) return -1;
  std::lock_guard<std::mutex> lk(s->mu);
  if (completed) *completed = s->completed;
  if (peak_bytes) *peak_bytes = (int64_t)s->peak_bytes;
  if (peak_running) *peak_running = s->peak_running;
  return RQ_OK;
}

rq_status rq_serve_stop(rq_server s) {
  if (!s) return -1;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stopping = true;
    s->cv.notify_one();
  }
  if (s->th.joinable()) s->th.join();
  DeviceGuard guard(s->device);
  for (rq_handle h : s->handles) rq_destroy(h);
  for (hipEvent_t e : s->done) (void)hipEventDestroy(e);
  for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
  if (s->arena) (void)hipFree(s->arena);
  delete s->adm;
  delete s;
  return RQ_OK;
}

}  // extern "C"
