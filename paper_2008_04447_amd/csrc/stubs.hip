// Entry points whose GPU paths are not part of this build yet: they validate
// nothing and report RQ_E_UNSUPPORTED so callers fail loudly.
#include "host.hpp"

extern "C" {

rq_status qrcp_factor(rq_handle h, int64_t, int64_t, int64_t, int64_t, double*, int64_t, int64_t*,
                      double*) {
  return h ? RQ_E_UNSUPPORTED : -1;
}

rq_status trqrcp_truncate(rq_handle h, rq_prec, int64_t, int64_t, int64_t, int64_t, int64_t,
                          const void*, int64_t, const double*, int64_t, int64_t*, double*, int64_t,
                          double*, int64_t, double*, int64_t) {
  return h ? RQ_E_UNSUPPORTED : -1;
}

rq_status tuxv_svd(rq_handle h, rq_prec, int64_t, int64_t, int64_t, int64_t, int64_t, const void*,
                   int64_t, const double*, int64_t, double*, int64_t, double*, int64_t, double*,
                   int64_t, int64_t*) {
  return h ? RQ_E_UNSUPPORTED : -1;
}

}  // extern "C"
