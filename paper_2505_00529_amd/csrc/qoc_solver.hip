// Trust-region solver and batched multi-problem evaluation (filled in below the core path).
#include <hip/hip_runtime.h>

#include "../../include/qoc.h"
#include "qoc_api_internal.h"

extern "C" {

qoc_status qoc_tr_solve(qoc_problem* p, const double* theta0, double gtol, int32_t max_iter, double* theta_out,
                        double* cost_out, int32_t* iters_out) {
  (void)theta0; (void)gtol; (void)max_iter; (void)theta_out; (void)cost_out; (void)iters_out;
  if (!p) return QOC_ERR_INVALID_ARG;
  return p->fail(QOC_ERR_UNSUPPORTED, "not built yet");
}

qoc_status qoc_batch_create(int device, int32_t count, qoc_problem* const* problems, qoc_batch** out) {
  (void)device; (void)count; (void)problems; (void)out;
  return QOC_ERR_UNSUPPORTED;
}
void qoc_batch_destroy(qoc_batch* b) { (void)b; }
qoc_status qoc_batch_hess(qoc_batch* b, const double* const* thetas, double* const* costs, double* const* grads,
                          double* const* hessians) {
  (void)b; (void)thetas; (void)costs; (void)grads; (void)hessians;
  return QOC_ERR_UNSUPPORTED;
}
qoc_status qoc_batch_hess_unbatched(qoc_batch* b, const double* const* thetas, double* const* costs,
                                    double* const* grads, double* const* hessians) {
  (void)b; (void)thetas; (void)costs; (void)grads; (void)hessians;
  return QOC_ERR_UNSUPPORTED;
}
const char* qoc_batch_last_error(const qoc_batch* b) { (void)b; return "not built yet"; }

}  // extern "C"
