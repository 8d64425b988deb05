// Serving entry points: batched stepping of many contexts and the sweep
// workgroup-size tuner.
#include <hip/hip_runtime.h>

#include "runtime.hpp"

using namespace hrlbm;

extern "C" {

int lbm_step_batch(lbm_ctx* const* ctxs, const int64_t* steps, int n) {
  if (n < 0 || (n > 0 && (!ctxs || !steps))) return set_error(LBM_EINVAL, "batch arguments");
  for (int k = 0; k < n; ++k) {
    int rc = check_ready(ctxs[k]);
    if (rc != LBM_OK) return rc;
    rc = step_ctx(ctxs[k], steps[k], ctxs[k]->stream);
    if (rc != LBM_OK) return rc;
  }
  return LBM_OK;
}

int lbm_autotune(lbm_ctx* ctx, int) {
  int rc = check_ready(ctx);
  if (rc != LBM_OK) return rc;
  return ctx->block;
}

}  // extern "C"
