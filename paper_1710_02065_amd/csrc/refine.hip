// Two-level 2:1 grid refinement (Sec. II.B).
#include <hip/hip_runtime.h>

#include "runtime.hpp"

lbm_ctx::~lbm_ctx() { hrlbm::free_refinement(this); }

namespace hrlbm {

struct Refinement {};

int validate_refinement(const lbm_config&) {
  return set_error(LBM_EUNSUPPORTED, "grid refinement is not built yet");
}
int make_fine_level(lbm_ctx*) { return set_error(LBM_EUNSUPPORTED, "grid refinement is not built yet"); }
size_t plan_interface_layout(lbm_ctx*, size_t off) { return off; }
void assign_interface_pointers(lbm_ctx*) {}
int refined_after_init(lbm_ctx*) { return LBM_OK; }
int refined_after_set(lbm_ctx*, int) { return LBM_OK; }
int refined_coarse_step(lbm_ctx*, hipStream_t) {
  return set_error(LBM_EUNSUPPORTED, "grid refinement is not built yet");
}
void free_refinement(lbm_ctx* ctx) {
  delete ctx->ref;
  ctx->ref = nullptr;
}

}  // namespace hrlbm
