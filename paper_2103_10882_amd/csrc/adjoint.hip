// Adjoint of the fixed-sphere drag: not built yet.
#include "context.hpp"

namespace vm {
struct AdjState {};
void adjoint_plan(vmlbm_ctx*, const Take&) {}
}  // namespace vm

extern "C" {
int vmlbm_set_params(vmlbm_ctx* c, double, double) {
  if (!c) return VMLBM_EINVAL;
  return VMLBM_ESTATE;
}
int vmlbm_forward_ckpt(vmlbm_ctx* c, int, int, int, int, double*) {
  if (!c) return VMLBM_EINVAL;
  return VMLBM_ESTATE;
}
int vmlbm_adjoint(vmlbm_ctx* c, double, double*) {
  if (!c) return VMLBM_EINVAL;
  return VMLBM_ESTATE;
}
}
