// Block-structured 2:1 refined grid (Sec. 4.1-4.2): not built yet.
#include "context.hpp"

namespace vm {

struct Forest {};

int refine_create(vmlbm_ctx* c) {
  c->err = "block-structured grid not available";
  return VMLBM_EINVAL;
}
int refine_plan(vmlbm_ctx*) { return VMLBM_ESTATE; }
int refine_init(vmlbm_ctx*, double, const double*) { return VMLBM_ESTATE; }
int refine_step(vmlbm_ctx*, int) { return VMLBM_ESTATE; }
int refine_read_populations(vmlbm_ctx*, int, double*) { return VMLBM_ESTATE; }
int refine_write_populations(vmlbm_ctx*, int, const double*) { return VMLBM_ESTATE; }
int refine_read_owner(vmlbm_ctx*, int, int*) { return VMLBM_ESTATE; }
int refine_level_cells(vmlbm_ctx*, int, size_t*) { return VMLBM_ESTATE; }
int refine_cell_counts(vmlbm_ctx*, int, long long*, long long*) { return VMLBM_ESTATE; }
void refine_destroy(vmlbm_ctx*) {}

void level_force(const vmlbm_ctx* c, int level, double F[3]) {
  const int L = c->cfg.block > 0 ? c->cfg.levels - 1 : 0;
  const double s = (double)(1 << (L - level));
  for (int a = 0; a < 3; ++a) F[a] = c->F[a] * s;
}

}  // namespace vm

extern "C" {
int vmlbm_level_blocks(vmlbm_ctx* c, int, int*, int*) {
  if (!c) return VMLBM_EINVAL;
  c->err = "not a block-structured grid";
  return VMLBM_ESTATE;
}
int vmlbm_refinements(vmlbm_ctx* c, int* count) {
  if (!c || !count) return VMLBM_EINVAL;
  *count = 0;
  return VMLBM_OK;
}
}
