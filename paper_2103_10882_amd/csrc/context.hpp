// Host-side context of the vmlbm library.
#pragma once

#include <hip/hip_runtime.h>
#include <functional>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "vmlbm.h"
#include "common.hpp"
#include "uniform.hpp"

namespace vm {
struct Forest;     // block-structured grid state (refine.hip)
struct AdjState;   // adjoint bookkeeping (adjoint.hip)
}

struct vmlbm_ctx {
  vmlbm_config cfg{};
  std::vector<vmlbm_sphere> spheres;
  bool moving = false;
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;              // boundary kernels, forked from and joined to `stream`
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  char* ws = nullptr;
  double* scratch = nullptr;   // this device's file-scope scratch array (api.hip), set at binding
  size_t ws_bytes = 0;
  size_t ws_needed = 0;
  bool initialized = false;
  bool use_flags = false;
  int wall_axis = -1;
  double sp = 0.0, sm = 0.0, sb = 0.0, F[3] = {0.0, 0.0, 0.0};
  std::string err;

  // uniform-grid workspace carving
  size_t off_status = 0, off_pdf[2] = {0, 0}, off_flags = 0, off_owner = 0, off_parts = 0, off_slots = 0,
         off_hist = 0, off_totals = 0, off_lcount = 0, off_links = 0, off_llen = 0;
  int cur = 0;
  int box = 0;
  size_t slot_stride = 0;

  // progress and timing
  long long steps_done = 0;          // steps of the uniform grid / coarse steps
  long long fine_steps_done = 0;     // finest-level steps (refined grid)
  double cell_updates = 0.0;
  double seconds = 0.0;
  hipEvent_t ev_start = nullptr, ev_end = nullptr;
  bool step_pending = false;
  bool profile = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> sweep_events;
  double sweep_seconds = 0.0;
  long long sweep_launches = 0;

  std::unique_ptr<vm::Forest, void (*)(vm::Forest*)> forest{nullptr, nullptr};
  std::unique_ptr<vm::AdjState, void (*)(vm::AdjState*)> adj{nullptr, nullptr};

  int* status() { return (int*)(ws + off_status); }
  uint8_t* flags() { return (uint8_t*)(ws + off_flags); }
  uint16_t* owner() { return (uint16_t*)(ws + off_owner); }
  vm::DevParticle* parts() { return (vm::DevParticle*)(ws + off_parts); }
  double* slots() { return (double*)(ws + off_slots); }
  double* hist() { return (double*)(ws + off_hist); }
  vm::LinkLists links() { return {(int*)(ws + off_lcount), (uint32_t*)(ws + off_links), (int*)(ws + off_llen)}; }
  long long particle_steps() const { return cfg.block > 0 ? fine_steps_done : steps_done; }
};

namespace vm {
using Take = std::function<size_t(size_t)>;

// Seeds of the stochastic-rounding streams: the sweep that produces state
// n+1 from state n uses step_seed(n) (a recomputation from a checkpoint
// reproduces the forward states bit for bit); level l of the refined grid
// uses level_seed(finest steps done, l); initial states and data migrated
// between levels use their own streams.
inline uint32_t step_seed(long long n) { return (uint32_t)n; }
inline uint32_t level_seed(long long fine_steps, int l) { return (uint32_t)(fine_steps * 16 + l); }
constexpr uint32_t kInitSeed = 0xa511e9b3u;
constexpr uint32_t kMigrateSeed = 0x63d83595u;

int fail(vmlbm_ctx* c, int code, const char* fmt, ...);
#define HIP_TRY(ctx, expr)                                                                           \
  do {                                                                                               \
    hipError_t e_ = (expr);                                                                          \
    if (e_ != hipSuccess) return vm::fail(ctx, VMLBM_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// run f with a null pointer of the storage type
template <typename F>
int dispatch(int storage, F&& f) {
  if (storage == VMLBM_F64) return f((double*)nullptr);
  if (storage == VMLBM_F32) return f((float*)nullptr);
  return f((__half*)nullptr);
}

struct SweepParams;
SweepParams sweep_params(const vmlbm_ctx* c);
int sweep_once(vmlbm_ctx* c, const SweepParams& p, void* src, void* dst, hipEvent_t e0, hipEvent_t e1,
               const UpdateParams* up = nullptr);
// particle-update parameters of finest step / uniform step `step`
UpdateParams update_params(const vmlbm_ctx* c, long long step);
size_t storage_bytes(int storage);
// host conversion to IEEE binary16 bits, round to nearest even (api.hip)
uint16_t half_bits_rne(double v);

int uniform_step(vmlbm_ctx* c, int nsteps);

// deterministic sums over cells: kTotalsGroups workgroup partials of
// (fluid cells, sum d, sum c d) per call
constexpr int kTotalsGroups = 1024;
// (lay: the uniform grid's population layout; unused with a slot list)
hipError_t launch_totals(int storage, const void* pdf, const uint8_t* flags, const PopLayout& lay, uint32_t cells,
                         const int* slot_list, int nslots, double* partials, hipStream_t st);
int refine_totals(vmlbm_ctx* c, double* part, double* h, double* mass, double mom[3]);

// adjoint (adjoint.hip)
void adjoint_plan(vmlbm_ctx* c, const Take& take);

// block-structured refined grid (refine.hip)
int refine_create(vmlbm_ctx* c);
int refine_plan(vmlbm_ctx* c);
int refine_init(vmlbm_ctx* c, double rho, const double* u0);
int refine_step(vmlbm_ctx* c, int n);
int refine_read_populations(vmlbm_ctx* c, int level, double* out);
int refine_write_populations(vmlbm_ctx* c, int level, const double* in);
int refine_read_owner(vmlbm_ctx* c, int level, int* out);
int refine_level_cells(vmlbm_ctx* c, int level, size_t* cells);
int refine_cell_counts(vmlbm_ctx* c, int level, long long* fluid, long long* interior);
void refine_destroy(vmlbm_ctx* c);
int refine_add_region(vmlbm_ctx* c, const int lo[3], const int hi[3], int level);
// body force of a level in that level's lattice units
void level_force(const vmlbm_ctx* c, int level, double F[3]);
}  // namespace vm
