// C-ABI of the vmlbm library: context, workspace carving, stepping in the
// order of Algorithm 1, and synchronous read-back for tests.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "vmlbm.h"
#include "common.hpp"
#include "uniform.hpp"
#include "context.hpp"

using namespace vm;

namespace vm {

// Scratch for callers that cannot allocate (vmlbm_totals_static): the
// per-workgroup partial sums of the totals reduction live in this
// file-scope device array instead of the context's workspace.  In host code
// its name is not a device address; each device's copy is looked up once,
// with that device current, when a workspace is bound on it (scratch_on).
constexpr int kStaticScratchDoubles = kTotalsGroups * 8;
static __device__ __align__(256) double scratch[kStaticScratchDoubles];

constexpr int kMaxDevices = 64;
static double* g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

// this device's copy of the scratch array (the current device)
static hipError_t scratch_on(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double*)p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

int fail(vmlbm_ctx* c, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

size_t storage_bytes(int storage) { return storage == VMLBM_F64 ? 8 : storage == VMLBM_F32 ? 4 : 2; }

// IEEE binary16 bits of v, rounded once to nearest with ties to even
// (subnormals kept, overflow to infinity); the scalings by powers of two are
// exact, so std::nearbyint in the default rounding mode does the rounding
uint16_t half_bits_rne(double v) {
  const uint16_t sgn = std::signbit(v) ? 0x8000u : 0u;
  const double a = std::fabs(v);
  if (std::isnan(v)) return 0x7e00u;
  if (a < std::ldexp(1.0, -14)) {                       // subnormal or zero: multiples of 2^-24
    const double k = std::nearbyint(std::ldexp(a, 24));  // 1024 rounds up to the smallest normal
    return (uint16_t)(sgn | (uint16_t)k);
  }
  int e = 0;
  std::frexp(a, &e);                                    // a = m 2^e, m in [0.5, 1)
  int E = e - 1;                                        // a in [2^E, 2^(E+1))
  double r = std::nearbyint(std::ldexp(a, 10 - E));     // in [1024, 2048]
  if (r == 2048.0) { r = 1024.0; E += 1; }
  if (E > 15) return (uint16_t)(sgn | 0x7c00u);
  return (uint16_t)(sgn | (uint16_t)((E + 15) << 10) | (uint16_t)(r - 1024.0));
}

}  // namespace vm

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// uniform-grid workspace layout
void plan_uniform(vmlbm_ctx* c) {
  const vmlbm_config& g = c->cfg;
  const size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
  const size_t S = storage_bytes(g.storage);
  const int np = (int)c->spheres.size();
  int box = 0;
  for (const auto& s : c->spheres) box = std::max(box, (int)std::ceil(2.0 * s.radius) + 7);
  c->box = box;
  // one force slot per workgroup of the link-cell pass of a sphere: with
  // moving spheres the pass scans each sphere's box (no link lists to
  // rebuild after every re-mapping), with fixed ones it reads the lists
  c->slot_stride = (size_t)(c->moving ? link_chunks(box) : kLinkGroups) * kSlotWords;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
  c->off_status = take(kStatusWords * sizeof(int));
  c->off_pdf[0] = take(19 * N * S);
  c->off_pdf[1] = take(19 * N * S);
  c->off_flags = take(N);
  c->off_owner = take(2 * N);
  c->off_parts = take(std::max(np, 1) * sizeof(DevParticle));
  c->off_slots = take(std::max<size_t>(np * c->slot_stride, 1) * sizeof(double));
  c->off_hist = take((size_t)std::max(g.history, 1) * std::max(np, 1) * kHistWords * sizeof(double));
  c->off_totals = take((size_t)kTotalsGroups * 8 * sizeof(double));
  c->off_lcount = take((size_t)std::max(np, 1) * link_chunks(box) * sizeof(int));
  c->off_links = take((size_t)std::max(np, 1) * box * box * box * sizeof(uint32_t));
  c->off_llen = take((size_t)std::max(np, 1) * sizeof(int));
  adjoint_plan(c, take);
  c->ws_needed = off;
}

double dev_to_double(const void* buf, int storage, size_t i) {
  if (storage == VMLBM_F64) return ((const double*)buf)[i];
  if (storage == VMLBM_F32) return (double)((const float*)buf)[i];
  return (double)__half2float(((const __half*)buf)[i]);
}

void double_to_dev(void* buf, int storage, size_t i, double v) {
  if (storage == VMLBM_F64) ((double*)buf)[i] = v;
  else if (storage == VMLBM_F32) ((float*)buf)[i] = (float)v;
  else ((uint16_t*)buf)[i] = half_bits_rne(v);
}

int check_ready(vmlbm_ctx* c) {
  if (!c) return VMLBM_EINVAL;
  if (!c->ws) return fail(c, VMLBM_ESTATE, "workspace not bound");
  if (!c->initialized) return fail(c, VMLBM_ESTATE, "vmlbm_init_equilibrium not called");
  return VMLBM_OK;
}

int read_status(vmlbm_ctx* c) {
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  int st[kStatusWords];
  HIP_TRY(c, hipMemcpy(st, c->ws + c->off_status, sizeof(st), hipMemcpyDeviceToHost));
  if (st[kStatusUnstable]) return fail(c, VMLBM_EUNSTABLE, "non-finite state flagged (code %d)", st[kStatusUnstable]);
  if (st[kStatusRange]) return fail(c, VMLBM_ERANGE, "particle geometry out of range (code %d)", st[kStatusRange]);
  return VMLBM_OK;
}

void fold_timing(vmlbm_ctx* c) {
  for (auto& ev : c->sweep_events) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ev.first, ev.second) == hipSuccess) c->sweep_seconds += ms * 1e-3;
    c->sweep_launches += 1;
    (void)hipEventDestroy(ev.first);
    (void)hipEventDestroy(ev.second);
  }
  c->sweep_events.clear();
  if (c->step_pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, c->ev_start, c->ev_end) == hipSuccess) c->seconds += ms * 1e-3;
    c->step_pending = false;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// uniform-grid stepping (Algorithm 1): sweep (LBM step + link forces) ->
// reduction, averaging, virtual-mass update -> refill -> re-mapping
// ---------------------------------------------------------------------------
namespace vm {

SweepParams sweep_params(const vmlbm_ctx* c) {
  const vmlbm_config& g = c->cfg;
  SweepParams p{};
  p.nx = g.n[0]; p.ny = g.n[1]; p.nz = g.n[2];
  for (int a = 0; a < 3; ++a) p.per[a] = g.periodic[a];
  p.wall_axis = c->wall_axis;
  for (int s = 0; s < 2; ++s)
    for (int a = 0; a < 3; ++a) p.wall_v[s][a] = g.wall_velocity[s][a];
  p.sp = c->sp;
  p.sm = c->sm;
  p.sb = c->sb;
  for (int a = 0; a < 3; ++a) p.F[a] = c->F[a];
  p.N = (uint32_t)((size_t)g.n[0] * g.n[1] * g.n[2]);
  const PopLayout lay = pop_layout(g.storage, g.n);
  p.sq = lay.sq;
  p.sz = lay.sz;
  p.box = c->box;
  p.slot_stride = c->slot_stride;
  return p;
}

UpdateParams update_params(const vmlbm_ctx* c, long long step) {
  UpdateParams u{};
  for (int a = 0; a < 3; ++a) u.g[a] = c->cfg.gravity[a];
  u.hist_len = std::max(c->cfg.history, 1);
  u.step = (int)(step % u.hist_len);
  u.np = (int)c->spheres.size();
  return u;
}

// one sweep src -> dst: boundary cells on the side stream, concurrently with
// the interior sweep; joined back into the main stream.  With `up`, the
// force/torque reduction and particle update follow the boundary cells on
// the side stream (they read the link pass's slots and the particle
// records, which the interior sweep does not touch), so they too run
// beside the interior sweep.
int sweep_once(vmlbm_ctx* c, const SweepParams& p, void* src, void* dst, hipEvent_t e0, hipEvent_t e1,
               const UpdateParams* up) {
  const int np = (int)c->spheres.size();
  const bool flags = c->use_flags;
  if (flags) {
    HIP_TRY(c, hipEventRecord(c->ev_fork, c->stream));
    HIP_TRY(c, hipStreamWaitEvent(c->side, c->ev_fork, 0));
  }
  int rc = dispatch(c->cfg.storage, [&](auto* tag) -> int {
    using S = std::remove_pointer_t<decltype(tag)>;
    if (flags) {
      HIP_TRY(c, launch_boundary<S>(src, dst, c->flags(), c->owner(), c->parts(), np, c->links(), c->slots(),
                                    c->status(), p, c->side, c->moving));
      if (up && np > 0)
        HIP_TRY(c, launch_reduce_update(c->parts(), np, c->slots(), c->hist(), c->status(), p, *up, c->side));
    }
    HIP_TRY(c, launch_interior<S>(src, dst, c->flags(), c->status(), p, flags, c->stream, e0, e1));
    return VMLBM_OK;
  });
  if (rc) return rc;
  if (flags) {
    HIP_TRY(c, hipEventRecord(c->ev_join, c->side));
    HIP_TRY(c, hipStreamWaitEvent(c->stream, c->ev_join, 0));
  }
  return VMLBM_OK;
}

int uniform_step(vmlbm_ctx* c, int nsteps) {
  SweepParams p = sweep_params(c);
  const int np = (int)c->spheres.size();
  for (int s = 0; s < nsteps; ++s) {
    p.seed = step_seed(c->steps_done);
    void* src = c->ws + c->off_pdf[c->cur];
    void* dst = c->ws + c->off_pdf[1 - c->cur];
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->profile) {
      HIP_TRY(c, hipEventCreate(&e0));
      HIP_TRY(c, hipEventCreate(&e1));
      c->sweep_events.emplace_back(e0, e1);
    }
    const UpdateParams up = update_params(c, c->steps_done);
    int rc = sweep_once(c, p, src, dst, e0, e1, &up);
    if (rc) return rc;
    if (np > 0) {
      if (c->moving) {
        rc = dispatch(c->cfg.storage, [&](auto* tag) -> int {
          using S = std::remove_pointer_t<decltype(tag)>;
          HIP_TRY(c, launch_refill_remap<S>(dst, c->flags(), c->owner(), c->parts(), np, c->links(), p, c->status(),
                                            c->stream, true));
          return VMLBM_OK;
        });
        if (rc) return rc;
      }
    }
    c->cur = 1 - c->cur;
    c->steps_done += 1;
    c->cell_updates += (double)p.N;
  }
  return VMLBM_OK;
}

}  // namespace vm

// ---------------------------------------------------------------------------
// C API
// ---------------------------------------------------------------------------
extern "C" {

int vmlbm_create(const vmlbm_config* cfg, vmlbm_ctx** out) {
  if (!cfg || !out) return VMLBM_EINVAL;
  *out = nullptr;
  for (int a = 0; a < 3; ++a)
    if (cfg->n[a] <= 0) return VMLBM_EINVAL;
  if (cfg->storage < VMLBM_F64 || cfg->storage > VMLBM_F16) return VMLBM_EINVAL;
  if (!(cfg->omega > 0.0 && cfg->omega < 2.0) || !(cfg->magic > 0.0)) return VMLBM_EINVAL;
  if (cfg->block < 0) return VMLBM_EINVAL;
  if (cfg->block == 0) {
    const double N = (double)cfg->n[0] * cfg->n[1] * cfg->n[2];
    if (N >= 2147483648.0) return VMLBM_ERANGE;
  }
  auto* c = new (std::nothrow) vmlbm_ctx();
  if (!c) return VMLBM_ENOMEM;
  c->cfg = *cfg;
  if (c->cfg.history < 1) c->cfg.history = 1;
  c->wall_axis = -1;
  for (int a = 0; a < 3; ++a)
    if (!cfg->periodic[a]) { c->wall_axis = a; break; }
  c->sp = cfg->omega;
  c->sm = s_minus_of(c->sp, cfg->magic);
  c->sb = s_bulk_of(c->sp, cfg->bulk_factor);
  for (int a = 0; a < 3; ++a) c->F[a] = cfg->body_force[a];
  if (cfg->block > 0) {
    int rc = refine_create(c);
    if (rc) { delete c; return rc; }
  }
  *out = c;
  return VMLBM_OK;
}

int vmlbm_add_sphere(vmlbm_ctx* c, const vmlbm_sphere* s, int* id) {
  if (!c || !s) return VMLBM_EINVAL;
  if (c->ws) return fail(c, VMLBM_ESTATE, "spheres must be added before the workspace is bound");
  if (!(s->radius > 0.0) || !(s->density_ratio > 0.0) || s->cv < 0.0 || s->cv_omega < 0.0 || s->fixed < 0 ||
      s->fixed > 2 || s->vm_scheme < 0 || s->vm_scheme > 2)
    return fail(c, VMLBM_EINVAL, "bad sphere parameters");
  if (c->spheres.size() >= 65535) return fail(c, VMLBM_ERANGE, "too many spheres");
  const int box = (int)std::ceil(2.0 * s->radius) + 8;
  const int* n = c->cfg.n;
  const int scale = c->cfg.block > 0 ? (1 << (c->cfg.levels - 1)) : 1;
  for (int a = 0; a < 3; ++a)
    if (box > n[a] * scale) return fail(c, VMLBM_ERANGE, "sphere larger than the domain");
  for (const auto& o : c->spheres) {
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      double d = s->x[a] - o.x[a];
      const double L = (double)n[a] * scale;
      if (c->cfg.periodic[a]) d -= L * std::round(d / L);
      d2 += d * d;
    }
    if (std::sqrt(d2) < s->radius + o.radius + 3.0)
      return fail(c, VMLBM_ERANGE, "spheres closer than 3 cells");
  }
  c->spheres.push_back(*s);
  if (s->fixed == 0) c->moving = true;
  if (id) *id = (int)c->spheres.size() - 1;
  return VMLBM_OK;
}

int vmlbm_required_bytes(const vmlbm_ctx* cc, size_t* bytes) {
  auto* c = const_cast<vmlbm_ctx*>(cc);
  if (!c || !bytes) return VMLBM_EINVAL;
  if (c->cfg.block > 0) {
    int rc = refine_plan(c);
    if (rc) return rc;
  } else {
    plan_uniform(c);
  }
  *bytes = c->ws_needed;
  return VMLBM_OK;
}

int vmlbm_bind_workspace(vmlbm_ctx* c, void* dev_ptr, size_t bytes) {
  if (!c || !dev_ptr) return VMLBM_EINVAL;
  if (((uintptr_t)dev_ptr) & 255) return fail(c, VMLBM_EINVAL, "workspace must be 256-byte aligned");
  size_t need = 0;
  int rc = vmlbm_required_bytes(c, &need);
  if (rc) return rc;
  if (bytes < need) return fail(c, VMLBM_ENOMEM, "workspace %zu < required %zu bytes", bytes, need);
  c->ws = (char*)dev_ptr;
  c->ws_bytes = bytes;
  HIP_TRY(c, scratch_on(&c->scratch));
  c->use_flags = !c->spheres.empty() || c->wall_axis >= 0;
  if (!c->side) {
    HIP_TRY(c, hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    HIP_TRY(c, hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming));
    HIP_TRY(c, hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming));
  }
  return VMLBM_OK;
}

int vmlbm_set_stream(vmlbm_ctx* c, void* stream) {
  if (!c) return VMLBM_EINVAL;
  c->stream = (hipStream_t)stream;
  return VMLBM_OK;
}

int vmlbm_init_equilibrium(vmlbm_ctx* c, double rho, const double* u0) {
  if (!c) return VMLBM_EINVAL;
  if (!c->ws) return fail(c, VMLBM_ESTATE, "workspace not bound");
  if (c->cfg.block > 0) return refine_init(c, rho, u0);
  SweepParams p0 = sweep_params(c);
  p0.seed = kInitSeed;
  const int np = (int)c->spheres.size();
  HIP_TRY(c, hipMemsetAsync(c->status(), 0, kStatusWords * sizeof(int), c->stream));
  // particle records
  std::vector<DevParticle> hp(np);
  for (int i = 0; i < np; ++i) {
    const vmlbm_sphere& s = c->spheres[i];
    DevParticle& P = hp[i];
    memset(&P, 0, sizeof(P));
    for (int a = 0; a < 3; ++a) {
      P.x[a] = s.x[a];
      P.xold[a] = s.x[a];
      P.u[a] = s.fixed ? 0.0 : s.u[a];
      P.w[a] = s.fixed == 1 ? 0.0 : s.w[a];
    }
    P.r = s.radius; P.rho = s.density_ratio; P.cv = s.cv; P.cvw = s.cv_omega;
    P.fixed = s.fixed; P.have_prev = 0;
    P.scheme = s.vm_scheme; P.nvel = 1;
    for (int a = 0; a < 3; ++a) {
      int lo = (int)std::floor(s.x[a] - s.radius) - 3;
      if (c->cfg.periodic[a]) lo = ((lo % c->cfg.n[a]) + c->cfg.n[a]) % c->cfg.n[a];
      P.box_lo[a] = lo;
      P.remap_lo[a] = lo;
    }
  }
  if (np) HIP_TRY(c, hipMemcpyAsync(c->parts(), hp.data(), np * sizeof(DevParticle), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->hist(), 0, (size_t)c->cfg.history * std::max(np, 1) * kHistWords * sizeof(double), c->stream));
  if (c->use_flags)
    HIP_TRY(c, launch_map_all(c->flags(), c->owner(), c->parts(), np, c->links(), p0, c->status(), c->stream));
  double* u0d = nullptr;
  if (u0) {
    u0d = (double*)(c->ws + c->off_pdf[1]);   // staging in the second population buffer
    HIP_TRY(c, hipMemcpyAsync(u0d, u0, 3 * (size_t)p0.N * sizeof(double), hipMemcpyHostToDevice, c->stream));
  }
  int rc = dispatch(c->cfg.storage, [&](auto* tag) -> int {
    using S = std::remove_pointer_t<decltype(tag)>;
    HIP_TRY(c, launch_init<S>(c->ws + c->off_pdf[0], c->use_flags ? c->flags() : nullptr, u0d, rho - 1.0, p0,
                              c->stream));
    return VMLBM_OK;
  });
  if (rc) return rc;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->cur = 0;
  c->steps_done = 0;
  c->initialized = true;
  return VMLBM_OK;
}

int vmlbm_step(vmlbm_ctx* c, int n) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (n < 0) return fail(c, VMLBM_EINVAL, "negative step count");
  if (n == 0) return VMLBM_OK;
  if (!c->step_pending) {
    if (!c->ev_start) { HIP_TRY(c, hipEventCreate(&c->ev_start)); HIP_TRY(c, hipEventCreate(&c->ev_end)); }
    HIP_TRY(c, hipEventRecord(c->ev_start, c->stream));
  }
  rc = c->cfg.block > 0 ? refine_step(c, n) : uniform_step(c, n);
  if (rc) return rc;
  HIP_TRY(c, hipEventRecord(c->ev_end, c->stream));
  c->step_pending = true;
  return VMLBM_OK;
}

int vmlbm_sync(vmlbm_ctx* c) {
  if (!c) return VMLBM_EINVAL;
  if (!c->ws) return fail(c, VMLBM_ESTATE, "workspace not bound");
  int rc = read_status(c);
  fold_timing(c);
  return rc;
}

int vmlbm_get_particle(vmlbm_ctx* c, int id, double x[3], double u[3], double w[3]) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (id < 0 || id >= (int)c->spheres.size()) return fail(c, VMLBM_EINVAL, "bad sphere id");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  DevParticle P;
  HIP_TRY(c, hipMemcpy(&P, c->parts() + id, sizeof(P), hipMemcpyDeviceToHost));
  for (int a = 0; a < 3; ++a) {
    if (x) x[a] = P.x[a];
    if (u) u[a] = P.u[a];
    if (w) w[a] = P.w[a];
  }
  return VMLBM_OK;
}

int vmlbm_set_sphere_motion(vmlbm_ctx* c, int id, const double u[3], const double w[3], int fixed) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (id < 0 || id >= (int)c->spheres.size() || fixed < 0 || fixed > 2)
    return fail(c, VMLBM_EINVAL, "bad sphere id or mode");
  if (fixed == 0 && !c->moving)
    return fail(c, VMLBM_EINVAL, "a sphere can move freely only if one was added free");
  if ((fixed == 0 && !u) || (fixed != 1 && !w)) return fail(c, VMLBM_EINVAL, "velocity missing");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  DevParticle P;
  HIP_TRY(c, hipMemcpy(&P, c->parts() + id, sizeof(P), hipMemcpyDeviceToHost));
  P.fixed = fixed;
  for (int a = 0; a < 3; ++a) {
    P.u[a] = fixed ? 0.0 : u[a];
    P.w[a] = fixed == 1 ? 0.0 : w[a];
  }
  HIP_TRY(c, hipMemcpy(c->parts() + id, &P, sizeof(P), hipMemcpyHostToDevice));
  c->spheres[id].fixed = fixed;
  return VMLBM_OK;
}

int vmlbm_get_force_torque(vmlbm_ctx* c, int id, double F[3], double T[3]) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (id < 0 || id >= (int)c->spheres.size()) return fail(c, VMLBM_EINVAL, "bad sphere id");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  DevParticle P;
  HIP_TRY(c, hipMemcpy(&P, c->parts() + id, sizeof(P), hipMemcpyDeviceToHost));
  for (int a = 0; a < 3; ++a) {
    if (F) F[a] = P.F[a];
    if (T) T[a] = P.T[a];
  }
  return VMLBM_OK;
}

int vmlbm_get_history(vmlbm_ctx* c, int id, int n, double* out) {
  int rc = check_ready(c);
  if (rc) return rc;
  const int np = (int)c->spheres.size();
  const int H = c->cfg.history;
  if (id < 0 || id >= np || !out) return fail(c, VMLBM_EINVAL, "bad argument");
  const long long done = c->particle_steps();
  if (n < 0 || n > H || n > done) return fail(c, VMLBM_EINVAL, "history holds %d of %lld steps", H, done);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  std::vector<double> h((size_t)H * np * kHistWords);
  HIP_TRY(c, hipMemcpy(h.data(), c->hist(), h.size() * sizeof(double), hipMemcpyDeviceToHost));
  for (int i = 0; i < n; ++i) {
    const long long step = done - n + i;
    const double* src = h.data() + ((size_t)(step % H) * np + id) * kHistWords;
    memcpy(out + kHistWords * i, src, kHistWords * sizeof(double));
  }
  return VMLBM_OK;
}

int vmlbm_read_populations(vmlbm_ctx* c, int level, double* out) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!out) return VMLBM_EINVAL;
  if (c->cfg.block > 0) return refine_read_populations(c, level, out);
  if (level != 0) return fail(c, VMLBM_EINVAL, "uniform grid has level 0 only");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const size_t N = (size_t)c->cfg.n[0] * c->cfg.n[1] * c->cfg.n[2];
  const size_t S = storage_bytes(c->cfg.storage);
  std::vector<char> raw(19 * N * S);
  HIP_TRY(c, hipMemcpy(raw.data(), c->ws + c->off_pdf[c->cur], raw.size(), hipMemcpyDeviceToHost));
  std::vector<uint8_t> fl(N, 0);
  if (c->use_flags) HIP_TRY(c, hipMemcpy(fl.data(), c->flags(), N, hipMemcpyDeviceToHost));
  const PopLayout lay = pop_layout(c->cfg.storage, c->cfg.n);
  for (int q = 0; q < 19; ++q)
    for (size_t i = 0; i < N; ++i)
      out[q * N + i] =
          (fl[i] & kSolid) ? 0.0 : w_of(q) + dev_to_double(raw.data(), c->cfg.storage, lay.pop(q, (uint32_t)i));
  return VMLBM_OK;
}

int vmlbm_write_populations(vmlbm_ctx* c, int level, const double* in) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!in) return VMLBM_EINVAL;
  if (c->cfg.block > 0) return refine_write_populations(c, level, in);
  if (level != 0) return fail(c, VMLBM_EINVAL, "uniform grid has level 0 only");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const size_t N = (size_t)c->cfg.n[0] * c->cfg.n[1] * c->cfg.n[2];
  const size_t S = storage_bytes(c->cfg.storage);
  std::vector<char> raw(19 * N * S);
  const PopLayout lay = pop_layout(c->cfg.storage, c->cfg.n);
  for (int q = 0; q < 19; ++q)
    for (size_t i = 0; i < N; ++i)
      double_to_dev(raw.data(), c->cfg.storage, lay.pop(q, (uint32_t)i), in[q * N + i] - w_of(q));
  HIP_TRY(c, hipMemcpy(c->ws + c->off_pdf[c->cur], raw.data(), raw.size(), hipMemcpyHostToDevice));
  return VMLBM_OK;
}

int vmlbm_read_owner(vmlbm_ctx* c, int level, int* out) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!out) return VMLBM_EINVAL;
  if (c->cfg.block > 0) return refine_read_owner(c, level, out);
  if (level != 0) return fail(c, VMLBM_EINVAL, "uniform grid has level 0 only");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const size_t N = (size_t)c->cfg.n[0] * c->cfg.n[1] * c->cfg.n[2];
  std::vector<uint8_t> fl(N, 0);
  std::vector<uint16_t> ow(N, 0);
  if (c->use_flags) {
    HIP_TRY(c, hipMemcpy(fl.data(), c->flags(), N, hipMemcpyDeviceToHost));
    HIP_TRY(c, hipMemcpy(ow.data(), c->owner(), 2 * N, hipMemcpyDeviceToHost));
  }
  for (size_t i = 0; i < N; ++i) out[i] = (fl[i] & kSolid) ? (int)ow[i] : -1;
  return VMLBM_OK;
}

int vmlbm_read_fields(vmlbm_ctx* c, int level, double* rho, double* u) {
  int rc = check_ready(c);
  if (rc) return rc;
  size_t N = 0;
  if (c->cfg.block > 0) {
    rc = refine_level_cells(c, level, &N);
    if (rc) return rc;
  } else {
    if (level != 0) return fail(c, VMLBM_EINVAL, "uniform grid has level 0 only");
    N = (size_t)c->cfg.n[0] * c->cfg.n[1] * c->cfg.n[2];
  }
  std::vector<double> f(19 * N);
  rc = vmlbm_read_populations(c, level, f.data());
  if (rc) return rc;
  double Fl[3];
  level_force(c, level, Fl);
  for (size_t i = 0; i < N; ++i) {
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < 19; ++q) {
      const double v = f[q * N + i];
      r += v; j[0] += cx_of(q) * v; j[1] += cy_of(q) * v; j[2] += cz_of(q) * v;
    }
    const bool fluid = r != 0.0;
    if (rho) rho[i] = r;
    // post-collision momentum minus F/2 is the macroscopic velocity
    if (u)
      for (int a = 0; a < 3; ++a) u[a * N + i] = fluid ? j[a] - 0.5 * Fl[a] : 0.0;
  }
  return VMLBM_OK;
}

int vmlbm_stats(vmlbm_ctx* c, double* cell_updates, double* seconds) {
  if (!c) return VMLBM_EINVAL;
  if (c->ws) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    fold_timing(c);
  }
  if (cell_updates) *cell_updates = c->cell_updates;
  if (seconds) *seconds = c->seconds;
  return VMLBM_OK;
}

int vmlbm_profile(vmlbm_ctx* c, int enable) {
  if (!c) return VMLBM_EINVAL;
  c->profile = enable != 0;
  return VMLBM_OK;
}

int vmlbm_sweep_time(vmlbm_ctx* c, double* seconds, long long* launches) {
  if (!c) return VMLBM_EINVAL;
  if (c->ws) {
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    fold_timing(c);
  }
  if (seconds) *seconds = c->sweep_seconds;
  if (launches) *launches = c->sweep_launches;
  return VMLBM_OK;
}

int vmlbm_stream_copy(void* dst, const void* src, size_t bytes, void* stream) {
  if (!dst || !src || bytes % 16) return VMLBM_EINVAL;
  if (bytes / 16 > (size_t)UINT32_MAX * 256) return VMLBM_ERANGE;
  return launch_stream_copy(dst, src, bytes, (hipStream_t)stream) == hipSuccess ? VMLBM_OK : VMLBM_EDEVICE;
}

int vmlbm_stream_pull(void* dst, const void* src, int storage, const int n[3], void* stream) {
  if (!dst || !src || !n || storage < VMLBM_F64 || storage > VMLBM_F16) return VMLBM_EINVAL;
  if (n[0] < 1 || n[1] < 1 || n[2] < 1 || n[1] > 65535 || n[2] > 65535) return VMLBM_ERANGE;
  return launch_stream_pull(dst, src, storage, n, (hipStream_t)stream) == hipSuccess ? VMLBM_OK : VMLBM_EDEVICE;
}

int vmlbm_cell_counts(vmlbm_ctx* c, int level, long long* fluid, long long* interior) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (c->cfg.block > 0) return refine_cell_counts(c, level, fluid, interior);
  if (level != 0) return fail(c, VMLBM_EINVAL, "uniform grid has level 0 only");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const size_t N = (size_t)c->cfg.n[0] * c->cfg.n[1] * c->cfg.n[2];
  long long nf = (long long)N, ni = (long long)N;
  if (c->use_flags) {
    std::vector<uint8_t> fl(N);
    HIP_TRY(c, hipMemcpy(fl.data(), c->flags(), N, hipMemcpyDeviceToHost));
    nf = ni = 0;
    for (size_t i = 0; i < N; ++i) {
      nf += !(fl[i] & kSolid);
      ni += fl[i] == 0;
    }
  }
  if (fluid) *fluid = nf;
  if (interior) *interior = ni;
  return VMLBM_OK;
}

// totals with device partials `part` and a host buffer `h`, both of
// kTotalsGroups x 8 doubles
static int totals_with(vmlbm_ctx* c, double* part, double* h, double* mass, double mom[3]) {
  if (c->cfg.block > 0) return refine_totals(c, part, h, mass, mom);
  const uint32_t N = (uint32_t)((size_t)c->cfg.n[0] * c->cfg.n[1] * c->cfg.n[2]);
  HIP_TRY(c, launch_totals(c->cfg.storage, c->ws + c->off_pdf[c->cur], c->use_flags ? c->flags() : nullptr,
                           pop_layout(c->cfg.storage, c->cfg.n), N, nullptr, 0, part, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  HIP_TRY(c, hipMemcpy(h, part, (size_t)kTotalsGroups * 8 * sizeof(double), hipMemcpyDeviceToHost));
  long double n = 0, m = 0, j[3] = {0, 0, 0};
  for (int g = 0; g < kTotalsGroups; ++g) {
    n += h[8 * g]; m += h[8 * g + 1];
    for (int a = 0; a < 3; ++a) j[a] += h[8 * g + 2 + a];
  }
  if (mass) *mass = (double)(n + m);
  if (mom) for (int a = 0; a < 3; ++a) mom[a] = (double)j[a];
  return VMLBM_OK;
}

int vmlbm_totals(vmlbm_ctx* c, double* mass, double mom[3]) {
  int rc = check_ready(c);
  if (rc) return rc;
  std::vector<double> h((size_t)kTotalsGroups * 8);
  return totals_with(c, (double*)(c->ws + c->off_totals), h.data(), mass, mom);
}

int vmlbm_totals_static(vmlbm_ctx* c, double* mass, double mom[3]) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!c->scratch) return fail(c, VMLBM_ESTATE, "no scratch array on this device");
  // the partials come back into a stack buffer: no heap use on this path
  double h[kStaticScratchDoubles];
  return totals_with(c, c->scratch, h, mass, mom);
}

int vmlbm_read_box(vmlbm_ctx* c, const int lo[3], const int size[3], double* out) {
  int rc = check_ready(c);
  if (rc) return rc;
  if (!lo || !size || !out) return VMLBM_EINVAL;
  if (c->cfg.block > 0) return fail(c, VMLBM_EINVAL, "box read-back is for the uniform grid");
  const int* n = c->cfg.n;
  for (int a = 0; a < 3; ++a)
    if (size[a] <= 0 || size[a] > n[a]) return fail(c, VMLBM_EINVAL, "bad box size");
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const PopLayout lay = pop_layout(c->cfg.storage, n);
  const size_t S = storage_bytes(c->cfg.storage);
  const char* base = c->ws + c->off_pdf[c->cur];
  std::vector<char> row((size_t)size[0] * S);
  std::vector<uint8_t> frow(size[0], 0);
  const size_t cells = (size_t)size[0] * size[1] * size[2];
  for (int q = 0; q < 19; ++q)
    for (int k = 0; k < size[2]; ++k)
      for (int j = 0; j < size[1]; ++j) {
        const int z = ((lo[2] + k) % n[2] + n[2]) % n[2], y = ((lo[1] + j) % n[1] + n[1]) % n[1];
        const int x0 = ((lo[0] % n[0]) + n[0]) % n[0];
        const int first = std::min(size[0], n[0] - x0);
        const size_t r = ((size_t)z * n[1] + y) * n[0];
        const size_t pr = lay.pop(q, (uint32_t)r);   // population q of the row's first cell
        HIP_TRY(c, hipMemcpy(row.data(), base + (pr + x0) * S, first * S, hipMemcpyDeviceToHost));
        if (first < size[0])
          HIP_TRY(c, hipMemcpy(row.data() + first * S, base + pr * S, (size[0] - first) * S,
                               hipMemcpyDeviceToHost));
        if (q == 0 && c->use_flags) {
          HIP_TRY(c, hipMemcpy(frow.data(), c->flags() + r + x0, first, hipMemcpyDeviceToHost));
          if (first < size[0]) HIP_TRY(c, hipMemcpy(frow.data() + first, c->flags() + r, size[0] - first,
                                                    hipMemcpyDeviceToHost));
        }
        for (int i = 0; i < size[0]; ++i) {
          const size_t o = (size_t)q * cells + ((size_t)k * size[1] + j) * size[0] + i;
          out[o] = w_of(q) + dev_to_double(row.data(), c->cfg.storage, i);
        }
        if (q == 0)
          for (int i = 0; i < size[0]; ++i)
            if (frow[i] & kSolid) out[((size_t)k * size[1] + j) * size[0] + i] = -1.0;
      }
  // solid cells: all 19 read 0 (marked through q = 0 above)
  for (size_t cc = 0; cc < cells; ++cc)
    if (out[cc] == -1.0)
      for (int q = 0; q < 19; ++q) out[q * cells + cc] = 0.0;
  return VMLBM_OK;
}

int vmlbm_destroy(vmlbm_ctx* c) {
  if (!c) return VMLBM_EINVAL;
  if (c->ws) (void)hipStreamSynchronize(c->stream);
  fold_timing(c);
  if (c->ev_start) (void)hipEventDestroy(c->ev_start);
  if (c->ev_end) (void)hipEventDestroy(c->ev_end);
  if (c->side) (void)hipStreamSynchronize(c->side);
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  if (c->side) (void)hipStreamDestroy(c->side);
  refine_destroy(c);
  delete c;
  return VMLBM_OK;
}

const char* vmlbm_last_error(const vmlbm_ctx* c) { return c ? c->err.c_str() : "null context"; }

}  // extern "C"
