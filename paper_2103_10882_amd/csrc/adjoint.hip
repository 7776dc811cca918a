// Discrete adjoint of the fixed-sphere drag (uniform periodic grid).
//
// Forward map (post-collision states s_n, fixed spheres, v_b = 0):
//   s_{n+1} = C_theta(P(s_n)),   F^n = G(s_n)   (Eqs. 10-12),
// with P the pull with CLI links (linear, parameter free), C_theta the TRT
// collision with Guo forcing, theta = (F_z, omega) and Lambda fixed, and
//   J = 1/W sum_{n=A}^{N-1} F_z^n.
// Reverse recursion: lambda_N = 0,
//   lambda_n = P^T [ J_C(P(s_n))^T lambda_{n+1} + w_n e ] + w_n g_direct,
//   dJ/dtheta = sum_n lambda_{n+1} . dC/dtheta (P(s_n)) + lambda_0 . dC/dtheta (w),
// where e and g_direct are the derivatives of the link-force sum with respect
// to the incoming and the post-collision populations, w_n = 1/W inside the
// averaging window.  States inside a segment are recomputed from checkpoints.
//
// P^T is applied as a push: the cell that pulled population r from y writes
// lambda(y, r).  Each location is written by exactly one thread, except the
// CLI term -kappa0 lambda(x, r) for links whose cell x + c_r is fluid, which a
// small fix-up kernel adds after the main kernels.
#include <cmath>
#include <vector>

#include "common.hpp"
#include "uniform.hpp"
#include "stencil.hpp"
#include "particle.hpp"
#include "context.hpp"

namespace vm {

template <typename S> struct Lam { using L = float; };
template <> struct Lam<double> { using L = double; };

struct AdjState {
  int n_steps = 0, avg_from = 0, ckpt_every = 0, sphere = 0;
  bool have_forward = false;
  double F[3] = {0.0, 0.0, 0.0}, sp = 0.0;   // parameters the checkpoints were taken with
  size_t off_ckpt = 0, off_seg = 0, off_lam[2] = {0, 0}, off_g = 0;
  size_t state_bytes = 0, lam_bytes = 0;
  int n_ckpt = 0;
  int interior_groups = 0, boundary_waves = 0;
};

namespace {

// nu = J_C(d)^T lam and the parameter derivatives lam . dC/dF_z, lam . dC/domega
// of the TRT collision on deviations d (same formulas as lbm_collide with s_b = s+).
template <typename T>
__device__ __forceinline__ void collide_adjoint(const T (&d)[kQ], const T (&lam)[kQ], T sp, T sm, T Fx, T Fy,
                                                T Fz, double dsm_dw, T (&nu)[kQ], double& gF, double& gW) {
  T drho = d[0];
#pragma unroll
  for (int q = 1; q < kQ; ++q) drho += d[q];
  const T jx = (d[1] - d[2]) + (d[7] - d[10]) + (d[8] - d[9]) + (d[11] - d[14]) + (d[12] - d[13]);
  const T jy = (d[3] - d[4]) + (d[7] - d[10]) + (d[9] - d[8]) + (d[15] - d[18]) + (d[16] - d[17]);
  const T jz = (d[5] - d[6]) + (d[11] - d[14]) + (d[13] - d[12]) + (d[15] - d[18]) + (d[17] - d[16]);
  const T ux = jx + T(0.5) * Fx, uy = jy + T(0.5) * Fy, uz = jz + T(0.5) * Fz;
  const T usq = ux * ux + uy * uy + uz * uz;
  const T uF = ux * Fx + uy * Fy + uz * Fz;
  const T kp = T(1) - T(0.5) * sp, km = T(1) - T(0.5) * sm;
  T A, Bx, By, Bz;
  double gsp, gsm, gfz;
  {
    const T w = T(w_of(0));
    const T l = lam[0];
    const T ep = w * (drho - T(1.5) * usq);
    const T Sp = w * (T(-3) * uF);
    A = l * sp * w;
    Bx = l * (sp * w * (T(-3) * ux) + kp * w * (T(-3) * Fx));
    By = l * (sp * w * (T(-3) * uy) + kp * w * (T(-3) * Fy));
    Bz = l * (sp * w * (T(-3) * uz) + kp * w * (T(-3) * Fz));
    gsp = (double)(l * (-(d[0] - ep) - T(0.5) * Sp));
    gsm = 0.0;
    gfz = (double)(l * kp * w * (T(-3) * uz));
  }
#pragma unroll
  for (int k = 0; k < kPairs; ++k) {
    const int q = pair_q(k), qb = opp_of(q);
    const T cxq = T(cx_of(q)), cyq = T(cy_of(q)), czq = T(cz_of(q));
    const T w = T(w_of(q));
    const T cu = cxq * ux + cyq * uy + czq * uz;
    const T cF = cxq * Fx + cyq * Fy + czq * Fz;
    const T ep = w * (drho + T(4.5) * cu * cu - T(1.5) * usq);
    const T em = T(3) * w * cu;
    const T Sp = w * (T(9) * cu * cF - T(3) * uF);
    const T Sm = T(3) * w * cF;
    const T fp = T(0.5) * (d[q] + d[qb]);
    const T fm = T(0.5) * (d[q] - d[qb]);
    const T lp = lam[q] + lam[qb];
    const T lm = lam[q] - lam[qb];
    A += lp * sp * w;
    // even equilibrium and even forcing depend on u; odd equilibrium too
    const T ce = lp * sp * w * T(9) * cu + lp * kp * w * T(9) * cF + lm * sm * T(3) * w;
    Bx += ce * cxq - lp * (sp * w * T(3) * ux + kp * w * T(3) * Fx);
    By += ce * cyq - lp * (sp * w * T(3) * uy + kp * w * T(3) * Fy);
    Bz += ce * czq - lp * (sp * w * T(3) * uz + kp * w * T(3) * Fz);
    gsp += (double)(lp * (-(fp - ep) - T(0.5) * Sp));
    gsm += (double)(lm * (-(fm - em) - T(0.5) * Sm));
    gfz += (double)(lp * kp * w * (T(9) * cu * czq - T(3) * uz) + lm * km * T(3) * w * czq);
  }
  nu[0] = lam[0] - sp * lam[0] + A;
#pragma unroll
  for (int k = 0; k < kPairs; ++k) {
    const int q = pair_q(k), qb = opp_of(q);
    const T cB = T(cx_of(q)) * Bx + T(cy_of(q)) * By + T(cz_of(q)) * Bz;
    const T lp = T(0.5) * (lam[q] + lam[qb]), lm = T(0.5) * (lam[q] - lam[qb]);
    const T even = lp - sp * lp + A;
    const T odd = lm - sm * lm + cB;
    nu[q] = even + odd;
    nu[qb] = even - odd;
  }
  gF = gfz + 0.5 * (double)Bz;
  gW = gsp + dsm_dw * gsm;
}

template <typename L, typename T, int... Qs>
__device__ __forceinline__ void push_all(L* __restrict__ lout, uint32_t N, const Idx& I, int x, const T (&nu)[kQ],
                                         std::integer_sequence<int, Qs...>) {
  ((lout[(size_t)Qs * N + pull_index<Qs>(I, x)] = L(nu[Qs])), ...);
}

// workgroup sum of two doubles added to slot g (fixed order)
__device__ __forceinline__ void group_accumulate(double a, double b, double* __restrict__ slots, size_t g) {
  __shared__ double red[2][16];
  a = wave_sum(a);
  b = wave_sum(b);
  const int wave = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  if ((threadIdx.x & 63) == 0) { red[0][wave] = a; red[1][wave] = b; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int i = 0; i < nw; ++i) { sa += red[0][i]; sb += red[1][i]; }
    slots[2 * g] += sa;
    slots[2 * g + 1] += sb;
  }
}

template <typename S>
__global__ __launch_bounds__(512) void k_adj_interior(const S* __restrict__ s, const typename Lam<S>::L* __restrict__ lin,
                                                      typename Lam<S>::L* __restrict__ lout,
                                                      const uint8_t* __restrict__ flags, double* __restrict__ gslots,
                                                      SweepParams p, double dsm_dw) {
  using T = typename Store<S>::T;
  using L = typename Lam<S>::L;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y, z = blockIdx.z;
  const uint32_t N = p.N;
  const uint32_t c = ((uint32_t)z * p.ny + y) * p.nx + x;
  double gF = 0.0, gW = 0.0;
  if (x < p.nx && flags[c] == 0) {
    T d[kQ], lam[kQ], nu[kQ];
    // the state in its population layout, the adjoint fields [q][z][y][x]
    const Idx Is = make_idx(x, y, z, p.nx, p.ny, p.nz, p.sz);
    const Idx I = make_idx(x, y, z, p.nx, p.ny, p.nz, (size_t)p.nx * p.ny);
    load_all<S>(s, p.sq, Is, x, d, std::make_integer_sequence<int, kQ>{});
#pragma unroll
    for (int q = 0; q < kQ; ++q) lam[q] = T(lin[(size_t)q * N + c]);
    collide_adjoint<T>(d, lam, T(p.sp), T(p.sm), T(p.F[0]), T(p.F[1]), T(p.F[2]), dsm_dw, nu, gF, gW);
    // push: the pull of direction q at this cell read (x - c_q, q)
    push_all<L, T>(lout, N, I, x, nu, std::make_integer_sequence<int, kQ>{});
  }
  const size_t g = blockIdx.x + (size_t)gridDim.x * (blockIdx.y + (size_t)gridDim.y * blockIdx.z);
  group_accumulate(gF, gW, gslots, g);
}

__device__ __forceinline__ uint32_t wrap_index(int x, int y, int z, const SweepParams& p) {
  x = x < 0 ? x + p.nx : (x >= p.nx ? x - p.nx : x);
  y = y < 0 ? y + p.ny : (y >= p.ny ? y - p.ny : y);
  z = z < 0 ? z + p.nz : (z >= p.nz ? z - p.nz : z);
  return ((uint32_t)z * p.ny + y) * p.nx + x;
}

// Cells with particle links, in the box pass of the sphere they link to.
// FIXUP = false: main adjoint for these cells; FIXUP = true: the -kappa0 term
// on locations (x, r) with x - c_r solid and x + c_r fluid.
template <typename S, bool FIXUP>
__global__ __launch_bounds__(256) void k_adj_boundary(const S* __restrict__ s, const typename Lam<S>::L* __restrict__ lin,
                                                      typename Lam<S>::L* __restrict__ lout,
                                                      const uint8_t* __restrict__ flags,
                                                      const uint16_t* __restrict__ owner,
                                                      const DevParticle* __restrict__ parts,
                                                      double* __restrict__ gslots, int* __restrict__ status,
                                                      SweepParams p, double dsm_dw, double wn, size_t slot0) {
  using T = typename Store<S>::T;
  using L = typename Lam<S>::L;
  const int pi = blockIdx.y;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int edge = p.box;
  const uint32_t N = p.N;
  int x = 0, y = 0, z = 0;
  bool active = false;
  if (k < edge * edge * edge) {
    const int i = k % edge, j = (k / edge) % edge, l = k / (edge * edge);
    const int* lo = parts[pi].box_lo;
    x = ((lo[0] + i) % p.nx + p.nx) % p.nx;
    y = ((lo[1] + j) % p.ny + p.ny) % p.ny;
    z = ((lo[2] + l) % p.nz + p.nz) % p.nz;
    const uint32_t c0 = ((uint32_t)z * p.ny + y) * p.nx + x;
    active = (flags[c0] & kNearP) && owner[c0] == pi;
  }
  double gF = 0.0, gW = 0.0;
  if (active) {
    const uint32_t c = ((uint32_t)z * p.ny + y) * p.nx + x;
    T d[kQ], lam[kQ], nu[kQ], kap[kQ];
    uint32_t mask = 0;
    int pid = -1;
    double Fl[3] = {0, 0, 0}, Tl[3] = {0, 0, 0}, Kl[3] = {0, 0, 0}, Bl[3] = {0, 0, 0};
    UAddrOf<S> ad = uaddr<sizeof(S) == 2>(p);
    ad.per[0] = ad.per[1] = ad.per[2] = 1;
    boundary_cell<S, UAddrOf<S>>(s, flags, owner, parts, p, ad, x, y, z, c, d, pid, Fl, Tl, Kl, Bl, status, &mask, kap,
                            pi);
#pragma unroll
    for (int q = 0; q < kQ; ++q) lam[q] = T(lin[(size_t)q * N + c]);
    collide_adjoint<T>(d, lam, T(p.sp), T(p.sm), T(p.F[0]), T(p.F[1]), T(p.F[2]), dsm_dw, nu, gF, gW);
    // link force: F_z = -c_qz (s_qbar(x) + f_q(x)) per link of pull direction q
#pragma unroll
    for (int q = 1; q < kQ; ++q)
      if (mask & (1u << q)) nu[q] += T(-wn * cz_of(q));
    if (FIXUP) {
      gF = gW = 0.0;
#pragma unroll
      for (int r = 1; r < kQ; ++r) {
        const int rb = opp_of(r);
        if ((mask & (1u << r)) && !(mask & (1u << rb)) && kap[r] != T(0))
          lout[(size_t)r * N + c] = L(T(lout[(size_t)r * N + c]) - kap[r] * nu[r]);
      }
    } else {
#pragma unroll
      for (int r = 0; r < kQ; ++r) {
        const int rb = opp_of(r);
        const bool src_link = r > 0 && (mask & (1u << r));     // x - c_r solid
        const bool own_link = r > 0 && (mask & (1u << rb));    // x + c_r solid
        if (!src_link) {
          T v = nu[r];
          if (own_link) v += kap[rb] * nu[rb];
          lout[(size_t)r * N + wrap_index(x - cx_of(r), y - cy_of(r), z - cz_of(r), p)] = L(v);
        }
        if (own_link) {
          T v = nu[rb] + T(wn * cz_of(r));
          if (src_link) v -= kap[r] * nu[r];
          lout[(size_t)r * N + c] = L(v);
        }
      }
    }
  }
  if (!FIXUP) {
    gF = wave_sum(gF);
    gW = wave_sum(gW);
    if ((threadIdx.x & 63) == 0) {
      const size_t g = slot0 + (size_t)pi * (((size_t)edge * edge * edge + 255) / 256) * 4 + (k >> 6);
      gslots[2 * g] += gF;
      gslots[2 * g + 1] += gW;
    }
  }
}

// lambda_0 . dC/dtheta at the initial state f = w (d = 0) on every fluid cell
template <typename S>
__global__ __launch_bounds__(512) void k_adj_init(const typename Lam<S>::L* __restrict__ lin,
                                                  const uint8_t* __restrict__ flags, double* __restrict__ gslots,
                                                  SweepParams p, double dsm_dw) {
  using T = typename Store<S>::T;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y, z = blockIdx.z;
  const uint32_t N = p.N;
  const uint32_t c = ((uint32_t)z * p.ny + y) * p.nx + x;
  double gF = 0.0, gW = 0.0;
  if (x < p.nx && !(flags[c] & kSolid)) {
    T d[kQ], lam[kQ], nu[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) { d[q] = T(0); lam[q] = T(lin[(size_t)q * N + c]); }
    collide_adjoint<T>(d, lam, T(p.sp), T(p.sm), T(p.F[0]), T(p.F[1]), T(p.F[2]), dsm_dw, nu, gF, gW);
  }
  const size_t g = blockIdx.x + (size_t)gridDim.x * (blockIdx.y + (size_t)gridDim.y * blockIdx.z);
  group_accumulate(gF, gW, gslots, g);
}

dim3 interior_block(const SweepParams& p) { return dim3(p.nx >= 512 ? 512 : ((p.nx + 63) / 64) * 64); }
dim3 interior_grid(const SweepParams& p) {
  const int bx = interior_block(p).x;
  return dim3((p.nx + bx - 1) / bx, p.ny, p.nz);
}

double dsm_domega(double omega, double magic) {
  const double a = 1.0 / omega - 0.5;
  const double den = 0.5 * a + magic;
  return -magic / (omega * omega * den * den);
}

void adj_free(AdjState* a) { delete a; }

}  // namespace

void adjoint_plan(vmlbm_ctx* c, const Take& take) {
  const vmlbm_config& g = c->cfg;
  if (g.adjoint_steps <= 0 || g.ckpt_every <= 0 || g.block > 0) return;
  if (!c->adj) c->adj = std::unique_ptr<AdjState, void (*)(AdjState*)>(new AdjState(), adj_free);
  AdjState& A = *c->adj;
  const size_t N = (size_t)g.n[0] * g.n[1] * g.n[2];
  const size_t S = storage_bytes(g.storage);
  A.state_bytes = 19 * N * S;
  A.lam_bytes = 19 * N * (g.storage == VMLBM_F64 ? 8 : 4);
  A.n_ckpt = (g.adjoint_steps + g.ckpt_every - 1) / g.ckpt_every;
  A.off_ckpt = take(A.state_bytes * A.n_ckpt);
  A.off_seg = take(A.state_bytes * g.ckpt_every);
  A.off_lam[0] = take(A.lam_bytes);
  A.off_lam[1] = take(A.lam_bytes);
  const SweepParams p = sweep_params(c);
  const dim3 gi = interior_grid(p);
  A.interior_groups = gi.x * gi.y * gi.z;
  const int np = (int)c->spheres.size();
  A.boundary_waves = np * (int)(((size_t)c->box * c->box * c->box + 255) / 256) * 4;
  A.off_g = take(sizeof(double) * 2 * (size_t)(A.interior_groups + A.boundary_waves));
}

}  // namespace vm

using namespace vm;

extern "C" {

int vmlbm_set_params(vmlbm_ctx* c, double body_force_z, double omega) {
  if (!c) return VMLBM_EINVAL;
  if (!(omega > 0.0 && omega < 2.0)) return fail(c, VMLBM_EINVAL, "omega must lie in (0, 2)");
  // checkpoints taken with other parameters no longer belong to them
  if (c->adj) c->adj->have_forward = false;
  c->F[2] = body_force_z;
  c->sp = omega;
  c->sm = s_minus_of(omega, c->cfg.magic);
  c->sb = s_bulk_of(omega, c->cfg.bulk_factor);
  return VMLBM_OK;
}

int vmlbm_forward_ckpt(vmlbm_ctx* c, int sphere, int n_steps, int avg_from, int ckpt_every, double* J) {
  if (!c || !J) return VMLBM_EINVAL;
  if (!c->ws) return fail(c, VMLBM_ESTATE, "workspace not bound");
  if (!c->adj) return fail(c, VMLBM_ESTATE, "no adjoint workspace: set adjoint_steps and ckpt_every");
  AdjState& A = *c->adj;
  const vmlbm_config& g = c->cfg;
  if (g.block > 0) return fail(c, VMLBM_EINVAL, "adjoint needs the uniform grid");
  if (c->sb != c->sp) return fail(c, VMLBM_EINVAL, "adjoint needs the TRT collision (bulk_factor 1)");
  for (int a = 0; a < 3; ++a)
    if (!g.periodic[a]) return fail(c, VMLBM_EINVAL, "adjoint needs a periodic domain");
  for (const auto& s : c->spheres)
    if (s.fixed != 1) return fail(c, VMLBM_EINVAL, "adjoint needs spheres held in place");
  if (sphere < 0 || sphere >= (int)c->spheres.size()) return fail(c, VMLBM_EINVAL, "bad sphere id");
  if (n_steps <= 0 || n_steps > g.adjoint_steps || ckpt_every != g.ckpt_every || n_steps % ckpt_every)
    return fail(c, VMLBM_EINVAL, "n_steps must be a multiple of ckpt_every (%d) and <= %d", g.ckpt_every,
                g.adjoint_steps);
  if (avg_from < 0 || avg_from >= n_steps) return fail(c, VMLBM_EINVAL, "bad averaging window");
  const int W = n_steps - avg_from;
  if (g.history < W) return fail(c, VMLBM_EINVAL, "history (%d) shorter than the window (%d)", g.history, W);
  // f(0) = w, s_0 = C(w)
  int rc = vmlbm_init_equilibrium(c, 1.0, nullptr);
  if (rc) return rc;
  for (int n = 0; n < n_steps; ++n) {
    if (n % ckpt_every == 0)
      HIP_TRY(c, hipMemcpyAsync(c->ws + A.off_ckpt + (size_t)(n / ckpt_every) * A.state_bytes,
                                c->ws + c->off_pdf[c->cur], A.state_bytes, hipMemcpyDeviceToDevice, c->stream));
    rc = uniform_step(c, 1);
    if (rc) return rc;
  }
  rc = vmlbm_sync(c);
  if (rc) return rc;
  std::vector<double> h((size_t)W * kHistWords);
  rc = vmlbm_get_history(c, sphere, W, h.data());
  if (rc) return rc;
  long double acc = 0.0L;
  for (int i = 0; i < W; ++i) acc += h[(size_t)i * kHistWords + 2];
  *J = (double)(acc / W);
  A.n_steps = n_steps;
  A.avg_from = avg_from;
  A.ckpt_every = ckpt_every;
  A.sphere = sphere;
  for (int a = 0; a < 3; ++a) A.F[a] = c->F[a];
  A.sp = c->sp;
  A.have_forward = true;
  return VMLBM_OK;
}

int vmlbm_adjoint(vmlbm_ctx* c, double dJ, double grad[2]) {
  if (!c || !grad) return VMLBM_EINVAL;
  if (!c->adj || !c->adj->have_forward) return fail(c, VMLBM_ESTATE, "vmlbm_forward_ckpt must run first");
  AdjState& A = *c->adj;
  if (A.sp != c->sp || A.F[0] != c->F[0] || A.F[1] != c->F[1] || A.F[2] != c->F[2])
    return fail(c, VMLBM_ESTATE, "parameters changed since vmlbm_forward_ckpt: run it again");
  const SweepParams p = sweep_params(c);
  const int np = (int)c->spheres.size();
  const int K = A.ckpt_every, N = A.n_steps, W = N - A.avg_from;
  const double dsm = dsm_domega(c->sp, c->cfg.magic);
  double* gsl = (double*)(c->ws + A.off_g);
  const size_t ng = (size_t)A.interior_groups + A.boundary_waves;
  HIP_TRY(c, hipMemsetAsync(gsl, 0, 2 * ng * sizeof(double), c->stream));
  HIP_TRY(c, hipMemsetAsync(c->ws + A.off_lam[0], 0, A.lam_bytes, c->stream));
  HIP_TRY(c, hipMemsetAsync(c->ws + A.off_lam[1], 0, A.lam_bytes, c->stream));
  int lcur = 0;   // lambda_{n+1} lives in off_lam[lcur]
  const dim3 gi = interior_grid(p), bi = interior_block(p);
  const int cells = c->box * c->box * c->box;
  const dim3 gb((cells + 255) / 256, np), bb(256);
  for (int seg = N / K - 1; seg >= 0; --seg) {
    // recompute the segment's states s_{seg K} .. s_{seg K + K - 1}
    char* segbuf = c->ws + A.off_seg;
    HIP_TRY(c, hipMemcpyAsync(segbuf, c->ws + A.off_ckpt + (size_t)seg * A.state_bytes, A.state_bytes,
                              hipMemcpyDeviceToDevice, c->stream));
    for (int j = 1; j < K; ++j) {
      SweepParams pr = p;
      pr.seed = step_seed((long long)seg * K + j - 1);
      int rc = sweep_once(c, pr, segbuf + (size_t)(j - 1) * A.state_bytes, segbuf + (size_t)j * A.state_bytes,
                          nullptr, nullptr);
      if (rc) return rc;
    }
    for (int j = K - 1; j >= 0; --j) {
      const int n = seg * K + j;
      const double wn = n >= A.avg_from ? 1.0 / W : 0.0;
      const void* s = segbuf + (size_t)j * A.state_bytes;
      void* lin = c->ws + A.off_lam[lcur];
      void* lout = c->ws + A.off_lam[1 - lcur];
      int rc = dispatch(c->cfg.storage, [&](auto* tag) -> int {
        using S = std::remove_pointer_t<decltype(tag)>;
        using L = typename Lam<S>::L;
        k_adj_interior<S><<<gi, bi, 0, c->stream>>>((const S*)s, (const L*)lin, (L*)lout, c->flags(), gsl, p, dsm);
        HIP_TRY(c, hipGetLastError());
        if (np > 0) {
          k_adj_boundary<S, false><<<gb, bb, 0, c->stream>>>((const S*)s, (const L*)lin, (L*)lout, c->flags(),
                                                              c->owner(), c->parts(), gsl, c->status(), p, dsm, wn,
                                                              (size_t)A.interior_groups);
          HIP_TRY(c, hipGetLastError());
          k_adj_boundary<S, true><<<gb, bb, 0, c->stream>>>((const S*)s, (const L*)lin, (L*)lout, c->flags(),
                                                             c->owner(), c->parts(), gsl, c->status(), p, dsm, wn,
                                                             (size_t)A.interior_groups);
          HIP_TRY(c, hipGetLastError());
        }
        return VMLBM_OK;
      });
      if (rc) return rc;
      lcur = 1 - lcur;
    }
  }
  int rc = dispatch(c->cfg.storage, [&](auto* tag) -> int {
    using S = std::remove_pointer_t<decltype(tag)>;
    using L = typename Lam<S>::L;
    k_adj_init<S><<<gi, bi, 0, c->stream>>>((const L*)(c->ws + A.off_lam[lcur]), c->flags(), gsl, p, dsm);
    HIP_TRY(c, hipGetLastError());
    return VMLBM_OK;
  });
  if (rc) return rc;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  std::vector<double> h(2 * ng);
  HIP_TRY(c, hipMemcpy(h.data(), gsl, h.size() * sizeof(double), hipMemcpyDeviceToHost));
  long double g0 = 0.0L, g1 = 0.0L;
  for (size_t i = 0; i < ng; ++i) { g0 += h[2 * i]; g1 += h[2 * i + 1]; }
  grad[0] = dJ * (double)g0;
  grad[1] = dJ * (double)g1;
  return VMLBM_OK;
}

}  // extern "C"
