// Per-particle force/torque reduction (fixed order, FP64) fused with the
// two-step average and the virtual-mass velocity-Verlet update (Sec. 2.2,
// Sec. 3.3, Algorithm 1); one workgroup per sphere after the link-cell pass,
// on the uniform grid and on the refined grid's finest level.
#pragma once

#include "common.hpp"
#include "uniform.hpp"
#include "stencil.hpp"

namespace vm {

// ---------------------------------------------------------------------------
// Particle update.  The acceleration inside the virtual force and torque is
// the previous step's (Sec. 3.3) or the derivative of the quadratic through
// the three most recent velocities (the Lagrange alternative the paper
// attributes to Schwarz et al.), taken at the new time level (scheme 1:
// 5/2 u_{n-1} - 4 u_{n-2} + 3/2 u_{n-3}) or at the newest velocity (scheme
// 2: 3/2 u_{n-1} - 2 u_{n-2} + 1/2 u_{n-3}); the previous step's stands in
// until three velocities are known.  Held
// spheres (fixed = 1) are not moved; fixed = 2 (position held, rotation
// free, Sec. 3.4.2) integrates the rotation only.
// ---------------------------------------------------------------------------
__device__ inline void particle_update(DevParticle& P, const double (&F)[3], const double (&T)[3],
                                       int* __restrict__ status, const SweepParams& p, const UpdateParams& u) {
#pragma clang fp contract(off)
  // the mapping in place was made at the position before this update
  for (int a = 0; a < 3; ++a) P.xold[a] = P.x[a];
  bool finite = true;
  for (int a = 0; a < 3; ++a) finite = finite && isfinite(F[a]) && isfinite(T[a]);
  if (!finite) status[kStatusUnstable] = 2;
  for (int a = 0; a < 3; ++a) { P.F[a] = F[a]; P.T[a] = T[a]; }
  if (P.fixed == 1) return;
  const double xold[3] = {P.x[0], P.x[1], P.x[2]};
  const double PI = 3.14159265358979323846;
  const double V = 4.0 / 3.0 * PI * P.r * P.r * P.r;
  const double m = (P.rho + P.cv) * V;
  const double I = 0.4 * (P.rho + P.cvw) * V * P.r * P.r;
  const bool lagrange = P.scheme != 0 && P.nvel >= 3;
  const bool at_new = P.scheme == 1;
  const double k0 = at_new ? 2.5 : 1.5, k1 = at_new ? -4.0 : -2.0, k2 = at_new ? 1.5 : 0.5;
  const bool translate = P.fixed == 0;
  for (int a = 0; a < 3; ++a) {
    const double Fav = P.have_prev ? 0.5 * (F[a] + P.Fprev[a]) : F[a];
    const double Tav = P.have_prev ? 0.5 * (T[a] + P.Tprev[a]) : T[a];
    const double a_est = lagrange ? k0 * P.u[a] + k1 * P.uh[0][a] + k2 * P.uh[1][a] : P.a[a];
    const double b_est = lagrange ? k0 * P.w[a] + k1 * P.wh[0][a] + k2 * P.wh[1][a] : P.b[a];
    const double Fg = (P.rho - 1.0) * u.g[a] * V;
    const double an = (Fav + Fg + P.cv * V * a_est) / m;
    const double bn = (Tav + 0.4 * P.cvw * V * P.r * P.r * b_est) / I;
    P.uh[1][a] = P.uh[0][a];
    P.uh[0][a] = P.u[a];
    P.wh[1][a] = P.wh[0][a];
    P.wh[0][a] = P.w[a];
    P.w[a] = P.w[a] + 0.5 * (P.b[a] + bn);
    P.b[a] = bn;
    if (!translate) continue;
    P.u[a] = P.u[a] + 0.5 * (P.a[a] + an);
    double xn = P.x[a] + P.u[a] + 0.5 * an;
    if (p.per[a]) {
      const double na = a == 0 ? p.nx : (a == 1 ? p.ny : p.nz);
      if (xn < 0.0) xn += na;
      else if (xn >= na) xn -= na;
    }
    P.x[a] = xn;
    P.a[a] = an;
  }
  P.nvel = P.nvel < 3 ? P.nvel + 1 : 3;
  if (translate) {
    double speed = P.u[0] * P.u[0] + P.u[1] * P.u[1] + P.u[2] * P.u[2];
    if (!(speed < 0.25)) {
      // blown up (the host reports it at the next sync): the sphere keeps
      // its last position, so boxes and mapping stay finite and in range
      status[kStatusUnstable] = 3;
      for (int a = 0; a < 3; ++a) P.x[a] = xold[a];
    }
    // new boxes: force slots around the new position, re-mapping region
    // covering old and new position
    for (int a = 0; a < 3; ++a) {
      const int na = a == 0 ? p.nx : (a == 1 ? p.ny : p.nz);
      int lo_new = (int)floor(P.x[a] - P.r) - 3;
      int lo_old = (int)floor(xold[a] - P.r) - 3;
      double dx = P.x[a] - xold[a];
      if (p.per[a]) {
        if (dx > 0.5 * na) dx -= na;
        else if (dx < -0.5 * na) dx += na;
      }
      if (!(fabs(dx) < 0.5)) status[kStatusRange] = 3;
      int lo = dx >= 0.0 ? lo_old : lo_new;
      if (p.per[a]) { lo = ((lo % na) + na) % na; lo_new = ((lo_new % na) + na) % na; }
      P.remap_lo[a] = lo;
      P.box_lo[a] = lo_new;
    }
  }
}

// Sum of the kSlotWords-double slots of sphere pi in a fixed order, then
// the two-step average and the particle update; run by one whole workgroup.
__device__ inline void reduce_update(DevParticle* __restrict__ parts, const double* __restrict__ slots,
                                     double* __restrict__ hist, int* __restrict__ status, const SweepParams& p,
                                     const UpdateParams& u, int pi) {
  __shared__ double red[kSlotWords][4];
  double acc[kSlotWords];
#pragma unroll
  for (int j = 0; j < kSlotWords; ++j) acc[j] = 0.0;
  const double* s = slots + (size_t)pi * p.slot_stride;
  const int nslots = (int)(p.slot_stride / kSlotWords);
  for (int k = threadIdx.x; k < nslots; k += blockDim.x) {
#pragma unroll
    for (int j = 0; j < kSlotWords; ++j) acc[j] += s[(size_t)k * kSlotWords + j];
  }
#pragma unroll
  for (int j = 0; j < kSlotWords; ++j) acc[j] = wave_sum(acc[j]);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int j = 0; j < kSlotWords; ++j) red[j][threadIdx.x >> 6] = acc[j];
  __syncthreads();
  if (threadIdx.x != 0) return;
  double tot[kSlotWords];
#pragma unroll
  for (int j = 0; j < kSlotWords; ++j) tot[j] = (red[j][0] + red[j][1]) + (red[j][2] + red[j][3]);
  DevParticle& P = parts[pi];
  // deviation parts plus the weight constants (Eq. 11 on f = w + d): the
  // integer sums K and L x K give K / 36 and L x K / 72 - x_p x K / 36
  const double K[3] = {tot[6], tot[7], tot[8]}, B[3] = {tot[9], tot[10], tot[11]};
  const double Fc[3] = {K[0] / 36.0, K[1] / 36.0, K[2] / 36.0};
  const double Tc[3] = {B[0] / 72.0 - (P.x[1] * Fc[2] - P.x[2] * Fc[1]),
                        B[1] / 72.0 - (P.x[2] * Fc[0] - P.x[0] * Fc[2]),
                        B[2] / 72.0 - (P.x[0] * Fc[1] - P.x[1] * Fc[0])};
  double F[3] = {tot[0] + Fc[0], tot[1] + Fc[1], tot[2] + Fc[2]};
  double T[3] = {tot[3] + Tc[0], tot[4] + Tc[1], tot[5] + Tc[2]};
  particle_update(P, F, T, status, p, u);
  for (int a = 0; a < 3; ++a) { P.Fprev[a] = F[a]; P.Tprev[a] = T[a]; }
  P.have_prev = 1;
  double* h = hist + ((size_t)(u.step % u.hist_len) * u.np + pi) * kHistWords;
  for (int a = 0; a < 3; ++a) {
    h[a] = F[a];
    h[3 + a] = T[a];
    h[6 + a] = P.x[a];
    h[9 + a] = P.u[a];
    h[12 + a] = P.w[a];
  }
}


}  // namespace vm
