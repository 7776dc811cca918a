// Device helpers shared by the forward and adjoint sweeps: periodic
// neighbour indexing, the pull of one cell with its wall and particle links,
// and wave reductions.
#pragma once

#include <utility>

#include "common.hpp"
#include "uniform.hpp"

namespace vm {

struct Idx {
  int xm, xp;            // x-1, x+1 wrapped
  uint32_t rm, r0, rp;   // row offsets of y-1, y, y+1 (wrapped) within a plane
  uint32_t pm, p0, pp;   // plane offsets of z-1, z, z+1 (wrapped)
};

__device__ __forceinline__ Idx make_idx(int x, int y, int z, int nx, int ny, int nz) {
  Idx I;
  I.xm = x == 0 ? nx - 1 : x - 1;
  I.xp = x + 1 == nx ? 0 : x + 1;
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y + 1 == ny ? 0 : y + 1;
  const int zm = z == 0 ? nz - 1 : z - 1, zp = z + 1 == nz ? 0 : z + 1;
  I.rm = (uint32_t)ym * nx; I.r0 = (uint32_t)y * nx; I.rp = (uint32_t)yp * nx;
  const uint32_t plane = (uint32_t)nx * ny;
  I.pm = (uint32_t)zm * plane; I.p0 = (uint32_t)z * plane; I.pp = (uint32_t)zp * plane;
  return I;
}

// index of the pull source x - c_q (periodic wrap; walls handled elsewhere)
template <int Q>
__device__ __forceinline__ uint32_t pull_index(const Idx& I, int x) {
  constexpr int cx = cx_of(Q), cy = cy_of(Q), cz = cz_of(Q);
  const uint32_t xs = cx == 1 ? I.xm : (cx == -1 ? I.xp : x);
  const uint32_t ys = cy == 1 ? I.rm : (cy == -1 ? I.rp : I.r0);
  const uint32_t zs = cz == 1 ? I.pm : (cz == -1 ? I.pp : I.p0);
  return zs + ys + xs;
}

template <typename S, int Q>
__device__ __forceinline__ void load_pull(const S* __restrict__ src, uint32_t N, const Idx& I, int x,
                                          typename Store<S>::T (&d)[kQ]) {
  d[Q] = Store<S>::load(src[(size_t)Q * N + pull_index<Q>(I, x)]);
}

template <typename S, int... Qs>
__device__ __forceinline__ void load_all(const S* __restrict__ src, uint32_t N, const Idx& I, int x,
                                         typename Store<S>::T (&d)[kQ], std::integer_sequence<int, Qs...>) {
  (load_pull<S, Qs>(src, N, I, x, d), ...);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Slow path for a fluid cell with wall or particle links: builds the 19
// incoming populations with Eq. 10 (CLI) on particle links and halfway
// bounce-back on walls, and accumulates the link forces of Eq. 11 and their
// torques (Eq. 12) in FP64.  The constant part 2 w_q c_q of each link force
// is left out: summed over the closed surface of a body it vanishes exactly
// (every lattice line enters and leaves the body equally often), and so does
// its torque (entry and exit points of a line differ by a multiple of c_q).
template <typename S>
__device__ void boundary_cell(const S* __restrict__ src, const uint8_t* __restrict__ flags,
                              const uint16_t* __restrict__ owner, const DevParticle* __restrict__ parts,
                              const SweepParams& p, int x, int y, int z, uint32_t c,
                              typename Store<S>::T (&d)[kQ], int& pid, double (&Fl)[3], double (&Tl)[3],
                              int* __restrict__ status, uint32_t* link_mask = nullptr,
                              typename Store<S>::T* kappa_out = nullptr) {
  using T = typename Store<S>::T;
  const uint32_t N = p.N;
  const int n[3] = {p.nx, p.ny, p.nz};
  // pass 1: pull source of every direction and its flag, loads issued together
  uint32_t sidx[kQ];
  int8_t wall[kQ];          // -1: inside the domain, else 2*axis + side of the wall crossed
  uint8_t sfl[kQ];
#pragma unroll
  for (int q = 1; q < kQ; ++q) {
    const int cq[3] = {cx_of(q), cy_of(q), cz_of(q)};
    int s3[3] = {x - cq[0], y - cq[1], z - cq[2]};
    wall[q] = -1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (s3[a] < 0 || s3[a] >= n[a]) {
        if (p.per[a]) s3[a] = s3[a] < 0 ? s3[a] + n[a] : s3[a] - n[a];
        else if (wall[q] < 0) { wall[q] = (int8_t)(2 * a + (s3[a] < 0 ? 0 : 1)); s3[a] = 0; }
        else s3[a] = 0;
      }
    }
    sidx[q] = ((uint32_t)s3[2] * n[1] + s3[1]) * n[0] + s3[0];
  }
#pragma unroll
  for (int q = 1; q < kQ; ++q) sfl[q] = wall[q] < 0 ? flags[sidx[q]] : 0;
  // pass 2: plain streaming where the source is fluid
  d[0] = Store<S>::load(src[c]);
#pragma unroll
  for (int q = 1; q < kQ; ++q)
    if (wall[q] < 0 && !(sfl[q] & kSolid)) d[q] = Store<S>::load(src[(size_t)q * N + sidx[q]]);
  // pass 3: links
  if (link_mask) *link_mask = 0;
#pragma unroll
  for (int q = 1; q < kQ; ++q) {
    if (kappa_out) kappa_out[q] = T(0);
    if (wall[q] < 0 && !(sfl[q] & kSolid)) continue;
    if (link_mask) *link_mask |= 1u << q;
    const int cq[3] = {cx_of(q), cy_of(q), cz_of(q)};
    const int qq = opp_of(q);
    const double w = w_of(q);
    const T own_qq = Store<S>::load(src[(size_t)qq * N + c]);
    if (wall[q] >= 0) {
      // halfway wall: delta = 1/2 -> kappa0 = 0, alpha = 2
      const int wa = wall[q] >> 1, ws = wall[q] & 1;
      double cv = 0.0;
      if (wa == p.wall_axis)
        cv = -(cq[0] * p.wall_v[ws][0] + cq[1] * p.wall_v[ws][1] + cq[2] * p.wall_v[ws][2]);
      d[q] = own_qq - T(6.0 * w * cv);
      continue;
    }
    // particle link in direction qq (c_qq = -c_q points into the solid)
    const int pi = owner[sidx[q]];
    const DevParticle& P = parts[pi];
    double off[3];
    sphere_offset(P.x, x + 0.5, y + 0.5, z + 0.5, n[0], n[1], n[2], p.per, off);
    const double delta = ray_delta(off, -cq[0], -cq[1], -cq[2], P.r);
    double rb[3] = {off[0] - delta * cq[0], off[1] - delta * cq[1], off[2] - delta * cq[2]};
    double v[3] = {P.u[0] + (P.w[1] * rb[2] - P.w[2] * rb[1]),
                   P.u[1] + (P.w[2] * rb[0] - P.w[0] * rb[2]),
                   P.u[2] + (P.w[0] * rb[1] - P.w[1] * rb[0])};
    double kappa = (1.0 - 2.0 * delta) / (1.0 + 2.0 * delta);
    double alpha = 4.0 / (1.0 + 2.0 * delta);
    // second node x - c_qq = x + c_q
    int t[3] = {x + cq[0], y + cq[1], z + cq[2]};
    bool second_ok = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (t[a] < 0 || t[a] >= n[a]) {
        if (p.per[a]) t[a] = t[a] < 0 ? t[a] + n[a] : t[a] - n[a];
        else second_ok = false;
      }
    }
    uint32_t tidx = 0;
    if (second_ok) {
      tidx = ((uint32_t)t[2] * n[1] + t[1]) * n[0] + t[0];
      if (flags[tidx] & kSolid) second_ok = false;
    }
    if (!second_ok) { kappa = 0.0; alpha = 2.0; }
    if (kappa_out) kappa_out[q] = T(kappa);
    // c_qq . v with c_qq = -c_q
    const double cqv = -(cq[0] * v[0] + cq[1] * v[1] + cq[2] * v[2]);
    T val = own_qq - T(3.0 * alpha * w * cqv);
    if (second_ok) {
      const T sec = Store<S>::load(src[(size_t)qq * N + tidx]);
      const T own_q = Store<S>::load(src[(size_t)q * N + c]);
      val = val + T(kappa) * (sec - own_q);
    }
    d[q] = val;
    // link force: (c_qq - v) d~_qq(x) + (c_qq + v) d_q(x, t+1)
    const double a0 = (double)own_qq, a1 = (double)val;
    double Fq[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) Fq[a] = (-cq[a] - v[a]) * a0 + (-cq[a] + v[a]) * a1;
    if (pid >= 0 && pid != pi) status[kStatusRange] = 2;
    pid = pi;
    Fl[0] += Fq[0]; Fl[1] += Fq[1]; Fl[2] += Fq[2];
    Tl[0] += rb[1] * Fq[2] - rb[2] * Fq[1];
    Tl[1] += rb[2] * Fq[0] - rb[0] * Fq[2];
    Tl[2] += rb[0] * Fq[1] - rb[1] * Fq[0];
  }
}

}  // namespace vm
