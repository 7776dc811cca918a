// Particle coupling kernels shared by the uniform grid and the finest level
// of the block-structured grid, written against an addressing policy
// (UAddr / BAddr): the pull of a cell with its wall and particle links, the
// per-sphere box pass, mapping, re-mapping and refill.
#pragma once

#include "common.hpp"
#include "uniform.hpp"
#include "stencil.hpp"
#include "motion.hpp"

namespace vm {

// Slow path for a fluid cell with wall or particle links: builds the 19
// incoming populations with Eq. 10 (CLI) on particle links and halfway
// bounce-back on walls, and accumulates the link forces of Eq. 11 and their
// torques (Eq. 12) in FP64.  Populations are held as deviations d = f - w,
// so the link force splits into a deviation part (Fl, Tl) and the constant
// part of the weights: with c_qq the direction into the solid,
// (c_qq - v) w + (c_qq + v) w = 2 w c_qq.  Over a body whose every lattice
// line enters and leaves through fluid these constants cancel, but a line
// that leaves the body into a domain wall has no exit link, so they are
// kept, and summed exactly: K = 36 * 2 w c_qq is an integer vector, and the
// torque arm x_b - x_p = (x - x_p) + delta c_qq contributes only through
// x - x_p (c_qq x c_qq = 0), whose unwrapped cell centre L = 2 (x - x_p + x_p)
// is an odd integer vector.  Kl accumulates K and Bl accumulates L x K;
// the constant force is then Kl / 36 and its torque Bl / 72 - x_p x Kl / 36,
// both exactly zero where the constants cancel.
// `sphere` >= 0 names the particle whose links the caller expects: its state
// is then read once instead of per link (a link of another particle still
// sets pid to that one, for the caller's check).  Every stage issues the
// loads of all directions before their first use, and errors are recorded
// after the loops, so that no store can order the loads of one direction
// after those of the previous one.
template <typename S, typename A>
__device__ void boundary_cell(const S* __restrict__ src, const uint8_t* __restrict__ flags,
                              const uint16_t* __restrict__ owner, const DevParticle* __restrict__ parts,
                              const SweepParams& p, const A& ad, int x, int y, int z, uint32_t c,
                              typename Store<S>::T (&d)[kQ], int& pid, double (&Fl)[3], double (&Tl)[3],
                              double (&Kl)[3], double (&Bl)[3],
                              int* __restrict__ status, uint32_t* link_mask = nullptr,
                              typename Store<S>::T* kappa_out = nullptr, int sphere = -1) {
  using T = typename Store<S>::T;
  const int n[3] = {p.nx, p.ny, p.nz};
  // pass 1: pull source of every direction and its flag
  uint32_t sidx[kQ];
  int8_t wall[kQ];          // -1: inside the domain, else 2*axis + side of the wall crossed
  uint8_t sfl[kQ];
  bool unstored = false;
#pragma unroll
  for (int q = 1; q < kQ; ++q) {
    int wa = 0, ws = 0;
    uint32_t si = c;
    const int st = ad.locate(x - cx_of(q), y - cy_of(q), z - cz_of(q), si, wa, ws);
    wall[q] = st == 0 ? (int8_t)(2 * wa + ws) : (int8_t)-1;
    unstored = unstored || st < 0;
    sidx[q] = st < 0 ? c : si;
  }
#pragma unroll
  for (int q = 1; q < kQ; ++q) sfl[q] = wall[q] < 0 ? flags[sidx[q]] : 0;   // sidx = c across walls
  // pass 2: plain streaming where the source is fluid (every source is a
  // stored cell, so the loads need no guard)
  d[0] = Store<S>::load(src[ad.pop(0, c)]);
#pragma unroll
  for (int q = 1; q < kQ; ++q) {
    const T v = Store<S>::load(src[ad.pop(q, sidx[q])]);
    if (wall[q] < 0 && !(sfl[q] & kSolid)) d[q] = v;
  }
  // pass 3: links (non-link directions read the cell itself)
  bool link[kQ];
  T own[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) own[q] = Store<S>::load(src[ad.pop(q, c)]);
  int pq[kQ];
#pragma unroll
  for (int q = 1; q < kQ; ++q) {
    link[q] = wall[q] >= 0 || (sfl[q] & kSolid);
    pq[q] = owner[(link[q] && wall[q] < 0) ? sidx[q] : c];
  }
  // second node x - c_qq = x + c_q of each particle link, located for every
  // direction and kept where it is a stored fluid cell
  uint32_t tidx[kQ];
  bool tok[kQ];
#pragma unroll
  for (int q = 1; q < kQ; ++q) {
    int wa2 = 0, ws2 = 0;
    uint32_t ti = c;
    const int st2 = ad.locate(x + cx_of(q), y + cy_of(q), z + cz_of(q), ti, wa2, ws2);
    tok[q] = link[q] && wall[q] < 0 && st2 == 1;
    tidx[q] = tok[q] ? ti : c;
  }
  uint8_t tfl[kQ];
#pragma unroll
  for (int q = 1; q < kQ; ++q) tfl[q] = flags[tidx[q]];
#pragma unroll
  for (int q = 1; q < kQ; ++q) tok[q] = tok[q] && !(tfl[q] & kSolid);
  T sec[kQ];
#pragma unroll
  for (int q = 1; q < kQ; ++q) sec[q] = Store<S>::load(src[ad.pop(opp_of(q), tok[q] ? tidx[q] : c)]);
  // state of the expected particle, read once
  double kx[3] = {0.0, 0.0, 0.0}, ku[3] = {0.0, 0.0, 0.0}, kw[3] = {0.0, 0.0, 0.0}, kr = 0.0;
  if (sphere >= 0) {
    const DevParticle& K = parts[sphere];
#pragma unroll
    for (int a = 0; a < 3; ++a) { kx[a] = K.x[a]; ku[a] = K.u[a]; kw[a] = K.w[a]; }
    kr = K.r;
  }
  bool mixed = false;
  if (link_mask) *link_mask = 0;
#pragma unroll
  for (int q = 1; q < kQ; ++q) {
    if (kappa_out) kappa_out[q] = T(0);
    if (!link[q]) continue;
    if (link_mask) *link_mask |= 1u << q;
    const int cq[3] = {cx_of(q), cy_of(q), cz_of(q)};
    const int qq = opp_of(q);
    const double w = w_of(q);
    const T own_qq = own[qq];
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
    const int pi = pq[q];
    double px[3], pu[3], pw[3], pr;
    if (sphere >= 0) {
#pragma unroll
      for (int a = 0; a < 3; ++a) { px[a] = kx[a]; pu[a] = ku[a]; pw[a] = kw[a]; }
      pr = kr;
    } else {
      const DevParticle& P = parts[pi];
#pragma unroll
      for (int a = 0; a < 3; ++a) { px[a] = P.x[a]; pu[a] = P.u[a]; pw[a] = P.w[a]; }
      pr = P.r;
    }
    double off[3];
    sphere_offset(px, x + 0.5, y + 0.5, z + 0.5, n[0], n[1], n[2], p.per, off);
    const double delta = ray_delta(off, -cq[0], -cq[1], -cq[2], pr);
    double rb[3] = {off[0] - delta * cq[0], off[1] - delta * cq[1], off[2] - delta * cq[2]};
    double v[3] = {pu[0] + (pw[1] * rb[2] - pw[2] * rb[1]),
                   pu[1] + (pw[2] * rb[0] - pw[0] * rb[2]),
                   pu[2] + (pw[0] * rb[1] - pw[1] * rb[0])};
    double kappa = (1.0 - 2.0 * delta) / (1.0 + 2.0 * delta);
    double alpha = 4.0 / (1.0 + 2.0 * delta);
    if (!tok[q]) { kappa = 0.0; alpha = 2.0; }
    if (kappa_out) kappa_out[q] = T(kappa);
    // c_qq . v with c_qq = -c_q
    const double cqv = -(cq[0] * v[0] + cq[1] * v[1] + cq[2] * v[2]);
    T val = own_qq - T(3.0 * alpha * w * cqv);
    if (tok[q]) val = val + T(kappa) * (sec[q] - own[q]);
    d[q] = val;
    // link force, deviation part: (c_qq - v) d~_qq(x) + (c_qq + v) d_q(x, t+1)
    const double a0 = (double)own_qq, a1 = (double)val;
    double Fq[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) Fq[a] = (-cq[a] - v[a]) * a0 + (-cq[a] + v[a]) * a1;
    mixed = mixed || (pid >= 0 && pid != pi);
    pid = pi;
    Fl[0] += Fq[0]; Fl[1] += Fq[1]; Fl[2] += Fq[2];
    Tl[0] += rb[1] * Fq[2] - rb[2] * Fq[1];
    Tl[1] += rb[2] * Fq[0] - rb[0] * Fq[2];
    Tl[2] += rb[0] * Fq[1] - rb[1] * Fq[0];
    // constant part, exact: K = 36 * 2 w c_qq, L = unwrapped 2 x
    const double kw = q <= 6 ? 4.0 : 2.0;
    const double K[3] = {-kw * cq[0], -kw * cq[1], -kw * cq[2]};
    const double L[3] = {rint(2.0 * (off[0] + px[0])), rint(2.0 * (off[1] + px[1])), rint(2.0 * (off[2] + px[2]))};
    Kl[0] += K[0]; Kl[1] += K[1]; Kl[2] += K[2];
    Bl[0] += L[1] * K[2] - L[2] * K[1];
    Bl[1] += L[2] * K[0] - L[0] * K[2];
    Bl[2] += L[0] * K[1] - L[1] * K[0];
  }
  if (unstored) status[kStatusRange] = 5;
  if (mixed) status[kStatusRange] = 2;
}


// cell k of a box of edge `edge` at origin lo -> lattice coordinates (periodic
// axes wrapped); false if it lies outside the domain
__device__ __forceinline__ bool box_cell(const int* lo, int k, int edge, const SweepParams& p, int& x, int& y,
                                         int& z) {
  const int i = k % edge, j = (k / edge) % edge, l = k / (edge * edge);
  int s[3] = {lo[0] + i, lo[1] + j, lo[2] + l};
  const int n[3] = {p.nx, p.ny, p.nz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (p.per[a]) s[a] = ((s[a] % n[a]) + n[a]) % n[a];
    else if (s[a] < 0 || s[a] >= n[a]) return false;
  }
  x = s[0]; y = s[1]; z = s[2];
  return true;
}

// Box cell k of sphere pi is a link cell of that sphere: a fluid cell with a
// particle link whose owner is pi.
template <typename A>
__device__ __forceinline__ bool link_cell(const uint8_t* __restrict__ flags, const uint16_t* __restrict__ owner,
                                          const DevParticle* __restrict__ parts, int pi, int k,
                                          const SweepParams& p, const A& ad, int& x, int& y, int& z,
                                          uint32_t& c) {
  const int edge = p.box;
  int wa = 0, ws = 0;
  if (k >= edge * edge * edge || !box_cell(parts[pi].box_lo, k, edge, p, x, y, z) ||
      ad.locate(x, y, z, c, wa, ws) != 1)
    return false;
  return (flags[c] & kNearP) && owner[c] == pi;
}

// Link-cell lists, in box order: count per 256-cell chunk, then each chunk
// writes its cells at the offset of the chunks before it.  links[pi][i] is
// the box index of the i-th link cell of sphere pi, llen[pi] their number.
template <typename A>
__global__ __launch_bounds__(256) void k_link_count(const uint8_t* __restrict__ flags,
                                                    const uint16_t* __restrict__ owner,
                                                    const DevParticle* __restrict__ parts, SweepParams p, A ad,
                                                    int* __restrict__ count) {
  const int pi = blockIdx.y;
  int x, y, z;
  uint32_t c;
  const bool in = link_cell<A>(flags, owner, parts, pi, blockIdx.x * 256 + threadIdx.x, p, ad, x, y, z, c);
  const int n = __syncthreads_count(in);
  if (threadIdx.x == 0) count[(size_t)pi * gridDim.x + blockIdx.x] = n;
}

template <typename A>
__global__ __launch_bounds__(256) void k_link_write(const uint8_t* __restrict__ flags,
                                                    const uint16_t* __restrict__ owner,
                                                    const DevParticle* __restrict__ parts, SweepParams p, A ad,
                                                    const int* __restrict__ count, uint32_t* __restrict__ links,
                                                    int* __restrict__ llen) {
  const int pi = blockIdx.y;
  const int k = blockIdx.x * 256 + threadIdx.x;
  __shared__ int part[4];
  __shared__ int wsum[4];
  // offset: cells of the chunks before this one
  const int* cnt = count + (size_t)pi * gridDim.x;
  int before = 0;
  for (int j = threadIdx.x; j < (int)blockIdx.x; j += 256) before += cnt[j];
  for (int m = 32; m >= 1; m >>= 1) before += __shfl_xor(before, m, 64);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) part[wave] = before;
  int x, y, z;
  uint32_t c;
  const bool in = link_cell<A>(flags, owner, parts, pi, k, p, ad, x, y, z, c);
  const unsigned long long m = __ballot(in);
  if (lane == 0) wsum[wave] = __popcll(m);
  __syncthreads();
  const int offset = part[0] + part[1] + part[2] + part[3];
  int base = offset;
  for (int w = 0; w < wave; ++w) base += wsum[w];
  if (in) {
    const int rank = __popcll(m & ((1ull << lane) - 1ull));
    links[(size_t)pi * ((size_t)p.box * p.box * p.box) + base + rank] = (uint32_t)k;
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0)
    llen[pi] = offset + wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

template <typename A>
inline hipError_t launch_link_lists(const uint8_t* flags, const uint16_t* owner, const DevParticle* parts, int np,
                                    const SweepParams& p, const A& ad, int* count, uint32_t* links, int* llen,
                                    hipStream_t st) {
  if (np <= 0) return hipSuccess;
  const dim3 grid(link_chunks(p.box), np), block(256);
  k_link_count<A><<<grid, block, 0, st>>>(flags, owner, parts, p, ad, count);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_link_write<A><<<grid, block, 0, st>>>(flags, owner, parts, p, ad, count, links, llen);
  return hipGetLastError();
}

// Sum of one 256-thread workgroup's force/torque partials into its slot,
// in a fixed order: wave sums, then the four waves (the constant sums are
// integers and add exactly).  Called by every thread of the workgroup.
__device__ __forceinline__ void write_force_slot(double* __restrict__ slots, const SweepParams& p, int pi,
                                                 const double (&Fl)[3], const double (&Tl)[3],
                                                 const double (&Kl)[3], const double (&Bl)[3]) {
  __shared__ double wv[4][kSlotWords];
  double v[kSlotWords] = {Fl[0], Fl[1], Fl[2], Tl[0], Tl[1], Tl[2], Kl[0], Kl[1], Kl[2], Bl[0], Bl[1], Bl[2]};
#pragma unroll
  for (int j = 0; j < kSlotWords; ++j) v[j] = wave_sum(v[j]);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int j = 0; j < kSlotWords; ++j) wv[threadIdx.x >> 6][j] = v[j];
  __syncthreads();
  if (threadIdx.x < kSlotWords) {
    const int j = threadIdx.x;
    slots[(size_t)pi * p.slot_stride + (size_t)blockIdx.x * kSlotWords + j] = (wv[0][j] + wv[1][j]) + (wv[2][j] + wv[3][j]);
  }
}

// Particle-link cells: kLinkGroups workgroups per sphere stride over its
// link list.  Every wave writes its FP64 partial force/torque (zero if it
// held no link) to its own slot, so the per-sphere reduction reads a fixed
// set in a fixed order.
template <typename S, typename A>
__global__ __launch_bounds__(256) void k_boundary_particles(const S* __restrict__ src, S* __restrict__ dst,
                                                            const uint8_t* __restrict__ flags,
                                                            const uint16_t* __restrict__ owner,
                                                            const DevParticle* __restrict__ parts,
                                                            const uint32_t* __restrict__ links,
                                                            const int* __restrict__ llen,
                                                            double* __restrict__ slots, int* __restrict__ status,
                                                            SweepParams p, A ad) {
  using T = typename Store<S>::T;
  const int pi = blockIdx.y;
  const int len = llen[pi];
  const uint32_t* list = links + (size_t)pi * ((size_t)p.box * p.box * p.box);
  double Fl[3] = {0.0, 0.0, 0.0}, Tl[3] = {0.0, 0.0, 0.0}, Kl[3] = {0.0, 0.0, 0.0}, Bl[3] = {0.0, 0.0, 0.0};
  for (int i = blockIdx.x * 256 + threadIdx.x; i < len; i += gridDim.x * 256) {
    int x, y, z;
    uint32_t c;
    if (!link_cell<A>(flags, owner, parts, pi, (int)list[i], p, ad, x, y, z, c)) {
      status[kStatusRange] = 9;
      continue;
    }
    int pid = -1;
    T d[kQ];
    boundary_cell<S, A>(src, flags, owner, parts, p, ad, x, y, z, c, d, pid, Fl, Tl, Kl, Bl, status, nullptr, nullptr,
                        pi);
    if (pid >= 0 && pid != pi) status[kStatusRange] = 2;
    const T drho = lbm_collide<T>(d, T(p.sp), T(p.sm), T(p.sb), T(p.F[0]), T(p.F[1]), T(p.F[2]));
    if (!(drho == drho)) status[kStatusUnstable] = 1;
    SrBits rb(c, p.seed);
#pragma unroll
    for (int q = 0; q < kQ; ++q) dst[ad.pop(q, c)] = Store<S>::store_sr(d[q], rb.next());
  }
  write_force_slot(slots, p, pi, Fl, Tl, Kl, Bl);
}

// Particle-link cells of sphere pi with kLinkLanes lanes per cell: lane s
// builds the incoming populations of directions q = 1 + s + kLinkLanes k
// with the rules of boundary_cell (plain pull, halfway wall, Eq. 10 on
// particle links) and accumulates their link forces and torques; the
// group's populations meet in LDS, and its first lane collides and stores
// the cell.  A lane so runs the per-direction chain of two or three
// directions instead of eighteen (measured against 1, 2, 4 and 16 lanes on
// the 3-level workload).
// Work: workgroup b of G takes the box cells b, b + G, b + 2G, ... (256 of
// them) of the sphere's box, finds its link cells from the current mapping,
// and compacts them in LDS, so no link list has to be built after a
// re-mapping; the stride spreads the surface evenly over the workgroups
// (consecutive cells would leave a few workgroups with most of the link
// cells).  Force and torque partials go to one slot per workgroup.
constexpr int kLinkLanes = 8;
template <typename S, typename A>
__global__ __launch_bounds__(256) void k_link_cells(const S* __restrict__ src, S* __restrict__ dst,
                                                    const uint8_t* __restrict__ flags,
                                                    const uint16_t* __restrict__ owner,
                                                    const DevParticle* __restrict__ parts,
                                                    double* __restrict__ slots, int* __restrict__ status,
                                                    SweepParams p, A ad) {
  using T = typename Store<S>::T;
  constexpr int kCells = 256 / kLinkLanes;
  __shared__ T din[kCells][kQ];
  __shared__ int lx[256], ly[256], lz[256];
  __shared__ uint32_t lc[256];
  __shared__ int wcount[4];
  const int pi = blockIdx.y;
  // link cells among this workgroup's box cells, in box order, with their
  // coordinates and cell index (no flag is written during the pass, so the
  // rounds below take them from here instead of locating them again)
  {
    const int k = blockIdx.x + threadIdx.x * gridDim.x;
    int x, y, z;
    uint32_t c;
    const bool in = link_cell<A>(flags, owner, parts, pi, k, p, ad, x, y, z, c);
    const unsigned long long m = __ballot(in);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) wcount[wave] = __popcll(m);
    __syncthreads();
    int base = 0;
    for (int w = 0; w < wave; ++w) base += wcount[w];
    if (in) {
      const int at = base + __popcll(m & ((1ull << lane) - 1ull));
      lx[at] = x; ly[at] = y; lz[at] = z; lc[at] = c;
    }
    __syncthreads();
  }
  const int len = wcount[0] + wcount[1] + wcount[2] + wcount[3];
  const int n[3] = {p.nx, p.ny, p.nz};
  const int g = threadIdx.x / kLinkLanes, s = threadIdx.x % kLinkLanes;
  double px[3], pu[3], pw[3];
  for (int a = 0; a < 3; ++a) { px[a] = parts[pi].x[a]; pu[a] = parts[pi].u[a]; pw[a] = parts[pi].w[a]; }
  const double pr = parts[pi].r;
  double Fl[3] = {0.0, 0.0, 0.0}, Tl[3] = {0.0, 0.0, 0.0}, Kl[3] = {0.0, 0.0, 0.0}, Bl[3] = {0.0, 0.0, 0.0};
  bool unstored = false, foreign = false;
  // rounds are uniform over the workgroup
  for (int base = 0; base < len; base += kCells) {
    const int i = base + g;
    const bool active = i < len;
    const int x = active ? lx[i] : 0, y = active ? ly[i] : 0, z = active ? lz[i] : 0;
    const uint32_t c = active ? lc[i] : 0;
    if (active) {
      if (s == 0) din[g][0] = Store<S>::load(src[ad.pop(0, c)]);
#pragma unroll
      for (int k = 0; k < (kQ - 2) / kLinkLanes + 1; ++k) {
        const int q = 1 + s + kLinkLanes * k;
        if (q >= kQ) break;
        const int cq[3] = {cx_of(q), cy_of(q), cz_of(q)};
        const int qq = opp_of(q);
        int wa = 0, ws = 0;
        uint32_t si = c;
        const int st = ad.locate(x - cq[0], y - cq[1], z - cq[2], si, wa, ws);
        unstored = unstored || st < 0;
        si = st < 0 ? c : si;
        const uint8_t sf = st == 1 ? flags[si] : 0;
        const int pq = owner[si];
        int wa2 = 0, ws2 = 0;
        uint32_t ti = c;
        const int st2 = ad.locate(x + cq[0], y + cq[1], z + cq[2], ti, wa2, ws2);
        ti = st2 == 1 ? ti : c;
        const uint8_t tf = flags[ti];
        const T v = Store<S>::load(src[ad.pop(q, si)]);
        const T own_q = Store<S>::load(src[ad.pop(q, c)]);
        const T own_qq = Store<S>::load(src[ad.pop(qq, c)]);
        // the second node's population is read before its flag decides
        // whether it is used (ti is the cell itself where it is not stored)
        const T sec_t = Store<S>::load(src[ad.pop(qq, ti)]);
        const bool wall = st == 0, link = wall || (sf & kSolid);
        const bool tok = link && !wall && st2 == 1 && !(tf & kSolid);
        const T sec = tok ? sec_t : own_qq;
        T out = v;
        if (link && wall) {
          // halfway wall: delta = 1/2 -> kappa0 = 0, alpha = 2
          double cv = 0.0;
          if (wa == p.wall_axis)
            cv = -(cq[0] * p.wall_v[ws][0] + cq[1] * p.wall_v[ws][1] + cq[2] * p.wall_v[ws][2]);
          out = own_qq - T(6.0 * w_of(q) * cv);
        } else if (link) {
          foreign = foreign || pq != pi;
          double off[3];
          sphere_offset(px, x + 0.5, y + 0.5, z + 0.5, n[0], n[1], n[2], p.per, off);
          const double delta = ray_delta(off, -cq[0], -cq[1], -cq[2], pr);
          const double rb[3] = {off[0] - delta * cq[0], off[1] - delta * cq[1], off[2] - delta * cq[2]};
          const double vw[3] = {pu[0] + (pw[1] * rb[2] - pw[2] * rb[1]),
                                pu[1] + (pw[2] * rb[0] - pw[0] * rb[2]),
                                pu[2] + (pw[0] * rb[1] - pw[1] * rb[0])};
          double kappa = (1.0 - 2.0 * delta) / (1.0 + 2.0 * delta);
          double alpha = 4.0 / (1.0 + 2.0 * delta);
          if (!tok) { kappa = 0.0; alpha = 2.0; }
          const double cqv = -(cq[0] * vw[0] + cq[1] * vw[1] + cq[2] * vw[2]);
          T val = own_qq - T(3.0 * alpha * w_of(q) * cqv);
          if (tok) val = val + T(kappa) * (sec - own_q);
          out = val;
          const double a0 = (double)own_qq, a1 = (double)val;
          double Fq[3];
#pragma unroll
          for (int a = 0; a < 3; ++a) Fq[a] = (-cq[a] - vw[a]) * a0 + (-cq[a] + vw[a]) * a1;
          Fl[0] += Fq[0]; Fl[1] += Fq[1]; Fl[2] += Fq[2];
          Tl[0] += rb[1] * Fq[2] - rb[2] * Fq[1];
          Tl[1] += rb[2] * Fq[0] - rb[0] * Fq[2];
          Tl[2] += rb[0] * Fq[1] - rb[1] * Fq[0];
          // constant part of the weights, exact (as in boundary_cell)
          const double kw = q <= 6 ? 4.0 : 2.0;
          const double K[3] = {-kw * cq[0], -kw * cq[1], -kw * cq[2]};
          const double L[3] = {rint(2.0 * (off[0] + px[0])), rint(2.0 * (off[1] + px[1])),
                               rint(2.0 * (off[2] + px[2]))};
          Kl[0] += K[0]; Kl[1] += K[1]; Kl[2] += K[2];
          Bl[0] += L[1] * K[2] - L[2] * K[1];
          Bl[1] += L[2] * K[0] - L[0] * K[2];
          Bl[2] += L[0] * K[1] - L[1] * K[0];
        }
        din[g][q] = out;
      }
    }
    __syncthreads();
    if (active && s == 0) {
      T d[kQ];
#pragma unroll
      for (int q = 0; q < kQ; ++q) d[q] = din[g][q];
      const T drho = lbm_collide<T>(d, T(p.sp), T(p.sm), T(p.sb), T(p.F[0]), T(p.F[1]), T(p.F[2]));
      if (!(drho == drho)) status[kStatusUnstable] = 1;
      SrBits rb(c, p.seed);
#pragma unroll
      for (int q = 0; q < kQ; ++q) dst[ad.pop(q, c)] = Store<S>::store_sr(d[q], rb.next());
    }
    __syncthreads();
  }
  if (unstored) status[kStatusRange] = 5;
  if (foreign) status[kStatusRange] = 2;
  write_force_slot(slots, p, pi, Fl, Tl, Kl, Bl);
}

// ---------------------------------------------------------------------------
// mapping (Sec. 2.3): a cell is solid for the first sphere whose centre lies
// within r of its centre; a fluid cell next to a solid one carries the
// particle-link flag and the id of that sphere, one next to a wall the
// wall-link flag
// ---------------------------------------------------------------------------
// OLD: with the positions the mapping in place was made with (xold) rather
// than the current ones
template <bool OLD = false>
__device__ inline int cell_owner(int x, int y, int z, const DevParticle* __restrict__ parts, int np,
                                 const SweepParams& p) {
  for (int i = 0; i < np; ++i) {
    double off[3];
    sphere_offset(OLD ? parts[i].xold : parts[i].x, x + 0.5, y + 0.5, z + 0.5, p.nx, p.ny, p.nz, p.per, off);
    if (inside_sphere(off, parts[i].r)) return i;
  }
  return -1;
}

template <typename A>
__device__ void map_cell(int x, int y, int z, uint32_t c, uint8_t* __restrict__ flags,
                         uint16_t* __restrict__ owner, const DevParticle* __restrict__ parts, int np,
                         const SweepParams& p, const A& ad, int* __restrict__ status) {
  const int o = cell_owner(x, y, z, parts, np, p);
  uint8_t f = 0;
  int link = -1;
  if (o >= 0) {
    f = kSolid;
    link = o;
  } else {
    // the neighbour lookups of all directions are issued before any is
    // used: the kernel is one short wave of latency-bound work
    int st[kQ];
#pragma unroll
    for (int q = 1; q < kQ; ++q) {
      uint32_t sc = 0;
      int wa = 0, ws = 0;
      st[q] = ad.locate(x + cx_of(q), y + cy_of(q), z + cz_of(q), sc, wa, ws);
    }
    bool mixed = false;
#pragma unroll
    for (int q = 1; q < kQ; ++q) {
      if (st[q] == 0) { f |= kNearW; continue; }
      if (st[q] < 0) continue;
      const int so = cell_owner(x + cx_of(q), y + cy_of(q), z + cz_of(q), parts, np, p);
      if (so >= 0) {
        mixed = mixed || (link >= 0 && link != so);
        if (link < 0) link = so;
        f |= kNearP;
      }
    }
    if (mixed) status[kStatusRange] = 4;
  }
  flags[c] = f;
  owner[c] = link < 0 ? 0 : (uint16_t)link;
}

// ---------------------------------------------------------------------------
// refill of cells uncovered by a moving sphere (Sec. 2.3, after Dorschner):
// rho = mean density of the D3Q19 neighbours that held fluid before the
// re-mapping; v = rigid-body velocity; strain rate S from central differences
// over the axis neighbours (fluid velocity where the neighbour held fluid,
// rigid-body velocity of its sphere or the wall velocity otherwise);
// f = f^eq(rho, v) - 3 w_q / s+ (c c - I/3) : S, then collided.  The mapping
// before the re-mapping is evaluated from the positions it was made with
// (xold), so the refill reads no flags and can share a kernel with the
// re-mapping that rewrites them.
// ---------------------------------------------------------------------------
// velocity at the neighbour of cell (x, y, z) across axis a on side `side`
// (0: -1, 1: +1): fluid momentum, the rigid-body velocity of a solid
// neighbour's sphere, or the wall velocity
template <typename S, typename A>
__device__ __forceinline__ void axis_velocity(const S* __restrict__ state, const DevParticle* __restrict__ parts,
                                              int np, const SweepParams& p, const A& ad, int x, int y, int z,
                                              uint32_t c, const DevParticle& P, int* __restrict__ status, int a,
                                              int side, double (&V)[3]) {
  int s[3] = {x, y, z};
  s[a] += side ? 1 : -1;
  uint32_t sc = c;
  int wa2 = 0, ws2 = 0;
  const int st = ad.locate(s[0], s[1], s[2], sc, wa2, ws2);
  const uint32_t src = st == 1 ? sc : c;
  const int ow = st == 1 ? cell_owner<true>(s[0], s[1], s[2], parts, np, p) : -1;
  double j[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const double dq = (double)Store<S>::load(state[ad.pop(q, src)]);
    j[0] += cx_of(q) * dq; j[1] += cy_of(q) * dq; j[2] += cz_of(q) * dq;
  }
  if (st == 0) {
    for (int b = 0; b < 3; ++b) V[b] = (wa2 == p.wall_axis) ? p.wall_v[ws2][b] : 0.0;
  } else if (st < 0) {
    status[kStatusRange] = 5;
    double off[3];
    sphere_offset(P.x, x + 0.5, y + 0.5, z + 0.5, p.nx, p.ny, p.nz, p.per, off);
    V[0] = P.u[0] + (P.w[1] * off[2] - P.w[2] * off[1]);
    V[1] = P.u[1] + (P.w[2] * off[0] - P.w[0] * off[2]);
    V[2] = P.u[2] + (P.w[0] * off[1] - P.w[1] * off[0]);
  } else if (ow < 0) {
    // post-collision momentum minus F/2 is the macroscopic velocity
    for (int b = 0; b < 3; ++b) V[b] = j[b] - 0.5 * p.F[b];
  } else {
    const DevParticle& Q = parts[ow];
    double o2[3];
    sphere_offset(Q.x, s[0] + 0.5, s[1] + 0.5, s[2] + 0.5, p.nx, p.ny, p.nz, p.per, o2);
    V[0] = Q.u[0] + (Q.w[1] * o2[2] - Q.w[2] * o2[1]);
    V[1] = Q.u[1] + (Q.w[2] * o2[0] - Q.w[0] * o2[2]);
    V[2] = Q.u[2] + (Q.w[0] * o2[1] - Q.w[1] * o2[0]);
  }
}

// One wave refills one cell (the cell is the same in every lane).  Lanes
// 0-17 take the D3Q19 neighbour q = lane + 1 for the density, lanes 32-34
// the two axis neighbours of axis lane - 32 for the strain rate; each lane
// reads its neighbours' 19 populations.  The partial results meet by
// shuffles, and every lane then sums them in the order a single thread would
// (neighbours 1 to 18 one after another, the rolled loop keeping one value
// live at a time), so the refilled state does not depend on the split; lane
// 0 stores it.  One thread per cell held 18 x 19 loads in flight and about
// 400 registers, which held the whole re-mapping kernel at one wave per SIMD.
template <typename S, typename A>
__device__ void refill_cell_wave(S* __restrict__ state, const DevParticle* __restrict__ parts, int np,
                                 const SweepParams& p, const A& ad, int x, int y, int z, uint32_t c,
                                 const DevParticle& P, int* __restrict__ status) {
  using T = typename Store<S>::T;
  const int lane = threadIdx.x & 63;
  // density part: 1 + sum of the deviations of an old-fluid neighbour
  double t = 0.0;
  int use = 0;
  if (lane < kQ - 1) {
    const int q = lane + 1;
    const int qx = x + cx_of(q), qy = y + cy_of(q), qz = z + cz_of(q);
    int wa = 0, ws = 0;
    uint32_t sc = c;
    const bool ok = ad.locate(qx, qy, qz, sc, wa, ws) == 1;
    const uint32_t nc = ok ? sc : c;
    use = ok && cell_owner<true>(qx, qy, qz, parts, np, p) < 0;
    double r = 0.0;
#pragma unroll
    for (int r2 = 0; r2 < kQ; ++r2) r += (double)Store<S>::load(state[ad.pop(r2, nc)]);
    t = 1.0 + r;
  }
  // velocity difference across axis a between the neighbours at +1 and -1
  // (fluid momentum, the rigid-body velocity of a solid neighbour's sphere,
  // or the wall velocity)
  double G[3] = {0.0, 0.0, 0.0};
  if (lane >= 32 && lane < 35) {
    double V0[3], V1[3];
    axis_velocity<S, A>(state, parts, np, p, ad, x, y, z, c, P, status, lane - 32, 0, V0);
    axis_velocity<S, A>(state, parts, np, p, ad, x, y, z, c, P, status, lane - 32, 1, V1);
    for (int b = 0; b < 3; ++b) G[b] = V1[b] - V0[b];
  }
  // every lane gathers the partials and computes the same refilled cell
  double rsum = 0.0;
  int cnt = 0;
#pragma unroll 1
  for (int k = 0; k < kQ - 1; ++k) {
    const double tk = __shfl(t, k, 64);
    const int uk = __shfl(use, k, 64);
    rsum = uk ? rsum + tk : rsum;
    cnt += uk;
  }
  double Ga[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) Ga[a][b] = __shfl(G[b], 32 + a, 64);
  const double rho = cnt ? rsum / cnt : 1.0;
  double off[3];
  sphere_offset(P.x, x + 0.5, y + 0.5, z + 0.5, p.nx, p.ny, p.nz, p.per, off);
  const double v[3] = {P.u[0] + (P.w[1] * off[2] - P.w[2] * off[1]),
                       P.u[1] + (P.w[2] * off[0] - P.w[0] * off[2]),
                       P.u[2] + (P.w[0] * off[1] - P.w[1] * off[0])};
  double Sab[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Sab[a][b] = 0.25 * (Ga[a][b] + Ga[b][a]);
  const double trS = Sab[0][0] + Sab[1][1] + Sab[2][2];
  const double usq = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  if (lane != 0) return;
  T d[kQ];
  for (int q = 0; q < kQ; ++q) {
    const int cq[3] = {cx_of(q), cy_of(q), cz_of(q)};
    const double cu = cq[0] * v[0] + cq[1] * v[1] + cq[2] * v[2];
    double QS = -trS / 3.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) QS += cq[a] * cq[b] * Sab[a][b];
    const double w = w_of(q);
    d[q] = T(w * (rho - 1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq) - 3.0 * w / p.sp * QS);
  }
  lbm_collide<T>(d, T(p.sp), T(p.sm), T(p.sb), T(p.F[0]), T(p.F[1]), T(p.F[2]));
  SrBits sr(c, ~p.seed);
  for (int q = 0; q < kQ; ++q) state[ad.pop(q, c)] = Store<S>::store_sr(d[q], sr.next());
}

// the box cell k of the re-mapping region and whether its centre lies within
// 1.6 cells of the sphere's surface at the old or the new position: a cell
// farther off at both keeps its flags, since neither it nor any of its
// neighbours (at most sqrt 2 away) changes side
template <typename A>
__device__ __forceinline__ bool remap_cell(const DevParticle& P, int k, int rb, const SweepParams& p, const A& ad,
                                           int& x, int& y, int& z, uint32_t& c) {
  int wa = 0, ws = 0;
  if (k >= rb * rb * rb || !box_cell(P.remap_lo, k, rb, p, x, y, z) || ad.locate(x, y, z, c, wa, ws) != 1)
    return false;
  double dn[3], dd[3];
  sphere_offset(P.x, x + 0.5, y + 0.5, z + 0.5, p.nx, p.ny, p.nz, p.per, dn);
  sphere_offset(P.xold, x + 0.5, y + 0.5, z + 0.5, p.nx, p.ny, p.nz, p.per, dd);
  const double an = sqrt(dn[0] * dn[0] + dn[1] * dn[1] + dn[2] * dn[2]);
  const double ao = sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
  constexpr double kMargin = 1.6;
  return !((an > P.r + kMargin && ao > P.r + kMargin) || (an < P.r - kMargin && ao < P.r - kMargin));
}

// Re-mapping of a moving sphere's region (its box around the old and the new
// position) and refill of the cells it uncovered.  The two are independent
// (the refill reads populations and the positions, the re-mapping writes
// flags), so the first half of the workgroups re-maps, one thread per cell,
// and the second half refills: each of its workgroups collects the
// uncovered cells among its 256 box cells in LDS, and its four waves take
// them one cell per wave.  The kernel lasts as long as the slower half.
template <typename S, typename A>
__global__ __launch_bounds__(256) void k_refill_remap(
    S* __restrict__ state, uint8_t* __restrict__ flags, uint16_t* __restrict__ owner,
    const DevParticle* __restrict__ parts, int np, SweepParams p, A ad, int* __restrict__ status) {
  const int pi = blockIdx.y;
  const DevParticle& P = parts[pi];
  if (P.fixed) return;
  const int rb = p.box + 1;
  const int half = (int)gridDim.x / 2;
  const bool refill = (int)blockIdx.x >= half;
  const int k = (refill ? (int)blockIdx.x - half : (int)blockIdx.x) * blockDim.x + threadIdx.x;
  int x = 0, y = 0, z = 0;
  uint32_t c = 0;
  const bool near = remap_cell<A>(P, k, rb, p, ad, x, y, z, c);
  if (!refill) {
    if (near) map_cell<A>(x, y, z, c, flags, owner, parts, np, p, ad, status);
    return;
  }
  __shared__ int list[256];
  __shared__ int wcount[4];
  const bool todo = near && cell_owner<true>(x, y, z, parts, np, p) == pi && cell_owner(x, y, z, parts, np, p) < 0;
  const unsigned long long m = __ballot(todo);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) wcount[wave] = __popcll(m);
  __syncthreads();
  int base = 0;
  for (int w = 0; w < wave; ++w) base += wcount[w];
  if (todo) list[base + __popcll(m & ((1ull << lane) - 1ull))] = k;
  __syncthreads();
  const int len = wcount[0] + wcount[1] + wcount[2] + wcount[3];
  for (int i = wave; i < len; i += 4) {
    int rx = 0, ry = 0, rz = 0, wa = 0, ws = 0;
    uint32_t rc = 0;
    box_cell(P.remap_lo, list[i], rb, p, rx, ry, rz);
    ad.locate(rx, ry, rz, rc, wa, ws);
    refill_cell_wave<S, A>(state, parts, np, p, ad, rx, ry, rz, rc, P, status);
  }
}

}  // namespace vm
