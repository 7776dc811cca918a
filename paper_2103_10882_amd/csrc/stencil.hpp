// Device helpers shared by the forward and adjoint sweeps: periodic
// neighbour indexing, the pull of one cell with its wall and particle links,
// and wave reductions.
#pragma once

#include <utility>

#include "common.hpp"

namespace vm {

struct Idx {
  int xm, xp;            // x-1, x+1 wrapped
  uint32_t rm, r0, rp;   // row offsets of y-1, y, y+1 (wrapped) within a plane
  size_t pm, p0, pp;     // offsets of planes z-1, z, z+1 (wrapped): z times the plane stride
};

// plane stride zs: nx ny for cell-indexed arrays, PopLayout::sz for populations
__device__ __forceinline__ Idx make_idx(int x, int y, int z, int nx, int ny, int nz, size_t zs) {
  Idx I;
  I.xm = x == 0 ? nx - 1 : x - 1;
  I.xp = x + 1 == nx ? 0 : x + 1;
  const int ym = y == 0 ? ny - 1 : y - 1, yp = y + 1 == ny ? 0 : y + 1;
  const int zm = z == 0 ? nz - 1 : z - 1, zp = z + 1 == nz ? 0 : z + 1;
  I.rm = (uint32_t)ym * nx; I.r0 = (uint32_t)y * nx; I.rp = (uint32_t)yp * nx;
  I.pm = (size_t)zm * zs; I.p0 = (size_t)z * zs; I.pp = (size_t)zp * zs;
  return I;
}

// offset of the pull source x - c_q within one population (periodic wrap;
// walls handled elsewhere)
template <int Q>
__device__ __forceinline__ size_t pull_index(const Idx& I, int x) {
  constexpr int cx = cx_of(Q), cy = cy_of(Q), cz = cz_of(Q);
  const uint32_t xs = cx == 1 ? I.xm : (cx == -1 ? I.xp : x);
  const uint32_t ys = cy == 1 ? I.rm : (cy == -1 ? I.rp : I.r0);
  const size_t zs = cz == 1 ? I.pm : (cz == -1 ? I.pp : I.p0);
  return zs + ys + xs;
}

template <typename S, int Q>
__device__ __forceinline__ void load_pull(const S* __restrict__ src, uint32_t sq, const Idx& I, int x,
                                          typename Store<S>::T (&d)[kQ]) {
  d[Q] = Store<S>::load(src[(size_t)Q * sq + pull_index<Q>(I, x)]);
}

template <typename S, int... Qs>
__device__ __forceinline__ void load_all(const S* __restrict__ src, uint32_t sq, const Idx& I, int x,
                                         typename Store<S>::T (&d)[kQ], std::integer_sequence<int, Qs...>) {
  (load_pull<S, Qs>(src, sq, I, x, d), ...);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Addressing of a lattice of one level: locate() maps (possibly out-of-range)
// cell coordinates to a cell index c; pop(q, c) is the element of
// population q of cell c.
//
// Uniform grid: cells [z][y][x], populations SoA [q][z][y][x]; periodic axes
// wrap, other axes end in walls.
// Population layout of the uniform grid: element (q, x, y, z) at
// q sq + z sz + y nx + x.  [q][z][y][x] has sq = N, sz = nx ny; [z][q][y][x]
// (the 19 populations of a z-plane side by side) has sq = nx ny,
// sz = 19 nx ny.  Cell indices (flags, owner, rounding streams) stay
// c = z nx ny + y nx + x in both.
struct PopLayout {
  uint32_t sq, plane;
  size_t sz;
  // offset of population q of cell c
  __host__ __device__ __forceinline__ size_t pop(int q, uint32_t c) const {
    const size_t o = (size_t)q * sq + c;
    return sz == plane ? o : o + (size_t)(c / plane) * (sz - plane);
  }
};

// Cell addressing of the uniform grid, its population layout fixed at
// compile time (a runtime choice would carry the plane-interleaved branch and
// its division into every kernel, and it cost the FP32/FP64 boundary kernels
// registers and scratch): PLANE = false [q][z][y][x], true [z][q][y][x].
template <bool PLANE>
struct UAddrT {
  int n[3];
  int per[3];
  PopLayout lay;
  // z = c / (nx ny) by multiplication with a precomputed magic number
  // (division by an invariant integer, Granlund and Montgomery 1994): with
  // l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1, t = hi32(m c),
  // c / d = (t + ((c - t) >> min(l, 1))) >> max(l - 1, 0) for all c < 2^32
  uint32_t zm, zs1, zs2;
  __device__ __forceinline__ size_t pop(int q, uint32_t c) const {
    if constexpr (PLANE) {
      const uint32_t t = __umulhi(zm, c);
      const uint32_t z = (t + ((c - t) >> zs1)) >> zs2;
      return (size_t)q * lay.sq + c + (size_t)z * (lay.sz - lay.plane);
    } else {
      return (size_t)q * lay.sq + c;
    }
  }
  // 1: stored cell c; 0: outside through the wall (axis wa, side ws)
  __device__ __forceinline__ int locate(int x, int y, int z, uint32_t& c, int& wa, int& ws) const {
    int s[3] = {x, y, z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (s[a] < 0 || s[a] >= n[a]) {
        if (per[a]) s[a] = s[a] < 0 ? s[a] + n[a] : s[a] - n[a];
        else { wa = a; ws = s[a] < 0 ? 0 : 1; return 0; }
      }
    }
    c = ((uint32_t)s[2] * n[1] + s[1]) * n[0] + s[0];
    return 1;
  }
};
// the layout of storage type S (FP16: plane-interleaved; see pop_layout)
template <typename S> using UAddrOf = UAddrT<sizeof(S) == 2>;
// flags and owner only (no population access)
using UAddr = UAddrT<false>;

// One level of the block-structured grid: 16^3-cell blocks in slots
// (cell index = slot * 4096 + local, local = (z * 16 + y) * 16 + x),
// periodic; a dense table gives the slot of every block position of the
// level (negative: not stored at this level).  Populations are blocked and
// plane-interleaved, [slot][z][q][16][16]: the 19 populations of a block
// are one contiguous range, and within it the 19 populations of one plane
// of the block sit side by side, so the sweep of a plane reads three
// contiguous runs of 19 x 256 elements (planes z-1, z, z+1) and writes one.
// Against [slot][q][16][16][16] this took the 3-level refined step from
// 27.6k to 28.4k MLUPS in FP16 and 20.8k to 21.1k in FP32 (FP64 within its
// run-to-run spread).
constexpr int kBlock = 16;
constexpr int kBlockCells = kBlock * kBlock * kBlock;
__host__ __device__ __forceinline__ size_t bpop(int q, uint32_t c) {
  return (size_t)(c >> 12) * (kQ * kBlockCells) + (size_t)((c >> 8) & 15u) * (kQ * 256) + (size_t)q * 256 +
         (c & 255u);
}
struct BAddr {
  int n[3];            // cells of the level per axis
  int nb[3];           // block positions of the level per axis
  const int* slot_of;  // [nb2][nb1][nb0]
  uint32_t N;          // cells of the slot pool: slot capacity * 4096
  __device__ __forceinline__ size_t pop(int q, uint32_t c) const { return bpop(q, c); }
  // 1: stored cell c; -1: not stored at this level (c unchanged).  Written
  // with bit masks rather than a branch on the loaded slot, so that callers
  // can issue the lookups of several cells before waiting for any.
  __device__ __forceinline__ int locate(int x, int y, int z, uint32_t& c, int&, int&) const {
    x = x < 0 ? x + n[0] : (x >= n[0] ? x - n[0] : x);
    y = y < 0 ? y + n[1] : (y >= n[1] ? y - n[1] : y);
    z = z < 0 ? z + n[2] : (z >= n[2] ? z - n[2] : z);
    const int s = slot_of[((z >> 4) * nb[1] + (y >> 4)) * nb[0] + (x >> 4)];
    const uint32_t cs = (uint32_t)s * kBlockCells + (uint32_t)((((z & 15) << 4) | (y & 15)) << 4 | (x & 15));
    const uint32_t miss = (uint32_t)(s >> 31);   // all ones where the block is not stored
    c = (cs & ~miss) | (c & miss);
    return (s >> 31) | 1;
  }
};

}  // namespace vm
