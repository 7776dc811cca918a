// Launch parameters and launchers of the uniform-grid kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "common.hpp"
#include "particle_state.hpp"
#include "stencil.hpp"

namespace vm {

struct SweepParams {
  int nx, ny, nz;
  int per[3];
  int wall_axis;          // first non-periodic axis or -1
  double wall_v[2][3];    // velocity of its low / high wall
  double sp, sm;          // s+ = omega, s- from the magic parameter
  double sb;              // s_b of the MRT bulk moments (= sp for TRT)
  double F[3];            // fluid body force
  uint32_t N;             // cells
  uint32_t sq;            // population stride of the layout (PopLayout)
  size_t sz;              // z-plane stride of the layout
  int box;                // edge of a sphere's box (cells); holds all its link cells
  size_t slot_stride;     // doubles per sphere in the force-slot array (kSlotWords per workgroup)
  uint32_t seed;          // stochastic-rounding stream of this sweep
};

// Population layout by storage format: FP16 keeps the 19 populations of a
// z-plane side by side ([z][q][y][x]), the others [q][z][y][x] (the kernels'
// UAddrOf<S> makes the same choice at compile time).  The sweep's
// access pattern without arithmetic moved 6.0 against 5.4 TB/s in FP16 with
// the first on 512^3 (5.6 against 5.6 in FP32, 5.1 against 5.4 in FP64).
inline PopLayout pop_layout(int storage, const int n[3]) {
  PopLayout L;
  L.plane = (uint32_t)n[0] * (uint32_t)n[1];
  if (storage == 2) {
    L.sq = L.plane;
    L.sz = (size_t)19 * L.plane;
  } else {
    L.sq = (uint32_t)((size_t)L.plane * (uint32_t)n[2]);
    L.sz = L.plane;
  }
  return L;
}

template <bool PLANE = false>
__host__ __device__ inline UAddrT<PLANE> uaddr(const SweepParams& p) {
  UAddrT<PLANE> a;
  a.n[0] = p.nx; a.n[1] = p.ny; a.n[2] = p.nz;
  for (int i = 0; i < 3; ++i) a.per[i] = p.per[i];
  a.lay.sq = p.sq;
  a.lay.plane = (uint32_t)p.nx * (uint32_t)p.ny;
  a.lay.sz = p.sz;
  const uint32_t d = a.lay.plane;
  uint32_t l = 0;
  while (l < 32 && ((uint64_t)1 << l) < d) ++l;   // ceil(log2 d)
  a.zm = (uint32_t)((((uint64_t)1 << 32) * (((uint64_t)1 << l) - d)) / d + 1);
  a.zs1 = l < 1 ? l : 1;
  a.zs2 = l > 0 ? l - 1 : 0;
  return a;
}

// Workgroups per sphere of the link-cell pass; each owns one force/torque
// slot of kSlotWords doubles: the deviation parts of force and torque, then
// the integer sums K and L x K of the weight constants (see boundary_cell).
constexpr int kLinkGroups = 32;
constexpr int kSlotWords = 12;
inline int link_chunks(int box) { return (box * box * box + 255) / 256; }

// Per-sphere lists of link cells in box order: counts per 256-cell chunk of
// the box, box indices (box^3 per sphere), list lengths.  Rebuilt after
// every (re-)mapping.
struct LinkLists {
  int* count;
  uint32_t* links;
  int* len;
};

struct UpdateParams {
  double g[3];
  int step;
  int hist_len;
  int np;
};

// interior sweep (cells without links); e0/e1, if given, are recorded
// around it
template <typename S>
hipError_t launch_interior(const void* src, void* dst, const uint8_t* flags, int* status, const SweepParams& p,
                           bool with_flags, hipStream_t st, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// particle-link and wall-link cells; writes cells disjoint from the
// interior sweep, so both may run concurrently.  scan: find the particle
// link cells in each sphere's box (k_link_cells, one force slot per 256 box
// cells) instead of reading the link lists (kLinkGroups slots per sphere)
template <typename S>
hipError_t launch_boundary(const void* src, void* dst, const uint8_t* flags, const uint16_t* owner,
                           const DevParticle* parts, int np, const LinkLists& ll, double* slots, int* status,
                           const SweepParams& p, hipStream_t st, bool scan = false);
template <typename S>
hipError_t launch_init(void* dst, const uint8_t* flags, const double* u0, double drho, const SweepParams& p,
                       hipStream_t st);
hipError_t launch_map_all(uint8_t* flags, uint16_t* owner, const DevParticle* parts, int np,
                          const LinkLists& ll, const SweepParams& p, int* status, hipStream_t st);
// re-mapping and refill; the link lists are rebuilt unless the boundary
// pass scans the boxes (scan)
template <typename S>
hipError_t launch_refill_remap(void* state, uint8_t* flags, uint16_t* owner, const DevParticle* parts, int np,
                               const LinkLists& ll, const SweepParams& p, int* status, hipStream_t st,
                               bool scan = false);
// plain device copy of bytes (a multiple of 16): the bandwidth reference
hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t st);
// the interior sweep's access pattern without arithmetic (a bandwidth
// reference): dst[q][c] = src[q][c - c_q] on a periodic n[0] x n[1] x n[2]
// box of storage format `storage`, in that format's population layout
hipError_t launch_stream_pull(void* dst, const void* src, int storage, const int n[3], hipStream_t st);
// per-sphere force/torque reduction and particle update (Algorithm 1)
hipError_t launch_reduce_update(DevParticle* parts, int np, const double* slots, double* hist, int* status,
                                const SweepParams& p, const UpdateParams& u, hipStream_t st);


}  // namespace vm
