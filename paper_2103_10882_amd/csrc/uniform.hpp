// Launch parameters and launchers of the uniform-grid kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "common.hpp"

namespace vm {

struct SweepParams {
  int nx, ny, nz;
  int per[3];
  int wall_axis;          // first non-periodic axis or -1
  double wall_v[2][3];    // velocity of its low / high wall
  double sp, sm;          // s+ = omega, s- from the magic parameter
  double F[3];            // fluid body force
  uint32_t N;             // cells
  int box;                // force-slot box edge (cells)
  int slot_wx;            // x-waves per box row
  int nwx;                // x-waves per grid row
  size_t slot_stride;     // doubles per particle in the slot array
};

struct UpdateParams {
  double g[3];
  int step;
  int hist_len;
  int np;
};

template <typename S>
hipError_t launch_sweep(const void* src, void* dst, const uint8_t* flags, const uint16_t* owner,
                        const DevParticle* parts, double* slots, int* status, const SweepParams& p,
                        bool with_flags, hipStream_t st);
template <typename S>
hipError_t launch_init(void* dst, const uint8_t* flags, const double* u0, double drho, const SweepParams& p,
                       hipStream_t st);
hipError_t launch_map_all(uint8_t* flags, uint16_t* owner, const DevParticle* parts, int np,
                          const SweepParams& p, hipStream_t st);
template <typename S>
hipError_t launch_refill_remap(void* state, uint8_t* flags, uint16_t* owner, const DevParticle* parts, int np,
                               const SweepParams& p, hipStream_t st);
hipError_t launch_reduce_update(DevParticle* parts, int np, double* slots, double* hist, int* status,
                                const SweepParams& p, const UpdateParams& u, hipStream_t st);

}  // namespace vm
