// Uniform-grid kernels: fused pull stream-collide sweep with the moving-wall
// CLI boundary and momentum-exchange link forces on particle links, refill
// of uncovered cells, and re-mapping.  The per-particle reduction and update
// are in motion.hip.
//
// Layout: populations SoA [q][z][y][x] as deviations in storage type S, two
// buffers (pull from src, write dst); flags uint8 [z][y][x]; owner uint16
// [z][y][x] (read only for solid cells).  One thread per cell, one wave per
// 64 consecutive x cells of a row, so every population load and store of a
// wave is a contiguous run shifted by at most one element.
#include <type_traits>
#include <utility>

#include "common.hpp"
#include "uniform.hpp"
#include "stencil.hpp"
#include "particle.hpp"
#include "context.hpp"

namespace vm {

namespace {

__host__ __device__ UAddr uaddr(const SweepParams& p) {
  UAddr a;
  a.n[0] = p.nx; a.n[1] = p.ny; a.n[2] = p.nz;
  for (int i = 0; i < 3; ++i) a.per[i] = p.per[i];
  a.N = p.N;
  return a;
}

// Interior sweep: every fluid cell without a wall or particle link.  Cells
// with a nonzero flag are left to the boundary kernels below (solid cells are
// not computed at all), so this kernel carries only the streaming pull and
// the collision and keeps its register footprint small.
template <typename S, bool FLAGS>
__global__ __launch_bounds__(512) void k_sweep(const S* __restrict__ src, S* __restrict__ dst,
                                               const uint8_t* __restrict__ flags, int* __restrict__ status,
                                               SweepParams p) {
  using T = typename Store<S>::T;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y, z = blockIdx.z;
  if (x >= p.nx) return;
  const uint32_t N = p.N;
  const uint32_t c = ((uint32_t)z * p.ny + y) * p.nx + x;
  if (FLAGS && flags[c] != 0) return;
  T d[kQ];
  const Idx I = make_idx(x, y, z, p.nx, p.ny, p.nz);
  load_all<S>(src, N, I, x, d, std::make_integer_sequence<int, kQ>{});
  const T drho = lbm_collide<T>(d, T(p.sp), T(p.sm), T(p.sb), T(p.F[0]), T(p.F[1]), T(p.F[2]));
  if (!(drho == drho)) status[kStatusUnstable] = 1;
  // streaming stores: the new state is not read again within this sweep
  SrBits rb(c, p.seed);
#pragma unroll
  for (int q = 0; q < kQ; ++q) store_nt(&dst[(size_t)q * N + c], Store<S>::store_sr(d[q], rb.next()));
}

// Wall-link cells without particle links: the two boundary planes of each
// non-periodic axis (a cell on planes of two axes is taken by the lower axis).
template <typename S>
__global__ __launch_bounds__(256) void k_boundary_walls(const S* __restrict__ src, S* __restrict__ dst,
                                                        const uint8_t* __restrict__ flags,
                                                        const uint16_t* __restrict__ owner,
                                                        const DevParticle* __restrict__ parts,
                                                        int* __restrict__ status, SweepParams p, int axis,
                                                        int side) {
  using T = typename Store<S>::T;
  const int n[3] = {p.nx, p.ny, p.nz};
  const int a1 = axis == 0 ? 1 : 0, a2 = axis == 2 ? 1 : 2;
  const int u = blockIdx.x * blockDim.x + threadIdx.x, v = blockIdx.y;
  if (u >= n[a1]) return;
  int r[3];
  r[axis] = side ? n[axis] - 1 : 0;
  r[a1] = u;
  r[a2] = v;
  for (int b = 0; b < axis; ++b)
    if (!p.per[b] && (r[b] == 0 || r[b] == n[b] - 1)) return;
  const uint32_t c = ((uint32_t)r[2] * p.ny + r[1]) * p.nx + r[0];
  const uint8_t fl = flags[c];
  if ((fl & kSolid) || (fl & kNearP) || !(fl & kNearW)) return;
  int pid = -1;
  double Fl[3] = {0.0, 0.0, 0.0}, Tl[3] = {0.0, 0.0, 0.0}, Kl[3] = {0.0, 0.0, 0.0}, Bl[3] = {0.0, 0.0, 0.0};
  T d[kQ];
  const UAddr ad = uaddr(p);
  boundary_cell<S, UAddr>(src, flags, owner, parts, p, ad, r[0], r[1], r[2], c, d, pid, Fl, Tl, Kl, Bl, status);
  const T drho = lbm_collide<T>(d, T(p.sp), T(p.sm), T(p.sb), T(p.F[0]), T(p.F[1]), T(p.F[2]));
  if (!(drho == drho)) status[kStatusUnstable] = 1;
  SrBits rb(c, p.seed);
#pragma unroll
  for (int q = 0; q < kQ; ++q) dst[(size_t)q * p.N + c] = Store<S>::store_sr(d[q], rb.next());
}

// ---------------------------------------------------------------------------
// f~(0) = collide(f^eq(rho, u0)) on fluid cells (Sec. 2.1)
// ---------------------------------------------------------------------------
template <typename S>
__global__ __launch_bounds__(256) void k_init(S* __restrict__ dst, const uint8_t* __restrict__ flags,
                                              const double* __restrict__ u0, double drho, SweepParams p) {
  using T = typename Store<S>::T;
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= p.N) return;
  if (flags && (flags[c] & kSolid)) return;
  double u[3] = {0.0, 0.0, 0.0};
  if (u0) { u[0] = u0[c]; u[1] = u0[p.N + c]; u[2] = u0[2 * (size_t)p.N + c]; }
  const double usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  T d[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const double cu = cx_of(q) * u[0] + cy_of(q) * u[1] + cz_of(q) * u[2];
    d[q] = T(w_of(q) * (drho + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq));
  }
  lbm_collide<T>(d, T(p.sp), T(p.sm), T(p.sb), T(p.F[0]), T(p.F[1]), T(p.F[2]));
  SrBits rb(c, p.seed);
#pragma unroll
  for (int q = 0; q < kQ; ++q) dst[(size_t)q * p.N + c] = Store<S>::store_sr(d[q], rb.next());
}

__global__ __launch_bounds__(256) void k_map_all(uint8_t* __restrict__ flags, uint16_t* __restrict__ owner,
                                                 const DevParticle* __restrict__ parts, int np, SweepParams p,
                                                 int* __restrict__ status) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= p.N) return;
  const int x = c % p.nx, y = (c / p.nx) % p.ny, z = c / ((uint32_t)p.nx * p.ny);
  map_cell<UAddr>(x, y, z, c, flags, owner, parts, np, p, uaddr(p), status);
}

// fixed-order partial sums over fluid cells: count, sum of deviations and
// their first moment; grid-stride over the cell range (or the listed 16^3
// slots of a block level)
template <typename S>
__global__ __launch_bounds__(256) void k_totals(const S* __restrict__ pdf, const uint8_t* __restrict__ flags,
                                                uint32_t N, uint32_t cells, const int* __restrict__ slots,
                                                int nslots, double* __restrict__ part) {
  double v[5] = {0, 0, 0, 0, 0};
  const uint32_t total = slots ? (uint32_t)nslots * 4096u : cells;
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
    const uint32_t c = slots ? (uint32_t)slots[t >> 12] * 4096u + (t & 4095u) : t;
    if (flags && (flags[c] & kSolid)) continue;
    v[0] += 1.0;
    for (int q = 0; q < kQ; ++q) {
      const double d = (double)Store<S>::load(pdf[(size_t)q * N + c]);
      v[1] += d;
      v[2] += cx_of(q) * d;
      v[3] += cy_of(q) * d;
      v[4] += cz_of(q) * d;
    }
  }
  __shared__ double red[5][4];
  for (int k = 0; k < 5; ++k) v[k] = wave_sum(v[k]);
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < 5; ++k) red[k][threadIdx.x >> 6] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < 5; ++k) part[8 * blockIdx.x + k] = red[k][0] + red[k][1] + red[k][2] + red[k][3];
}

}  // namespace

hipError_t launch_totals(int storage, const void* pdf, const uint8_t* flags, uint32_t N, uint32_t cells,
                         const int* slot_list, int nslots, double* partials, hipStream_t st) {
  if (storage == 0)
    k_totals<double><<<kTotalsGroups, 256, 0, st>>>((const double*)pdf, flags, N, cells, slot_list, nslots, partials);
  else if (storage == 1)
    k_totals<float><<<kTotalsGroups, 256, 0, st>>>((const float*)pdf, flags, N, cells, slot_list, nslots, partials);
  else
    k_totals<__half><<<kTotalsGroups, 256, 0, st>>>((const __half*)pdf, flags, N, cells, slot_list, nslots, partials);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename S>
hipError_t launch_interior(const void* src, void* dst, const uint8_t* flags, int* status, const SweepParams& p,
                           bool with_flags, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  // one workgroup per grid row segment: the x-shifted loads of a segment
  // stay within one workgroup's cache lines.  Segment length by measurement
  // on 512^3: 256 cells for FP32 and FP16 storage, whole 512-cell rows for
  // FP64.
  const int wmax = std::is_same<S, double>::value ? 512 : 256;
  const int bx = p.nx >= wmax ? wmax : ((p.nx + 63) / 64) * 64;
  dim3 grid((p.nx + bx - 1) / bx, p.ny, p.nz), block(bx);
  if (e0) {
    hipError_t er = hipEventRecord(e0, st);
    if (er != hipSuccess) return er;
  }
  if (with_flags)
    k_sweep<S, true><<<grid, block, 0, st>>>((const S*)src, (S*)dst, flags, status, p);
  else
    k_sweep<S, false><<<grid, block, 0, st>>>((const S*)src, (S*)dst, flags, status, p);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && e1) e = hipEventRecord(e1, st);
  return e;
}

template <typename S>
hipError_t launch_boundary(const void* src, void* dst, const uint8_t* flags, const uint16_t* owner,
                           const DevParticle* parts, int np, const LinkLists& ll, double* slots, int* status,
                           const SweepParams& p, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (np > 0) {
    k_boundary_particles<S, UAddr><<<dim3(kLinkGroups, np), dim3(256), 0, st>>>(
        (const S*)src, (S*)dst, flags, owner, parts, ll.links, ll.len, slots, status, p, uaddr(p));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int n[3] = {p.nx, p.ny, p.nz};
  for (int a = 0; a < 3; ++a) {
    if (p.per[a]) continue;
    const int a1 = a == 0 ? 1 : 0, a2 = a == 2 ? 1 : 2;
    for (int side = 0; side < 2; ++side) {
      if (side == 1 && n[a] == 1) break;
      k_boundary_walls<S><<<dim3((n[a1] + 63) / 64, n[a2]), dim3(64), 0, st>>>(
          (const S*)src, (S*)dst, flags, owner, parts, status, p, a, side);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

template <typename S>
hipError_t launch_init(void* dst, const uint8_t* flags, const double* u0, double drho, const SweepParams& p,
                       hipStream_t st) {
  dim3 grid((p.N + 255) / 256), block(256);
  k_init<S><<<grid, block, 0, st>>>((S*)dst, flags, u0, drho, p);
  return hipGetLastError();
}

hipError_t launch_map_all(uint8_t* flags, uint16_t* owner, const DevParticle* parts, int np,
                          const LinkLists& ll, const SweepParams& p, int* status, hipStream_t st) {
  dim3 grid((p.N + 255) / 256), block(256);
  k_map_all<<<grid, block, 0, st>>>(flags, owner, parts, np, p, status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_link_lists<UAddr>(flags, owner, parts, np, p, uaddr(p), ll.count, ll.links, ll.len, st);
}

template <typename S>
hipError_t launch_refill_remap(void* state, uint8_t* flags, uint16_t* owner, const DevParticle* parts, int np,
                               const LinkLists& ll, const SweepParams& p, int* status, hipStream_t st) {
  const int rb = p.box + 1;
  dim3 grid((rb * rb * rb + 255) / 256, np), block(256);
  k_refill<S, UAddr><<<grid, block, 0, st>>>((S*)state, flags, owner, parts, np, p, uaddr(p), status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_remap<UAddr><<<grid, block, 0, st>>>(flags, owner, parts, np, p, uaddr(p), status);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_link_lists<UAddr>(flags, owner, parts, np, p, uaddr(p), ll.count, ll.links, ll.len, st);
}

template hipError_t launch_interior<double>(const void*, void*, const uint8_t*, int*, const SweepParams&, bool,
                                            hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_boundary<double>(const void*, void*, const uint8_t*, const uint16_t*, const DevParticle*,
                                            int, const LinkLists&, double*, int*, const SweepParams&, hipStream_t);
template hipError_t launch_interior<float>(const void*, void*, const uint8_t*, int*, const SweepParams&, bool,
                                            hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_boundary<float>(const void*, void*, const uint8_t*, const uint16_t*, const DevParticle*,
                                            int, const LinkLists&, double*, int*, const SweepParams&, hipStream_t);
template hipError_t launch_interior<__half>(const void*, void*, const uint8_t*, int*, const SweepParams&, bool,
                                            hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_boundary<__half>(const void*, void*, const uint8_t*, const uint16_t*, const DevParticle*,
                                            int, const LinkLists&, double*, int*, const SweepParams&, hipStream_t);
template hipError_t launch_init<double>(void*, const uint8_t*, const double*, double, const SweepParams&, hipStream_t);
template hipError_t launch_init<float>(void*, const uint8_t*, const double*, double, const SweepParams&, hipStream_t);
template hipError_t launch_init<__half>(void*, const uint8_t*, const double*, double, const SweepParams&, hipStream_t);
template hipError_t launch_refill_remap<double>(void*, uint8_t*, uint16_t*, const DevParticle*, int,
                                                const LinkLists&, const SweepParams&, int*, hipStream_t);
template hipError_t launch_refill_remap<float>(void*, uint8_t*, uint16_t*, const DevParticle*, int,
                                               const LinkLists&, const SweepParams&, int*, hipStream_t);
template hipError_t launch_refill_remap<__half>(void*, uint8_t*, uint16_t*, const DevParticle*, int,
                                                const LinkLists&, const SweepParams&, int*, hipStream_t);

}  // namespace vm
