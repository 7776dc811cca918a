// Uniform-grid kernels: fused pull stream-collide sweep with the moving-wall
// CLI boundary and momentum-exchange link forces on particle links, refill
// of uncovered cells, and re-mapping.  The per-particle reduction and update
// are in motion.hpp.
//
// Layout: populations as deviations in storage type S, element (q, x, y, z)
// at q sq + z sz + y nx + x (PopLayout: [q][z][y][x], or [z][q][y][x] for
// FP16), two buffers (pull from src, write dst); flags uint8 [z][y][x];
// owner uint16 [z][y][x] (read only for solid cells).  One thread per cell,
// one wave per 64 consecutive x cells of a row, so every population load and
// store of a wave is a contiguous run shifted by at most one element.
#include <type_traits>
#include <utility>

#include "common.hpp"
#include "uniform.hpp"
#include "stencil.hpp"
#include "particle.hpp"
#include "context.hpp"

namespace vm {

namespace {

// Interior sweep: every fluid cell without a wall or particle link.  Cells
// with a nonzero flag are left to the boundary kernels below (solid cells are
// not computed at all), so this kernel carries only the streaming pull and
// the collision and keeps its register footprint small.
//
// Addressing: a workgroup holds one row segment, so the source row and plane
// of every direction (periodic wrap included) are workgroup-uniform.  Each
// load and store is a uniform base (population and row) plus one of three
// per-lane x offsets, so the address arithmetic stays in scalar registers.
// a workgroup-uniform global pointer, held in scalar registers
typedef __attribute__((address_space(1))) char gchar;
__device__ __forceinline__ gchar* uniform_ptr(char* p) {
  const uint64_t v = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (gchar*)(((uint64_t)hi << 32) | lo);
}

// sq: population stride; pm, p0, pp: offsets of planes z-1, z, z+1
template <typename S, int Q>
__device__ __forceinline__ void pull_row(const S* __restrict__ src, uint32_t sq, uint32_t rm, uint32_t r0,
                                         uint32_t rp, size_t pm, size_t p0, size_t pp, uint32_t xm,
                                         uint32_t x, uint32_t xp, typename Store<S>::T (&d)[kQ]) {
  constexpr int cx = cx_of(Q), cy = cy_of(Q), cz = cz_of(Q);
  const uint32_t ys = cy == 1 ? rm : (cy == -1 ? rp : r0);
  const size_t zs = cz == 1 ? pm : (cz == -1 ? pp : p0);
  const char* __restrict__ row = reinterpret_cast<const char*>(src + ((size_t)Q * sq + zs + ys));
  const uint32_t xb = (cx == 1 ? xm : (cx == -1 ? xp : x)) * (uint32_t)sizeof(S);   // byte offset, 32 bits
  d[Q] = Store<S>::load(*reinterpret_cast<const S*>(row + xb));
}

template <typename S, int... Qs>
__device__ __forceinline__ void pull_rows(const S* __restrict__ src, uint32_t sq, uint32_t rm, uint32_t r0,
                                          uint32_t rp, size_t pm, size_t p0, size_t pp, uint32_t xm,
                                          uint32_t x, uint32_t xp, typename Store<S>::T (&d)[kQ],
                                          std::integer_sequence<int, Qs...>) {
  (pull_row<S, Qs>(src, sq, rm, r0, rp, pm, p0, pp, xm, x, xp, d), ...);
}

// A workgroup is RY row segments of BX cells (RY consecutive rows of one
// plane); each wave lies within one row, so its row is wave-uniform.
template <typename S, bool FLAGS, bool MRT, int BX, int RY>
__global__ __launch_bounds__(BX * RY) void k_sweep(const S* __restrict__ src, S* __restrict__ dst,
                                                   const uint8_t* __restrict__ flags, int* __restrict__ status,
                                                   SweepParams p) {
  using T = typename Store<S>::T;
  static_assert(BX % 64 == 0, "row segments are whole waves");
  const uint32_t x = blockIdx.x * BX + (RY == 1 ? threadIdx.x : threadIdx.x % BX);
  const int y = RY == 1 ? blockIdx.y
                        : (int)__builtin_amdgcn_readfirstlane(blockIdx.y * RY + threadIdx.x / BX);
  const int z = blockIdx.z;
  if (x >= (uint32_t)p.nx || y >= p.ny) return;
  const uint32_t nx = p.nx;
  const uint32_t plane = nx * p.ny;
  const uint32_t c = (uint32_t)z * plane + (uint32_t)y * nx + x;
  if (FLAGS && flags[c] != 0) return;
  const uint32_t ym = y == 0 ? p.ny - 1 : y - 1, yp = y + 1 == p.ny ? 0 : y + 1;
  const uint32_t zm = z == 0 ? p.nz - 1 : z - 1, zp = z + 1 == p.nz ? 0 : z + 1;
  const uint32_t xm = x == 0 ? nx - 1 : x - 1, xp = x + 1 == nx ? 0 : x + 1;
  T d[kQ];
  pull_rows<S>(src, p.sq, ym * nx, (uint32_t)y * nx, yp * nx, (size_t)zm * p.sz, (size_t)z * p.sz,
               (size_t)zp * p.sz, xm, x, xp, d, std::make_integer_sequence<int, kQ>{});
  const T drho = lbm_collide<T, MRT>(d, T(p.sp), T(p.sm), T(p.sb), T(p.F[0]), T(p.F[1]), T(p.F[2]));
  if (!(drho == drho)) status[kStatusUnstable] = 1;
  // streaming stores: the new state is not read again within this sweep
  SrBits rb(c, p.seed);
  const uint32_t xb = x * (uint32_t)sizeof(S);
  const size_t row0 = (size_t)z * p.sz + (uint32_t)y * nx;
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    // the row base is workgroup-uniform; stating it so keeps the compiler
    // from folding it into a per-lane 64-bit address
    gchar* out = uniform_ptr(reinterpret_cast<char*>(dst + ((size_t)q * p.sq + row0)));
    store_nt_g(out + xb, Store<S>::store_sr(d[q], rb.next()));
  }
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
  const UAddrOf<S> ad = uaddr<sizeof(S) == 2>(p);
  boundary_cell<S, UAddrOf<S>>(src, flags, owner, parts, p, ad, r[0], r[1], r[2], c, d, pid, Fl, Tl, Kl, Bl,
                               status);
  const T drho = lbm_collide<T>(d, T(p.sp), T(p.sm), T(p.sb), T(p.F[0]), T(p.F[1]), T(p.F[2]));
  if (!(drho == drho)) status[kStatusUnstable] = 1;
  SrBits rb(c, p.seed);
#pragma unroll
  for (int q = 0; q < kQ; ++q) dst[ad.pop(q, c)] = Store<S>::store_sr(d[q], rb.next());
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
  const UAddrOf<S> ad = uaddr<sizeof(S) == 2>(p);
#pragma unroll
  for (int q = 0; q < kQ; ++q) dst[ad.pop(q, c)] = Store<S>::store_sr(d[q], rb.next());
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
// slots of a block level, whose populations are blocked)
template <typename S>
__global__ __launch_bounds__(256) void k_totals(const S* __restrict__ pdf, const uint8_t* __restrict__ flags,
                                                PopLayout lay, uint32_t cells, const int* __restrict__ slots,
                                                int nslots, double* __restrict__ part) {
  double v[5] = {0, 0, 0, 0, 0};
  const uint32_t total = slots ? (uint32_t)nslots * 4096u : cells;
  for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
    const uint32_t c = slots ? (uint32_t)slots[t >> 12] * 4096u + (t & 4095u) : t;
    if (flags && (flags[c] & kSolid)) continue;
    v[0] += 1.0;
    for (int q = 0; q < kQ; ++q) {
      const double d = (double)Store<S>::load(pdf[slots ? bpop(q, c) : lay.pop(q, c)]);
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

// plain copy, one 16-byte load and one streaming 16-byte store per thread
typedef float vec4f __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void k_stream_copy(const vec4f* __restrict__ src, vec4f* __restrict__ dst,
                                                     size_t n) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) __builtin_nontemporal_store(src[i], &dst[i]);
}

// Bandwidth reference with the interior sweep's memory access pattern and
// no arithmetic: per cell of a periodic box in the sweep's population layout
// for this storage format, population q pulled from the neighbour at
// x - c_q and stored, one thread per cell, streaming stores.
template <typename S>
__global__ __launch_bounds__(256) void k_stream_pull(const S* __restrict__ src, S* __restrict__ dst, int nx, int ny,
                                                     int nz, PopLayout lay) {
  const int x = blockIdx.x * 256 + threadIdx.x, y = blockIdx.y, z = blockIdx.z;
  if (x >= nx) return;
  S d[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    int xs = x - cx_of(q), ys = y - cy_of(q), zs = z - cz_of(q);
    xs = xs < 0 ? xs + nx : (xs >= nx ? xs - nx : xs);
    ys = ys < 0 ? ys + ny : (ys >= ny ? ys - ny : ys);
    zs = zs < 0 ? zs + nz : (zs >= nz ? zs - nz : zs);
    d[q] = src[(size_t)q * lay.sq + (size_t)zs * lay.sz + (size_t)ys * nx + xs];
  }
  const size_t row = (size_t)z * lay.sz + (size_t)y * nx + x;
#pragma unroll
  for (int q = 0; q < kQ; ++q) store_nt(&dst[(size_t)q * lay.sq + row], d[q]);
}

// one workgroup per sphere: force/torque reduction and particle update
__global__ __launch_bounds__(256) void k_reduce_update(DevParticle* __restrict__ parts, const double* __restrict__ slots,
                                                       double* __restrict__ hist, int* __restrict__ status,
                                                       SweepParams p, UpdateParams u) {
  reduce_update(parts, slots, hist, status, p, u, blockIdx.x);
}

}  // namespace

hipError_t launch_totals(int storage, const void* pdf, const uint8_t* flags, const PopLayout& lay, uint32_t cells,
                         const int* slot_list, int nslots, double* partials, hipStream_t st) {
  if (storage == 0)
    k_totals<double><<<kTotalsGroups, 256, 0, st>>>((const double*)pdf, flags, lay, cells, slot_list, nslots,
                                                    partials);
  else if (storage == 1)
    k_totals<float><<<kTotalsGroups, 256, 0, st>>>((const float*)pdf, flags, lay, cells, slot_list, nslots,
                                                   partials);
  else
    k_totals<__half><<<kTotalsGroups, 256, 0, st>>>((const __half*)pdf, flags, lay, cells, slot_list, nslots,
                                                    partials);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#ifndef VM_SWEEP_F64
#define VM_SWEEP_F64 128, 2
#endif
#ifndef VM_SWEEP_F32
#define VM_SWEEP_F32 256, 1
#endif
#ifndef VM_SWEEP_F16
#define VM_SWEEP_F16 512, 1
#endif
template <int B, int R> struct Shape { static constexpr int bx = B, ry = R; };
template <typename S> struct SweepShape;
template <> struct SweepShape<double> : Shape<VM_SWEEP_F64> {};
template <> struct SweepShape<float> : Shape<VM_SWEEP_F32> {};
template <> struct SweepShape<__half> : Shape<VM_SWEEP_F16> {};

template <typename S>
hipError_t launch_interior(const void* src, void* dst, const uint8_t* flags, int* status, const SweepParams& p,
                           bool with_flags, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  // One workgroup per RY row segments of BX cells: the x-shifted loads of a
  // segment stay within one workgroup's cache lines.  Shapes by measurement
  // on 512^3 (per storage format: the segment length, rows per workgroup);
  // rows shorter than BX take one segment of whole waves.
  constexpr int BX = SweepShape<S>::bx, RY = SweepShape<S>::ry;
  if (e0) {
    hipError_t er = hipEventRecord(e0, st);
    if (er != hipSuccess) return er;
  }
  const bool mrt = p.sb != p.sp;
  if (p.nx >= BX) {
    dim3 grid((p.nx + BX - 1) / BX, (p.ny + RY - 1) / RY, p.nz), block(BX * RY);
    if (with_flags && mrt)
      k_sweep<S, true, true, BX, RY><<<grid, block, 0, st>>>((const S*)src, (S*)dst, flags, status, p);
    else if (with_flags)
      k_sweep<S, true, false, BX, RY><<<grid, block, 0, st>>>((const S*)src, (S*)dst, flags, status, p);
    else if (mrt)
      k_sweep<S, false, true, BX, RY><<<grid, block, 0, st>>>((const S*)src, (S*)dst, flags, status, p);
    else
      k_sweep<S, false, false, BX, RY><<<grid, block, 0, st>>>((const S*)src, (S*)dst, flags, status, p);
  } else {
    // short rows: one segment of whole waves per row (at most 512 cells)
    dim3 grid(1, p.ny, p.nz), block(((p.nx + 63) / 64) * 64);
    if (with_flags && mrt)
      k_sweep<S, true, true, 512, 1><<<grid, block, 0, st>>>((const S*)src, (S*)dst, flags, status, p);
    else if (with_flags)
      k_sweep<S, true, false, 512, 1><<<grid, block, 0, st>>>((const S*)src, (S*)dst, flags, status, p);
    else if (mrt)
      k_sweep<S, false, true, 512, 1><<<grid, block, 0, st>>>((const S*)src, (S*)dst, flags, status, p);
    else
      k_sweep<S, false, false, 512, 1><<<grid, block, 0, st>>>((const S*)src, (S*)dst, flags, status, p);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && e1) e = hipEventRecord(e1, st);
  return e;
}

template <typename S>
hipError_t launch_boundary(const void* src, void* dst, const uint8_t* flags, const uint16_t* owner,
                           const DevParticle* parts, int np, const LinkLists& ll, double* slots, int* status,
                           const SweepParams& p, hipStream_t st, bool scan) {
  hipError_t e = hipSuccess;
  if (np > 0 && scan) {
    k_link_cells<S, UAddrOf<S>><<<dim3(link_chunks(p.box), np), dim3(256), 0, st>>>(
        (const S*)src, (S*)dst, flags, owner, parts, slots, status, p, uaddr<sizeof(S) == 2>(p));
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  } else if (np > 0) {
    k_boundary_particles<S, UAddrOf<S>><<<dim3(kLinkGroups, np), dim3(256), 0, st>>>(
        (const S*)src, (S*)dst, flags, owner, parts, ll.links, ll.len, slots, status, p, uaddr<sizeof(S) == 2>(p));
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

hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t st) {
  const size_t n = bytes / 16;
  if (n) k_stream_copy<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st>>>((const vec4f*)src, (vec4f*)dst, n);
  return hipGetLastError();
}

hipError_t launch_stream_pull(void* dst, const void* src, int storage, const int n[3], hipStream_t st) {
  const dim3 grid((unsigned)((n[0] + 255) / 256), (unsigned)n[1], (unsigned)n[2]);
  const PopLayout lay = pop_layout(storage, n);
  if (storage == 0)
    k_stream_pull<double><<<grid, 256, 0, st>>>((const double*)src, (double*)dst, n[0], n[1], n[2], lay);
  else if (storage == 1)
    k_stream_pull<float><<<grid, 256, 0, st>>>((const float*)src, (float*)dst, n[0], n[1], n[2], lay);
  else
    k_stream_pull<__half><<<grid, 256, 0, st>>>((const __half*)src, (__half*)dst, n[0], n[1], n[2], lay);
  return hipGetLastError();
}

hipError_t launch_reduce_update(DevParticle* parts, int np, const double* slots, double* hist, int* status,
                                const SweepParams& p, const UpdateParams& u, hipStream_t st) {
  k_reduce_update<<<dim3(np), dim3(256), 0, st>>>(parts, slots, hist, status, p, u);
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
                               const LinkLists& ll, const SweepParams& p, int* status, hipStream_t st, bool scan) {
  const int rb = p.box + 1;
  dim3 grid(2 * ((rb * rb * rb + 255) / 256), np), block(256);
  k_refill_remap<S, UAddrOf<S>><<<grid, block, 0, st>>>((S*)state, flags, owner, parts, np, p,
                                                        uaddr<sizeof(S) == 2>(p), status);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || scan) return e;
  return launch_link_lists<UAddr>(flags, owner, parts, np, p, uaddr(p), ll.count, ll.links, ll.len, st);
}

template hipError_t launch_interior<double>(const void*, void*, const uint8_t*, int*, const SweepParams&, bool,
                                            hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_boundary<double>(const void*, void*, const uint8_t*, const uint16_t*, const DevParticle*,
                                            int, const LinkLists&, double*, int*, const SweepParams&, hipStream_t, bool);
template hipError_t launch_interior<float>(const void*, void*, const uint8_t*, int*, const SweepParams&, bool,
                                            hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_boundary<float>(const void*, void*, const uint8_t*, const uint16_t*, const DevParticle*,
                                           int, const LinkLists&, double*, int*, const SweepParams&, hipStream_t, bool);
template hipError_t launch_interior<__half>(const void*, void*, const uint8_t*, int*, const SweepParams&, bool,
                                            hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_boundary<__half>(const void*, void*, const uint8_t*, const uint16_t*, const DevParticle*,
                                            int, const LinkLists&, double*, int*, const SweepParams&, hipStream_t, bool);
template hipError_t launch_init<double>(void*, const uint8_t*, const double*, double, const SweepParams&, hipStream_t);
template hipError_t launch_init<float>(void*, const uint8_t*, const double*, double, const SweepParams&, hipStream_t);
template hipError_t launch_init<__half>(void*, const uint8_t*, const double*, double, const SweepParams&, hipStream_t);
template hipError_t launch_refill_remap<double>(void*, uint8_t*, uint16_t*, const DevParticle*, int,
                                                const LinkLists&, const SweepParams&, int*, hipStream_t, bool);
template hipError_t launch_refill_remap<float>(void*, uint8_t*, uint16_t*, const DevParticle*, int,
                                               const LinkLists&, const SweepParams&, int*, hipStream_t, bool);
template hipError_t launch_refill_remap<__half>(void*, uint8_t*, uint16_t*, const DevParticle*, int,
                                                const LinkLists&, const SweepParams&, int*, hipStream_t, bool);

}  // namespace vm
