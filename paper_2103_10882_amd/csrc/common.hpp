// Shared device definitions for the vmlbm kernels (gfx950, wave64).
//
// Populations are stored as deviations d = f - w_q from the lattice weights
// (rho0 = 1), in FP64, FP32 or FP16; collision arithmetic runs in FP64 for
// FP64 storage and in FP32 otherwise.  Forces, torques and particle state are
// always FP64.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <cstdint>

namespace vm {

// D3Q19 in the library's canonical order (Sec. 2.1 names D3Q19 without
// printing it): rest; +x,-x,+y,-y,+z,-z; (1,1,0),(1,-1,0),(-1,1,0),(-1,-1,0);
// (1,0,1),(1,0,-1),(-1,0,1),(-1,0,-1); (0,1,1),(0,1,-1),(0,-1,1),(0,-1,-1).
constexpr int kQ = 19;
__device__ __host__ constexpr int cx_of(int q) {
  return (q == 1 || q == 7 || q == 8 || q == 11 || q == 12) ? 1
       : (q == 2 || q == 9 || q == 10 || q == 13 || q == 14) ? -1 : 0;
}
__device__ __host__ constexpr int cy_of(int q) {
  return (q == 3 || q == 7 || q == 9 || q == 15 || q == 16) ? 1
       : (q == 4 || q == 8 || q == 10 || q == 17 || q == 18) ? -1 : 0;
}
__device__ __host__ constexpr int cz_of(int q) {
  return (q == 5 || q == 11 || q == 13 || q == 15 || q == 17) ? 1
       : (q == 6 || q == 12 || q == 14 || q == 16 || q == 18) ? -1 : 0;
}
__device__ __host__ constexpr int opp_of(int q) {
  return q == 0 ? 0 : (q <= 6 ? (q & 1 ? q + 1 : q - 1)
       : (q == 7 ? 10 : q == 10 ? 7 : q == 8 ? 9 : q == 9 ? 8
       : q == 11 ? 14 : q == 14 ? 11 : q == 12 ? 13 : q == 13 ? 12
       : q == 15 ? 18 : q == 18 ? 15 : q == 16 ? 17 : 16));
}
__device__ __host__ constexpr double w_of(int q) {
  return q == 0 ? 1.0 / 3.0 : (q <= 6 ? 1.0 / 18.0 : 1.0 / 36.0);
}
// the nine (q, opp(q)) pairs with q the member of positive orientation
constexpr int kPairs = 9;
__device__ __host__ constexpr int pair_q(int k) {
  return k == 0 ? 1 : k == 1 ? 3 : k == 2 ? 5 : k == 3 ? 7 : k == 4 ? 8 : k == 5 ? 11 : k == 6 ? 12 : k == 7 ? 15 : 16;
}

// cell flags (uint8 per cell)
constexpr uint8_t kSolid = 0x80;   // covered by a particle (owner array holds which)
constexpr uint8_t kNearP = 0x40;   // fluid cell with a particle link (owner array holds which)
constexpr uint8_t kNearW = 0x20;   // fluid cell with a wall link

// status words in device memory
constexpr int kStatusUnstable = 0;  // non-finite density / force / torque
constexpr int kStatusRange = 1;     // particle moved too fast / links to two particles from one cell
constexpr int kStatusWords = 16;
constexpr int kHistWords = 15;     // per sphere and step: F, T, x, u, w

// ---------------------------------------------------------------------------
// storage precision: load/store of deviations
// ---------------------------------------------------------------------------
// Random bits for stochastic rounding: one counter-based stream per (cell,
// sweep).  An integer hash of the cell index and the sweep's seed (the
// "lowbias32" mixer of C. Wellons' hash-prospector) starts a Weyl sequence
// (increment 2^32 / golden ratio) advanced once per stored population.  Each
// value is uniform on its own, which is what unbiased rounding needs, and a
// step costs one integer add instead of a quarter-rate 32-bit multiply.
__host__ __device__ __forceinline__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return x;
}
struct SrBits {
  uint32_t h;
  __device__ __forceinline__ SrBits(uint32_t cell, uint32_t seed) : h(mix32(cell ^ mix32(seed + 0x9e3779b9u))) {}
  __device__ __forceinline__ uint32_t next() {
    h += 0x9e3779b9u;
    return h;
  }
};

// FP32 -> FP16 rounding up or down with probability proportional to the
// distance to the two neighbours (unbiased in expectation).  r: 32 random
// bits.  gfx950's v_cvt_sr_f16_f32 does this in one instruction, taking the
// uniform variate from the high bits of r, for normal and subnormal results
// alike (measured: a mean over 2^16 words of each value reproduces it to the
// 2^-16 quantisation of the variate).
__device__ __forceinline__ __half half_sr(float v, uint32_t r) {
  typedef _Float16 h2 __attribute__((ext_vector_type(2)));
  const h2 zero = {(_Float16)0.0f, (_Float16)0.0f};
  const h2 h = __builtin_amdgcn_cvt_sr_f16_f32(zero, v, r, false);
  return __ushort_as_half(__builtin_bit_cast(unsigned short, h[0]));
}

// Storage formats (reduced-precision storage is not part of the paper's
// method): the stored value is the deviation d = f - w, T the arithmetic
// type.  store() rounds to nearest and serves exact copies; store_sr() is
// used wherever a new value is produced (for FP16 the bias of rounding to
// nearest accumulates over steps when per-step changes are near half an FP16
// ulp, as the body-force increments are).
template <typename S> struct Store;
template <> struct Store<double> {
  using T = double;
  static __device__ __forceinline__ double load(double v) { return v; }
  static __device__ __forceinline__ double store(double v) { return v; }
  static __device__ __forceinline__ double store_sr(double v, uint32_t) { return v; }
};
template <> struct Store<float> {
  using T = float;
  static __device__ __forceinline__ float load(float v) { return v; }
  static __device__ __forceinline__ float store(float v) { return v; }
  static __device__ __forceinline__ float store_sr(float v, uint32_t) { return v; }
};
template <> struct Store<__half> {
  using T = float;
  static __device__ __forceinline__ float load(__half v) { return __half2float(v); }
  static __device__ __forceinline__ __half store(float v) { return __float2half_rn(v); }
  static __device__ __forceinline__ __half store_sr(float v, uint32_t r) { return half_sr(v, r); }
};

// streaming (nontemporal) store of one stored population
template <typename S>
__device__ __forceinline__ void store_nt(S* p, S v) {
  __builtin_nontemporal_store(v, p);
}
template <>
__device__ __forceinline__ void store_nt<__half>(__half* p, __half v) {
  __builtin_nontemporal_store(__half_as_ushort(v), reinterpret_cast<unsigned short*>(p));
}
// the same through a global (address space 1) byte pointer
template <typename S>
__device__ __forceinline__ void store_nt_g(__attribute__((address_space(1))) char* p, S v) {
  __builtin_nontemporal_store(v, (__attribute__((address_space(1))) S*)p);
}
template <>
__device__ __forceinline__ void store_nt_g<__half>(__attribute__((address_space(1))) char* p, __half v) {
  __builtin_nontemporal_store(__half_as_ushort(v), (__attribute__((address_space(1))) unsigned short*)p);
}

// ---------------------------------------------------------------------------
// Collision of Sec. 2.1 on deviations, incompressible equilibrium (rho0 = 1),
// forcing after Guo with the velocity shifted by F/2: odd non-equilibrium
// relaxed with s-, even with s+ = s_nu (TRT), except its isotropic part
// (the mean over each speed shell: rest, axis, diagonal), which the MRT of
// Sec. 2.1 relaxes with s_b; the even source is weighted likewise with
// 1 - s/2.  sb == sp gives TRT.  d[] holds pre-collision deviations on
// entry and post-collision on exit.  Returns the density deviation.
// ---------------------------------------------------------------------------
// MRT = false drops the shell-mean terms, which vanish for sb == sp (TRT).
template <typename T, bool MRT = true>
__device__ __forceinline__ T lbm_collide(T (&d)[kQ], T sp, T sm, T sb, T Fx, T Fy, T Fz) {
  T drho = d[0];
#pragma unroll
  for (int q = 1; q < kQ; ++q) drho += d[q];
  const T jx = (d[1] - d[2]) + (d[7] - d[10]) + (d[8] - d[9]) + (d[11] - d[14]) + (d[12] - d[13]);
  const T jy = (d[3] - d[4]) + (d[7] - d[10]) + (d[9] - d[8]) + (d[15] - d[18]) + (d[16] - d[17]);
  const T jz = (d[5] - d[6]) + (d[11] - d[14]) + (d[13] - d[12]) + (d[15] - d[18]) + (d[17] - d[16]);
  const T ux = jx + T(0.5) * Fx, uy = jy + T(0.5) * Fy, uz = jz + T(0.5) * Fz;
  const T usq = ux * ux + uy * uy + uz * uz;
  const T uF = ux * Fx + uy * Fy + uz * Fz;
  if (!MRT) sb = sp;
  const T kp = T(1) - T(0.5) * sp, km = T(1) - T(0.5) * sm, kb = T(1) - T(0.5) * sb;
  // rest population: a shell of its own, so purely isotropic
  {
    const T w = T(w_of(0));
    const T eq = w * (drho - T(1.5) * usq);
    d[0] = d[0] - sb * (d[0] - eq) + kb * (w * (T(-3) * uF));
  }
  T fp[kPairs], ne[kPairs], se[kPairs];
  T nax = T(0), ndg = T(0), sax = T(0), sdg = T(0);
#pragma unroll
  for (int k = 0; k < kPairs; ++k) {
    const int q = pair_q(k), qb = opp_of(q);
    const T w = T(w_of(q));
    const T cu = T(cx_of(q)) * ux + T(cy_of(q)) * uy + T(cz_of(q)) * uz;
    const T cF = T(cx_of(q)) * Fx + T(cy_of(q)) * Fy + T(cz_of(q)) * Fz;
    const T ep = w * (drho + T(4.5) * cu * cu - T(1.5) * usq);
    const T em = T(3) * w * cu;
    const T Sp = w * (T(9) * cu * cF - T(3) * uF);
    const T Sm = T(3) * w * cF;
    fp[k] = T(0.5) * (d[q] + d[qb]);
    const T fm = T(0.5) * (d[q] - d[qb]);
    ne[k] = fp[k] - ep;
    se[k] = Sp;
    if (MRT) {
      if (k < 3) { nax += ne[k]; sax += Sp; } else { ndg += ne[k]; sdg += Sp; }
    }
    // odd part now; the even part below, once the shell means are known
    const T nm = fm - sm * (fm - em) + km * Sm;
    d[q] = nm;
    d[qb] = -nm;
  }
  // shell means of the even non-equilibrium and source (axis shell: 3 pairs,
  // diagonal shell: 6 pairs), relaxed at s_b instead of s_nu
  const T dsb = sb - sp, dkb = kb - kp;
  const T mn_ax = nax * T(1.0 / 3.0), mn_dg = ndg * T(1.0 / 6.0);
  const T ms_ax = sax * T(1.0 / 3.0), ms_dg = sdg * T(1.0 / 6.0);
#pragma unroll
  for (int k = 0; k < kPairs; ++k) {
    const int q = pair_q(k), qb = opp_of(q);
    const T mn = k < 3 ? mn_ax : mn_dg, ms = k < 3 ? ms_ax : ms_dg;
    const T np = MRT ? fp[k] - sp * ne[k] - dsb * mn + kp * se[k] + dkb * ms : fp[k] - sp * ne[k] + kp * se[k];
    d[q] = np + d[q];
    d[qb] = np + d[qb];
  }
  return drho;
}

// s_b from s_nu and the bulk factor Lambda_b (Sec. 2.1); 0 or 1 gives s_nu
__host__ __device__ inline double s_bulk_of(double snu, double bulk_factor) {
  if (!(bulk_factor > 0.0) || bulk_factor == 1.0) return snu;
  return 1.0 / (0.5 + bulk_factor * (1.0 / snu - 0.5));
}

// s- from s+ and the magic parameter Lambda = (1/s+ - 1/2)(1/s- - 1/2)
__host__ __device__ inline double s_minus_of(double sp, double magic) {
  return 1.0 / (0.5 + magic / (1.0 / sp - 0.5));
}

// ---------------------------------------------------------------------------
// sphere geometry, FP64 without contraction so that the solid/fluid decision
// is reproducible: a cell is solid iff |x_c - x_p|^2 <= r^2 (minimum image).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double min_image(double d, int n, int periodic) {
  if (periodic) {
    if (d > 0.5 * n) d = __dadd_rn(d, -(double)n);
    else if (d < -0.5 * n) d = __dadd_rn(d, (double)n);
  }
  return d;
}

__device__ __forceinline__ void sphere_offset(const double* xp, double px, double py, double pz,
                                              int nx, int ny, int nz, const int* per, double* d) {
  d[0] = min_image(__dadd_rn(px, -xp[0]), nx, per[0]);
  d[1] = min_image(__dadd_rn(py, -xp[1]), ny, per[1]);
  d[2] = min_image(__dadd_rn(pz, -xp[2]), nz, per[2]);
}

__device__ __forceinline__ bool inside_sphere(const double* d, double r) {
  double dd = __dmul_rn(d[0], d[0]);
  dd = __dadd_rn(dd, __dmul_rn(d[1], d[1]));
  dd = __dadd_rn(dd, __dmul_rn(d[2], d[2]));
  return dd <= __dmul_rn(r, r);
}

// boundary distance ratio along integer direction c from offset d (Sec. 2.3):
// smallest root of |d + delta c|^2 = r^2
__device__ __forceinline__ double ray_delta(const double* d, int cx, int cy, int cz, double r) {
  const double cc = cx * cx + cy * cy + cz * cz;
  const double dc = d[0] * cx + d[1] * cy + d[2] * cz;
  const double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  double disc = dc * dc - cc * (dd - r * r);
  disc = disc > 0.0 ? disc : 0.0;
  double delta = (-dc - sqrt(disc)) / cc;
  return delta < 0.0 ? 0.0 : (delta > 1.0 ? 1.0 : delta);
}

}  // namespace vm
