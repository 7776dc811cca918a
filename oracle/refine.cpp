// CPU oracle for the block-structured 2:1 refined grid -- TEST INFRASTRUCTURE.
//
// Plain FP64, one dense array per level (cells of that level covering the
// whole domain) with a kind per cell, written from Sec. 4.1-4.2 of the paper
// and the reading of the non-uniform LBM it cites (volumetric populations,
// homogeneous explosion, averaging coalescence, fine levels sub-cycled):
//
//  * level l has cell size 2^-l (coarse units); a block of b^3 cells is split
//    into 8 blocks of the next level; neighbouring blocks (26-neighbourhood)
//    differ by at most one level;
//  * post-collision populations are the stored state; relaxation per level
//    follows acoustic scaling, 1/omega_{l+1} - 1/2 = 2 (1/omega_l - 1/2),
//    Lambda fixed; body force F_l = F_L 2^(L-l);
//  * Step(l): explode level-l populations into the ghost band G_{l+1} of
//    level l+1 (fine cells of level-l cells within one level-l cell of the
//    level-(l+1) region); Step(l+1) twice, ghost cells streaming only; then
//    the level-l sweep, where a population streaming from a level-l cell C
//    into C' keeps the fraction (1 - n_in/8) that did not cut into the fine
//    region, and the fine populations that left the fine region into the
//    ghost cells of C' are added with weight 1/8 (reading of the cited
//    scheme at edges and corners; it conserves mass exactly);
//  * the particle lives on the finest level only; its coupling is the same
//    as on the uniform grid (Eqs. 10-12, Algorithm 1, Sec. 2.3);
//  * refinement criterion (Sec. 4.2.1): blocks near the particle are on the
//    finest level, others take the level of the static refine regions;
//    2:1 balance by splitting, one level at a time; checked every
//    check_every coarse steps,
//    data moved by copying a cell to its 8 children or averaging them.
// Domains are periodic in all directions.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

#include "core.hpp"

extern "C" {
typedef struct {
  int n0[3];
  int block;
  int levels;
  double omega;
  double magic;
  double body_force[3];
  double gravity[3];
  int check_every;
  double bulk_factor;   /* Lambda_b of the MRT collision; 0 or 1 = TRT */
  double curl_threshold; /* sigma_c of the curl sensor (Eq. 23); 0 = off */
  double curl_coarsen;   /* c: coarsen below c sigma_c */
} orf_config;

typedef struct {
  double x[3], u[3], w[3];
  double radius, density_ratio, cv, cv_omega;
  int fixed;
  int vm_scheme;
} orf_sphere;
}

namespace {
using namespace ora;

enum Kind : uint8_t { NONE = 0, INTERIOR = 1, GHOST = 2 };

struct RLevel {
  int n[3] = {0, 0, 0};
  long N = 0;
  std::vector<double> cur, nxt, pre;   // [19][N]
  std::vector<uint8_t> kind;
  double sp = 0, sm = 0, sb = 0, F[3] = {0, 0, 0};
  bool mrt = false;
  // TRT, or the MRT of Sec. 2.1 when the bulk factor differs from 1
  void coll(const double a[19], const double Fl[3], double o[19]) const {
    if (mrt) collide_mrt(a, sp, sm, sb, Fl, o);
    else collide(a, sp, sm, Fl, o);
  }
};

struct RForest {
  orf_config cfg{};
  int L = 0, b = 0;
  int nb[3] = {0, 0, 0};        // finest-level block grid
  std::vector<int> leaf, base;  // per finest block position
  std::vector<RLevel> lv;
  std::vector<Sph> sph;
  std::vector<int> own;         // finest level: -1 fluid, else sphere id
  long long coarse_steps = 0, fine_steps = 0;
  int refinements = 0;

  long bpos(int i, int j, int k) const { return ((long)k * nb[1] + j) * nb[0] + i; }
  int wrap(int v, int n) const { return ((v % n) + n) % n; }
  long idx(int l, int i, int j, int k) const {
    const RLevel& V = lv[l];
    return ((long)wrap(k, V.n[2]) * V.n[1] + wrap(j, V.n[1])) * V.n[0] + wrap(i, V.n[0]);
  }
  // leaf level of the region holding level-l cell (i,j,k)
  int leaf_of(int l, int i, int j, int k) const {
    const RLevel& V = lv[l];
    i = wrap(i, V.n[0]); j = wrap(j, V.n[1]); k = wrap(k, V.n[2]);
    const int s = L - l;
    return leaf[bpos((i << s) / b, (j << s) / b, (k << s) / b)];
  }
  uint8_t kind_at(int l, int i, int j, int k) const { return lv[l].kind[idx(l, i, j, k)]; }

  void compute_kinds() {
    for (int l = 0; l <= L; ++l) {
      RLevel& V = lv[l];
#pragma omp parallel for schedule(static)
      for (int k = 0; k < V.n[2]; ++k)
        for (int j = 0; j < V.n[1]; ++j)
          for (int i = 0; i < V.n[0]; ++i) {
            const long c = idx(l, i, j, k);
            const int lf = leaf_of(l, i, j, k);
            uint8_t kd = NONE;
            if (lf == l) kd = INTERIOR;
            else if (l >= 1 && lf == l - 1) {
              const int pi = i >> 1, pj = j >> 1, pk = k >> 1;
              for (int dz = -1; dz <= 1 && kd == NONE; ++dz)
                for (int dy = -1; dy <= 1 && kd == NONE; ++dy)
                  for (int dx = -1; dx <= 1 && kd == NONE; ++dx)
                    if (leaf_of(l - 1, pi + dx, pj + dy, pk + dz) == l) kd = GHOST;
            }
            V.kind[c] = kd;
          }
    }
  }

  // leaf level of every finest block position from target levels, refined
  // until leaves that touch (face, edge or corner) differ by at most one level
  // (Sec. 4.1).  Reading: a leaf that touches one more than a level deeper is
  // split once, and the check repeats, so no block is finer than the targets
  // and the 2:1 rule need.
  std::vector<int> balance(std::vector<int> t) const {
    const long NB = (long)nb[0] * nb[1] * nb[2];
    std::vector<int> lf(NB);
    auto leaves = [&]() {
      for (long p = 0; p < NB; ++p) lf[p] = 0;
      for (int l = 0; l <= L; ++l) {
        const int s = 1 << (L - l);   // node edge in finest block positions
        for (int k = 0; k < nb[2]; k += s)
          for (int j = 0; j < nb[1]; j += s)
            for (int i = 0; i < nb[0]; i += s) {
              int mx = 0;
              for (int c = 0; c < s; ++c)
                for (int bb = 0; bb < s; ++bb)
                  for (int a = 0; a < s; ++a) mx = std::max(mx, t[bpos(i + a, j + bb, k + c)]);
              if (mx > l)
                for (int c = 0; c < s; ++c)
                  for (int bb = 0; bb < s; ++bb)
                    for (int a = 0; a < s; ++a) lf[bpos(i + a, j + bb, k + c)] = l + 1;
            }
      }
    };
    for (;;) {
      leaves();
      bool changed = false;
      for (int k = 0; k < nb[2]; ++k)
        for (int j = 0; j < nb[1]; ++j)
          for (int i = 0; i < nb[0]; ++i) {
            const int l = lf[bpos(i, j, k)];
            const int s = 1 << (L - l);
            const int ni = (i / s) * s, nj = (j / s) * s, nk = (k / s) * s;   // leaf node origin
            // deepest leaf touching this one: the positions of the one-wide
            // shell around the leaf node
            int mx = 0;
            for (int c = -1; c <= s; ++c)
              for (int bb = -1; bb <= s; ++bb)
                for (int a = -1; a <= s; ++a) {
                  if (a >= 0 && a < s && bb >= 0 && bb < s && c >= 0 && c < s) continue;
                  mx = std::max(mx, lf[bpos(wrap(ni + a, nb[0]), wrap(nj + bb, nb[1]), wrap(nk + c, nb[2]))]);
                }
            if (mx > l + 1 && t[bpos(i, j, k)] < l + 1) {
              t[bpos(i, j, k)] = l + 1;
              changed = true;
            }
          }
      if (!changed) return lf;
    }
  }

  // with_flow: add the curl-sensor targets (at the layout checks; the
  // initial layout comes from the static regions and the spheres)
  std::vector<int> targets(bool with_flow = false) const {
    std::vector<int> t = base;
    // Sec. 4.2.1: blocks intersecting the sphere's bounding box grown by one
    // finest block edge are on the finest level (reading: the open box, so a
    // block that only touches its face is not included)
    for (const Sph& s : sph) {
      int lo[3], hi[3];
      for (int a = 0; a < 3; ++a) {
        lo[a] = (int)std::floor((s.x[a] - s.r - b) / b);
        hi[a] = (int)std::ceil((s.x[a] + s.r + b) / b) - 1;
      }
      for (int k = lo[2]; k <= hi[2]; ++k)
        for (int j = lo[1]; j <= hi[1]; ++j)
          for (int i = lo[0]; i <= hi[0]; ++i) t[bpos(wrap(i, nb[0]), wrap(j, nb[1]), wrap(k, nb[2]))] = L;
    }
    if (with_flow && cfg.curl_threshold > 0.0) {
      // Sec. 4.2.2: a leaf whose sensor exceeds sigma_c wants one level more,
      // one below c sigma_c one level less
      const std::vector<int> ft = flow_targets();
      for (size_t p = 0; p < t.size(); ++p) t[p] = std::max(t[p], ft[p]);
    }
    return t;
  }

  // fluid velocity of level-l cell c from the stored post-collision state:
  // u = sum_q c_q f~_q - F_l / 2 (level lattice units, equal to finest units
  // under acoustic scaling)
  void velocity(int l, long c, double u[3]) const {
    const RLevel& V = lv[l];
    double j[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < 19; ++q) {
      const double f = V.cur[q * V.N + c];
      j[0] += CX[q] * f;
      j[1] += CY[q] * f;
      j[2] += CZ[q] * f;
    }
    for (int a = 0; a < 3; ++a) u[a] = j[a] - 0.5 * V.F[a];
  }

  // Curl sensor of Eq. 23 per level-l block, max over its cells:
  // phi = |curl u| s^((r+1)/r), r = 2, s = cell edge in finest cells
  // (reading: lengths in finest-level lattice units, central differences
  // over the six axis neighbours of the level, evaluated where all six are
  // interior cells of the level and, on the finest level, fluid).  Blocks
  // without such a cell read 0; non-leaf blocks read -1.
  std::vector<double> block_sensor(int l) const {
    const RLevel& V = lv[l];
    const int bn[3] = {V.n[0] / b, V.n[1] / b, V.n[2] / b};
    std::vector<double> out((long)bn[0] * bn[1] * bn[2], -1.0);
    const double s = (double)(1 << (L - l));
    const double scale = s * std::sqrt(s) / (2.0 * s);   // s^(3/2) and 1/(2 s) of the differences
    for (int k = 0; k < V.n[2]; ++k)
      for (int j = 0; j < V.n[1]; ++j)
        for (int i = 0; i < V.n[0]; ++i) {
          const long bidx = ((long)(k / b) * bn[1] + j / b) * bn[0] + i / b;
          if (kind_at(l, i, j, k) != INTERIOR) continue;
          if (out[bidx] < 0.0) out[bidx] = 0.0;
          const long c = idx(l, i, j, k);
          if (l == L && !own.empty() && own[c] >= 0) continue;
          double du[3][2][3];   // axis, side, component
          bool ok = true;
          for (int a = 0; a < 3 && ok; ++a)
            for (int sd = 0; sd < 2 && ok; ++sd) {
              int p[3] = {i, j, k};
              p[a] += sd ? 1 : -1;
              if (kind_at(l, p[0], p[1], p[2]) != INTERIOR) { ok = false; break; }
              const long cn = idx(l, p[0], p[1], p[2]);
              if (l == L && !own.empty() && own[cn] >= 0) { ok = false; break; }
              velocity(l, cn, du[a][sd]);
            }
          if (!ok) continue;
          // d u_comp / d x_axis ~ (u(+) - u(-)) (scaled below)
          auto d = [&](int comp, int axis) { return du[axis][1][comp] - du[axis][0][comp]; };
          const double cx = d(2, 1) - d(1, 2), cy = d(0, 2) - d(2, 0), cz = d(1, 0) - d(0, 1);
          const double phi = std::sqrt(cx * cx + cy * cy + cz * cz) * scale;
          out[bidx] = std::max(out[bidx], phi);
        }
    return out;
  }

  std::vector<int> flow_targets() const {
    std::vector<int> t(leaf.size(), 0);
    const double sig = cfg.curl_threshold, csig = cfg.curl_coarsen * cfg.curl_threshold;
    for (int l = 0; l <= L; ++l) {
      const RLevel& V = lv[l];
      const int bn[3] = {V.n[0] / b, V.n[1] / b, V.n[2] / b};
      const std::vector<double> sens = block_sensor(l);
      const int sh = L - l;
      for (int k = 0; k < bn[2]; ++k)
        for (int j = 0; j < bn[1]; ++j)
          for (int i = 0; i < bn[0]; ++i) {
            const double v = sens[((long)k * bn[1] + j) * bn[0] + i];
            if (v < 0.0) continue;   // not a leaf of this level
            const int want = v > sig ? std::min(l + 1, L) : (v < csig ? std::max(l - 1, 0) : l);
            for (int c = 0; c < (1 << sh); ++c)
              for (int bb = 0; bb < (1 << sh); ++bb)
                for (int a = 0; a < (1 << sh); ++a) {
                  int& tv = t[bpos((i << sh) + a, (j << sh) + bb, (k << sh) + c)];
                  tv = std::max(tv, want);
                }
          }
    }
    return t;
  }

  // ---- particle coupling on the finest level --------------------------------
  void offset(const double p[3], const Sph& s, double d[3]) const {
    for (int a = 0; a < 3; ++a) d[a] = min_image(p[a] - s.x[a], lv[L].n[a], 1);
  }
  bool inside(int i, int j, int k, const Sph& s) const {
    double p[3] = {i + 0.5, j + 0.5, k + 0.5}, d[3];
    offset(p, s, d);
    double dd = d[0] * d[0];
    dd = dd + d[1] * d[1];
    dd = dd + d[2] * d[2];
    return dd <= s.r * s.r;
  }
  void map_all(std::vector<int>& o) const {
    const RLevel& V = lv[L];
    o.assign(V.N, -1);
    if (sph.empty()) return;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < V.n[2]; ++k)
      for (int j = 0; j < V.n[1]; ++j)
        for (int i = 0; i < V.n[0]; ++i)
          for (int p = 0; p < (int)sph.size(); ++p)
            if (inside(i, j, k, sph[p])) { o[idx(L, i, j, k)] = p; break; }
  }
  static void body_velocity(const Sph& s, const double d[3], double v[3]) {
    v[0] = s.u[0] + (s.w[1] * d[2] - s.w[2] * d[1]);
    v[1] = s.u[1] + (s.w[2] * d[0] - s.w[0] * d[2]);
    v[2] = s.u[2] + (s.w[0] * d[1] - s.w[1] * d[0]);
  }

  // ---- one level ---------------------------------------------------------------
  void explode(int l) {
    RLevel& F = lv[l + 1];
    const RLevel& C = lv[l];
#pragma omp parallel for schedule(static)
    for (int k = 0; k < F.n[2]; ++k)
      for (int j = 0; j < F.n[1]; ++j)
        for (int i = 0; i < F.n[0]; ++i) {
          const long g = idx(l + 1, i, j, k);
          if (F.kind[g] != GHOST) continue;
          const long p = idx(l, i >> 1, j >> 1, k >> 1);
          for (int q = 0; q < 19; ++q) F.cur[q * F.N + g] = C.cur[q * C.N + p];
        }
  }

  // pre-collision value of population q for interior level-l cell (i,j,k)
  // without particle links
  double pull(int l, int i, int j, int k, int q) const {
    const RLevel& V = lv[l];
    const int si = i - CX[q], sj = j - CY[q], sk = k - CZ[q];
    const long s = idx(l, si, sj, sk);
    const uint8_t ks = V.kind[s];
    if (ks == GHOST) return V.cur[q * V.N + s];
    double val = 0.0;
    if (ks == INTERIOR) {
      int nin = 0;
      if (l < L)
        for (int c = 0; c < 8; ++c) {
          const int gi = 2 * si + (c & 1), gj = 2 * sj + ((c >> 1) & 1), gk = 2 * sk + (c >> 2);
          if (kind_at(l + 1, gi + CX[q], gj + CY[q], gk + CZ[q]) == INTERIOR) ++nin;
        }
      val = (1.0 - nin / 8.0) * V.cur[q * V.N + s];
    }
    if (l < L) {
      const RLevel& F = lv[l + 1];
      double acc = 0.0;
      for (int c = 0; c < 8; ++c) {
        const int gi = 2 * i + (c & 1), gj = 2 * j + ((c >> 1) & 1), gk = 2 * k + (c >> 2);
        if (kind_at(l + 1, gi, gj, gk) != GHOST) continue;
        const uint8_t k1 = kind_at(l + 1, gi - CX[q], gj - CY[q], gk - CZ[q]);
        const uint8_t k2 = kind_at(l + 1, gi - 2 * CX[q], gj - 2 * CY[q], gk - 2 * CZ[q]);
        if (k1 == INTERIOR || (k1 == GHOST && k2 == INTERIOR)) acc += F.cur[q * F.N + idx(l + 1, gi, gj, gk)];
      }
      val += acc / 8.0;
    }
    return val;
  }

  // finest level: incoming population with Eq. 10 on particle links
  double incoming_L(int i, int j, int k, int q, double* delta_out, double vb[3], int* pid) const {
    const RLevel& V = lv[L];
    const long c = idx(L, i, j, k);
    *pid = -1;
    if (q == 0) return V.cur[c];
    const long src = idx(L, i - CX[q], j - CY[q], k - CZ[q]);
    if (own.empty() || own[src] < 0) return pull(L, i, j, k, q);
    const int qq = opposite(q);
    const double w = weight(qq);
    const Sph& s = sph[own[src]];
    *pid = own[src];
    double p[3] = {i + 0.5, j + 0.5, k + 0.5}, d[3];
    offset(p, s, d);
    int cq[3] = {CX[qq], CY[qq], CZ[qq]};
    double delta = link_delta(d, cq, s.r);
    double rb[3] = {d[0] + delta * cq[0], d[1] + delta * cq[1], d[2] + delta * cq[2]};
    double v[3];
    body_velocity(s, rb, v);
    double kappa = (1.0 - 2.0 * delta) / (1.0 + 2.0 * delta);
    double alpha = 4.0 / (1.0 + 2.0 * delta);
    const long second = idx(L, i + CX[q], j + CY[q], k + CZ[q]);
    if (own[second] >= 0 || V.kind[second] != INTERIOR) { kappa = 0.0; alpha = 2.0; }
    double cv = cq[0] * v[0] + cq[1] * v[1] + cq[2] * v[2];
    double val = V.cur[qq * V.N + c] - 3.0 * alpha * w * cv;
    if (kappa != 0.0) val = val + kappa * (V.cur[qq * V.N + second] - V.cur[q * V.N + c]);
    *delta_out = delta;
    for (int a = 0; a < 3; ++a) vb[a] = v[a];
    return val;
  }

  void sweep(int l) {
    RLevel& V = lv[l];
    const bool coupled = (l == L) && !sph.empty();
#pragma omp parallel for schedule(static)
    for (int k = 0; k < V.n[2]; ++k)
      for (int j = 0; j < V.n[1]; ++j)
        for (int i = 0; i < V.n[0]; ++i) {
          const long c = idx(l, i, j, k);
          if (V.kind[c] == GHOST) {
            // stream only
            for (int q = 0; q < 19; ++q) {
              const long s = idx(l, i - CX[q], j - CY[q], k - CZ[q]);
              V.nxt[q * V.N + c] = V.kind[s] != NONE ? V.cur[q * V.N + s] : 0.0;
            }
            continue;
          }
          if (V.kind[c] != INTERIOR) continue;
          if (coupled && own[c] >= 0) continue;
          for (int q = 0; q < 19; ++q) {
            double delta, vb[3];
            int pid;
            V.pre[q * V.N + c] = coupled ? incoming_L(i, j, k, q, &delta, vb, &pid) : pull(l, i, j, k, q);
          }
        }
    if (coupled) couple();
    else if (l == L) fine_steps += 1;
#pragma omp parallel for schedule(static)
    for (long c = 0; c < V.N; ++c) {
      if (V.kind[c] != INTERIOR) continue;
      if (coupled && own[c] >= 0) continue;
      double a[19], o[19];
      for (int q = 0; q < 19; ++q) a[q] = V.pre[q * V.N + c];
      double Fl[3] = {V.F[0], V.F[1], V.F[2]};
      V.coll(a, Fl, o);
      for (int q = 0; q < 19; ++q) V.nxt[q * V.N + c] = o[q];
    }
    std::swap(V.cur, V.nxt);
  }

  // link forces (Eqs. 11-12), particle update (Algorithm 1), re-mapping and
  // refill (Sec. 2.3) on the finest level, in pre-collision form
  void couple() {
    RLevel& V = lv[L];
    std::vector<long double> Fs(3 * sph.size(), 0.0L), Ts(3 * sph.size(), 0.0L);
    for (int k = 0; k < V.n[2]; ++k)
      for (int j = 0; j < V.n[1]; ++j)
        for (int i = 0; i < V.n[0]; ++i) {
          const long c = idx(L, i, j, k);
          if (V.kind[c] != INTERIOR || own[c] >= 0) continue;
          for (int q = 1; q < 19; ++q) {
            double delta, vb[3];
            int pid;
            const double fin = incoming_L(i, j, k, q, &delta, vb, &pid);
            if (pid < 0) continue;
            const int qq = opposite(q);
            const Sph& s = sph[pid];
            double p[3] = {i + 0.5, j + 0.5, k + 0.5}, d[3];
            offset(p, s, d);
            double rb[3] = {d[0] + delta * CX[qq], d[1] + delta * CY[qq], d[2] + delta * CZ[qq]};
            const int cqq[3] = {CX[qq], CY[qq], CZ[qq]}, cq[3] = {CX[q], CY[q], CZ[q]};
            double Fl[3];
            for (int a = 0; a < 3; ++a) Fl[a] = (cqq[a] - vb[a]) * V.cur[qq * V.N + c] - (cq[a] - vb[a]) * fin;
            double Tl[3] = {rb[1] * Fl[2] - rb[2] * Fl[1], rb[2] * Fl[0] - rb[0] * Fl[2], rb[0] * Fl[1] - rb[1] * Fl[0]};
            for (int a = 0; a < 3; ++a) { Fs[3 * pid + a] += Fl[a]; Ts[3 * pid + a] += Tl[a]; }
          }
        }
    bool moving = false;
    for (size_t p = 0; p < sph.size(); ++p) {
      Sph& s = sph[p];
      for (int a = 0; a < 3; ++a) { s.F[a] = (double)Fs[3 * p + a]; s.T[a] = (double)Ts[3 * p + a]; }
      if (s.fixed != 1) {
        update_particle(s, cfg.gravity, V.n, periodic_all);
        moving = moving || s.fixed == 0;
      }
      for (int a = 0; a < 3; ++a) { s.Fprev[a] = s.F[a]; s.Tprev[a] = s.T[a]; }
      s.have_prev = 1;
    }
    fine_steps += 1;
    if (!moving) return;
    std::vector<int> old_own = own, new_own;
    map_all(new_own);
    for (int k = 0; k < V.n[2]; ++k)
      for (int j = 0; j < V.n[1]; ++j)
        for (int i = 0; i < V.n[0]; ++i) {
          const long c = idx(L, i, j, k);
          if (old_own[c] >= 0 && new_own[c] < 0) refill(old_own, i, j, k, old_own[c]);
        }
    own = new_own;
  }

  void refill(const std::vector<int>& old_own, int i, int j, int k, int pid) {
    RLevel& V = lv[L];
    const long c = idx(L, i, j, k);
    auto rho_of = [&](long m) { double r = 0.0; for (int q = 0; q < 19; ++q) r += V.pre[q * V.N + m]; return r; };
    auto u_of = [&](long m, double u[3]) {
      double jj[3] = {0, 0, 0};
      for (int q = 0; q < 19; ++q) { jj[0] += CX[q] * V.pre[q * V.N + m]; jj[1] += CY[q] * V.pre[q * V.N + m]; jj[2] += CZ[q] * V.pre[q * V.N + m]; }
      for (int a = 0; a < 3; ++a) u[a] = jj[a] + 0.5 * V.F[a];
    };
    double rsum = 0.0;
    int cnt = 0;
    for (int q = 1; q < 19; ++q) {
      const long m = idx(L, i + CX[q], j + CY[q], k + CZ[q]);
      if (old_own[m] >= 0 || V.kind[m] != INTERIOR) continue;
      rsum += rho_of(m);
      ++cnt;
    }
    const double rho = cnt ? rsum / cnt : 1.0;
    const Sph& s = sph[pid];
    double p[3] = {i + 0.5, j + 0.5, k + 0.5}, d[3];
    offset(p, s, d);
    double v[3];
    body_velocity(s, d, v);
    double Vn[3][2][3];
    for (int a = 0; a < 3; ++a)
      for (int side = 0; side < 2; ++side) {
        int o[3] = {0, 0, 0};
        o[a] = side ? 1 : -1;
        const long m = idx(L, i + o[0], j + o[1], k + o[2]);
        double* Vv = Vn[a][side];
        if (old_own[m] < 0) {
          u_of(m, Vv);
        } else {
          const Sph& t = sph[old_own[m]];
          double pk[3] = {p[0] + o[0], p[1] + o[1], p[2] + o[2]}, dk[3];
          offset(pk, t, dk);
          body_velocity(t, dk, Vv);
        }
      }
    double S[3][3];
    for (int a = 0; a < 3; ++a)
      for (int bb = 0; bb < 3; ++bb)
        S[a][bb] = 0.5 * (0.5 * (Vn[a][1][bb] - Vn[a][0][bb]) + 0.5 * (Vn[bb][1][a] - Vn[bb][0][a]));
    double out[19];
    refill_populations(rho, v, S, V.sp, out);
    for (int q = 0; q < 19; ++q) V.pre[q * V.N + c] = out[q];
  }

  void step_level(int l) {
    if (l < L) {
      explode(l);
      step_level(l + 1);
      step_level(l + 1);
    }
    sweep(l);
  }

  // move data to a new block layout: coarser representations by averaging,
  // finer ones by copying (the cells' kinds still describe the old layout)
  void migrate(const std::vector<int>& newleaf) {
    for (int l = L - 1; l >= 0; --l) {
      RLevel& V = lv[l];
      const RLevel& F = lv[l + 1];
#pragma omp parallel for schedule(static)
      for (int k = 0; k < V.n[2]; ++k)
        for (int j = 0; j < V.n[1]; ++j)
          for (int i = 0; i < V.n[0]; ++i) {
            if (leaf_of(l, i, j, k) <= l) continue;
            const long c = idx(l, i, j, k);
            for (int q = 0; q < 19; ++q) {
              double acc = 0.0;
              for (int m = 0; m < 8; ++m)
                acc += F.cur[q * F.N + idx(l + 1, 2 * i + (m & 1), 2 * j + ((m >> 1) & 1), 2 * k + (m >> 2))];
              V.cur[q * V.N + c] = acc / 8.0;
            }
          }
    }
    for (int l = 1; l <= L; ++l) {
      RLevel& V = lv[l];
      const RLevel& C = lv[l - 1];
#pragma omp parallel for schedule(static)
      for (int k = 0; k < V.n[2]; ++k)
        for (int j = 0; j < V.n[1]; ++j)
          for (int i = 0; i < V.n[0]; ++i) {
            if (leaf_of(l, i, j, k) >= l) continue;
            const long c = idx(l, i, j, k);
            const long p = idx(l - 1, i >> 1, j >> 1, k >> 1);
            for (int q = 0; q < 19; ++q) V.cur[q * V.N + c] = C.cur[q * C.N + p];
          }
    }
    leaf = newleaf;
    compute_kinds();
  }

  void coarse_step() {
    step_level(0);
    coarse_steps += 1;
    if (cfg.check_every > 0 && coarse_steps % cfg.check_every == 0) {
      std::vector<int> nl = balance(targets(true));
      if (nl != leaf) {
        migrate(nl);
        refinements += 1;
      }
    }
  }

  int periodic_all[3] = {1, 1, 1};
};

}  // namespace

extern "C" {

void* orf_create(const orf_config* cfg) {
  if (!cfg || cfg->levels < 1 || cfg->levels > 8 || cfg->block < 2) return nullptr;
  auto* R = new RForest();
  R->cfg = *cfg;
  R->L = cfg->levels - 1;
  R->b = cfg->block;
  if ((1 << R->L) > R->b) { delete R; return nullptr; }
  for (int a = 0; a < 3; ++a) {
    if (cfg->n0[a] % cfg->block) { delete R; return nullptr; }
    R->nb[a] = (cfg->n0[a] / cfg->block) << R->L;
  }
  R->base.assign((long)R->nb[0] * R->nb[1] * R->nb[2], 0);
  R->lv.resize(R->L + 1);
  double tau = 1.0 / cfg->omega;
  for (int l = R->L; l >= 0; --l) {
    RLevel& V = R->lv[l];
    for (int a = 0; a < 3; ++a) V.n[a] = cfg->n0[a] << l;
    V.N = (long)V.n[0] * V.n[1] * V.n[2];
    V.sp = 1.0 / tau;
    V.sm = s_minus(V.sp, cfg->magic);
    V.mrt = cfg->bulk_factor > 0.0 && cfg->bulk_factor != 1.0;
    if (V.mrt) V.sb = s_bulk(V.sp, cfg->bulk_factor);
    for (int a = 0; a < 3; ++a) V.F[a] = cfg->body_force[a] * (double)(1 << (R->L - l));
    tau = 0.5 + 0.5 * (tau - 0.5);
  }
  return R;
}

int orf_add_region(void* h, const int lo[3], const int hi[3], int level) {
  auto* R = static_cast<RForest*>(h);
  if (!R || level < 0 || level > R->L) return -1;
  // coarse-cell box [lo, hi): finest blocks intersecting it get target >= level
  const int s = 1 << R->L;
  for (int k = 0; k < R->nb[2]; ++k)
    for (int j = 0; j < R->nb[1]; ++j)
      for (int i = 0; i < R->nb[0]; ++i) {
        const int p[3] = {i, j, k};
        bool in = true;
        for (int a = 0; a < 3; ++a) {
          const double b0 = (double)p[a] * R->b / s, b1 = (double)(p[a] + 1) * R->b / s;
          if (!(b1 > lo[a] && b0 < hi[a])) in = false;
        }
        if (in) R->base[R->bpos(i, j, k)] = std::max(R->base[R->bpos(i, j, k)], level);
      }
  return 0;
}

int orf_add_sphere(void* h, const orf_sphere* s) {
  auto* R = static_cast<RForest*>(h);
  if (!R || !s) return -1;
  Sph p{};
  if (s->fixed < 0 || s->fixed > 2) return -1;
  for (int a = 0; a < 3; ++a) { p.x[a] = s->x[a]; p.u[a] = s->fixed ? 0.0 : s->u[a]; p.w[a] = s->fixed == 1 ? 0.0 : s->w[a]; }
  p.r = s->radius; p.rho = s->density_ratio; p.cv = s->cv; p.cvw = s->cv_omega; p.fixed = s->fixed;
  p.scheme = s->vm_scheme;
  p.nvel = 1;
  if (p.scheme < 0 || p.scheme > 2) return -1;
  R->sph.push_back(p);
  return (int)R->sph.size() - 1;
}

int orf_init(void* h, double rho, const double* u0_coarse) {
  auto* R = static_cast<RForest*>(h);
  if (!R) return -1;
  R->leaf = R->balance(R->targets());
  for (auto& V : R->lv) {
    V.cur.assign(19 * V.N, 0.0);
    V.nxt.assign(19 * V.N, 0.0);
    V.pre.assign(19 * V.N, 0.0);
    V.kind.assign(V.N, NONE);
  }
  R->compute_kinds();
  R->map_all(R->own);
  const RLevel& C0 = R->lv[0];
  for (int l = 0; l <= R->L; ++l) {
    RLevel& V = R->lv[l];
    for (int k = 0; k < V.n[2]; ++k)
      for (int j = 0; j < V.n[1]; ++j)
        for (int i = 0; i < V.n[0]; ++i) {
          const long c = R->idx(l, i, j, k);
          if (l == R->L && !R->own.empty() && R->own[c] >= 0) continue;
          const long c0 = ((long)(k >> l) * C0.n[1] + (j >> l)) * C0.n[0] + (i >> l);
          double u[3];
          for (int a = 0; a < 3; ++a) u[a] = u0_coarse ? u0_coarse[a * C0.N + c0] : 0.0;
          double feq[19], o[19];
          equilibrium(rho, u, feq);
          V.coll(feq, V.F, o);
          for (int q = 0; q < 19; ++q) V.cur[q * V.N + c] = o[q];
        }
  }
  for (auto& s : R->sph) {
    for (int a = 0; a < 3; ++a) { s.a[a] = s.b[a] = 0.0; s.F[a] = s.T[a] = 0.0; }
    s.have_prev = 0;
  }
  R->coarse_steps = R->fine_steps = 0;
  R->refinements = 0;
  return 0;
}

// overwrite one level with f~ = collide(f^eq(rho, u)) from a velocity field
// given at that level's cells ([3][N_l])
int orf_set_level_velocity(void* h, int level, double rho, const double* u) {
  auto* R = static_cast<RForest*>(h);
  if (!R || level < 0 || level > R->L || !u) return -1;
  RLevel& V = R->lv[level];
  for (long c = 0; c < V.N; ++c) {
    double uc[3] = {u[c], u[V.N + c], u[2 * V.N + c]};
    double feq[19], o[19];
    equilibrium(rho, uc, feq);
    V.coll(feq, V.F, o);
    for (int q = 0; q < 19; ++q) V.cur[q * V.N + c] = o[q];
  }
  return 0;
}

int orf_step(void* h, int n) {
  auto* R = static_cast<RForest*>(h);
  if (!R || n < 0) return -1;
  for (int i = 0; i < n; ++i) R->coarse_step();
  return 0;
}

int orf_level_dims(void* h, int level, int n[3]) {
  auto* R = static_cast<RForest*>(h);
  if (!R || level < 0 || level > R->L) return -1;
  for (int a = 0; a < 3; ++a) n[a] = R->lv[level].n[a];
  return 0;
}

int orf_block_grid(void* h, int n[3]) {
  auto* R = static_cast<RForest*>(h);
  if (!R) return -1;
  for (int a = 0; a < 3; ++a) n[a] = R->nb[a];
  return 0;
}

int orf_leaf(void* h, int* out) {
  auto* R = static_cast<RForest*>(h);
  if (!R) return -1;
  for (size_t i = 0; i < R->leaf.size(); ++i) out[i] = R->leaf[i];
  return 0;
}

// post-collision populations of a level ([19][N_l]; cells that are not
// interior fluid read 0) and the cell kinds (0 none, 1 interior, 2 ghost)
int orf_read_level(void* h, int level, double* out, unsigned char* kind) {
  auto* R = static_cast<RForest*>(h);
  if (!R || level < 0 || level > R->L) return -1;
  const RLevel& V = R->lv[level];
  for (long c = 0; c < V.N; ++c) {
    const bool fluid = V.kind[c] == INTERIOR && !(level == R->L && !R->own.empty() && R->own[c] >= 0);
    if (kind) kind[c] = V.kind[c];
    if (out)
      for (int q = 0; q < 19; ++q) out[q * V.N + c] = fluid ? V.cur[q * V.N + c] : 0.0;
  }
  return 0;
}

// total mass sum_l 8^-l sum over interior fluid cells of sum_q f~
int orf_mass(void* h, double* mass) {
  auto* R = static_cast<RForest*>(h);
  if (!R || !mass) return -1;
  long double m = 0.0L;
  for (int l = 0; l <= R->L; ++l) {
    const RLevel& V = R->lv[l];
    long double ml = 0.0L;
    for (long c = 0; c < V.N; ++c) {
      if (V.kind[c] != INTERIOR) continue;
      if (l == R->L && !R->own.empty() && R->own[c] >= 0) continue;
      for (int q = 0; q < 19; ++q) ml += V.cur[q * V.N + c];
    }
    m += ml / (long double)(1L << (3 * l));
  }
  *mass = (double)m;
  return 0;
}

int orf_force_torque(void* h, int id, double F[3], double T[3]) {
  auto* R = static_cast<RForest*>(h);
  if (!R || id < 0 || id >= (int)R->sph.size()) return -1;
  for (int a = 0; a < 3; ++a) { F[a] = R->sph[id].F[a]; T[a] = R->sph[id].T[a]; }
  return 0;
}

int orf_particle(void* h, int id, double x[3], double u[3], double w[3]) {
  auto* R = static_cast<RForest*>(h);
  if (!R || id < 0 || id >= (int)R->sph.size()) return -1;
  for (int a = 0; a < 3; ++a) { x[a] = R->sph[id].x[a]; u[a] = R->sph[id].u[a]; w[a] = R->sph[id].w[a]; }
  return 0;
}

int orf_owner(void* h, int* out) {
  auto* R = static_cast<RForest*>(h);
  if (!R) return -1;
  const RLevel& V = R->lv[R->L];
  for (long c = 0; c < V.N; ++c) out[c] = R->own.empty() ? -1 : R->own[c];
  return 0;
}

int orf_counters(void* h, long long* coarse, long long* fine, int* refinements) {
  auto* R = static_cast<RForest*>(h);
  if (!R) return -1;
  if (coarse) *coarse = R->coarse_steps;
  if (fine) *fine = R->fine_steps;
  if (refinements) *refinements = R->refinements;
  return 0;
}

// as ora_set_sphere_motion
int orf_set_sphere_motion(void* h, int id, const double u[3], const double w[3], int fixed) {
  auto* R = static_cast<RForest*>(h);
  if (!R || id < 0 || id >= (int)R->sph.size() || fixed < 0 || fixed > 2) return -1;
  Sph& s = R->sph[id];
  s.fixed = fixed;
  for (int a = 0; a < 3; ++a) {
    s.u[a] = fixed ? 0.0 : u[a];
    s.w[a] = fixed == 1 ? 0.0 : w[a];
  }
  return 0;
}

void orf_destroy(void* h) { delete static_cast<RForest*>(h); }

/* curl sensor of Eq. 23 per level-l block (level block grid order, x
 * fastest): max over the block's evaluated cells, 0 if none, -1 for blocks
 * that are not leaves of this level */
int orf_block_sensor(void* h, int level, double* out) {
  auto* R = static_cast<RForest*>(h);
  if (!R || !out || level < 0 || level > R->L) return -1;
  const std::vector<double> s = R->block_sensor(level);
  for (size_t i = 0; i < s.size(); ++i) out[i] = s[i];
  return 0;
}

}  // extern "C"
