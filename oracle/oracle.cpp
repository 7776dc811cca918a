// CPU oracle for the coupled LBM hot path -- TEST INFRASTRUCTURE ONLY.
//
// Plain FP64 (and dual-number) implementation written from the paper.  Every
// step is computed in the order the method states it, over whole arrays, with
// no blocking or fusion:
//   collide (Sec. 2.1, TRT with magic parameter) -> stream with boundary links
//   (Sec. 2.1 LBM update, Eq. 10 CLI boundary) -> link forces and their sums
//   (Eqs. 11-12) -> particle update (Sec. 2.2 velocity Verlet with the virtual
//   mass terms of Sec. 3.3, Algorithm 1) -> re-mapping and refill (Sec. 2.3).
// Readings of points the paper leaves open are marked "reading:".
//
// Pins (tests/test_oracle_pins.py, tests/test_oracle_refine.py): every
// function is checked against closed forms, invariants or brute force.  The
// refill (the paper only cites its scheme) is pinned in two parts: its
// populations for a given strain rate by their moments (density, momentum,
// and the Chapman-Enskog first-order stress), and its estimate of the strain
// rate by linear velocity fields, on which central differences are exact.
//
// Only tests/, the smoke check and the benchmark's CPU-baseline leg load this
// library.  It shares no code with the GPU library.
#include "oracle.h"

#include <cmath>
#include <cstdint>
#include <cstring>
#include <type_traits>
#include <vector>
#include <omp.h>

#include "core.hpp"

namespace {
using namespace ora;

// ---------------------------------------------------------------------------
// uniform grid
// ---------------------------------------------------------------------------
template <class T>
struct Grid {
  ora_config cfg;
  int nx, ny, nz;
  long N;
  std::vector<T> f, ft, fn;     // [19][N]
  std::vector<int> own;         // -1 fluid, else sphere id
  std::vector<unsigned char> has_link;
  std::vector<Sph> sph;
  T sp, sm, F[3];
  double sb = 0.0;              // MRT bulk rate (used when mrt)
  bool mrt = false;
  int steps = 0;
  int wall_axis = -1;

  long idx(int x, int y, int z) const { return ((long)z * ny + y) * nx + x; }
  double centre(int i) const { return i + 0.5; }

  explicit Grid(const ora_config& c) : cfg(c) {
    nx = c.n[0]; ny = c.n[1]; nz = c.n[2];
    N = (long)nx * ny * nz;
    for (int a = 0; a < 3; ++a)
      if (!c.periodic[a]) { wall_axis = a; break; }
    sp = T(c.omega);
    sm = s_minus(sp, c.magic);
    for (int a = 0; a < 3; ++a) F[a] = T(c.body_force[a]);
    mrt = c.bulk_factor > 0.0 && c.bulk_factor != 1.0;
    if (mrt) sb = s_bulk(c.omega, c.bulk_factor);
  }

  // offset from a sphere centre to a point, minimum image on periodic axes
  void offset(const double p[3], const Sph& s, double d[3]) const {
    const int n[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) d[a] = min_image(p[a] - s.x[a], n[a], cfg.periodic[a]);
  }
  bool inside(int x, int y, int z, const Sph& s) const {
    double p[3] = {centre(x), centre(y), centre(z)}, d[3];
    offset(p, s, d);
    double dd = d[0] * d[0];
    dd = dd + d[1] * d[1];
    dd = dd + d[2] * d[2];
    return dd <= s.r * s.r;
  }
  void map_all(std::vector<int>& o) const {
    o.assign(N, -1);
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x)
          for (int p = 0; p < (int)sph.size(); ++p)
            if (inside(x, y, z, sph[p])) { o[idx(x, y, z)] = p; break; }
  }

  // neighbour of (x,y,z) at offset (dx,dy,dz): returns false if it leaves the
  // domain through a wall; *axis / *side name the wall.
  bool neighbour(int x, int y, int z, int dx, int dy, int dz, long* out, int* axis, int* side) const {
    int p[3] = {x + dx, y + dy, z + dz};
    const int n[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
      if (p[a] < 0 || p[a] >= n[a]) {
        if (cfg.periodic[a]) { p[a] = (p[a] + n[a]) % n[a]; }
        else { *axis = a; *side = p[a] < 0 ? 0 : 1; return false; }
      }
    }
    *out = idx(p[0], p[1], p[2]);
    return true;
  }

  void wall_velocity(int axis, int side, double v[3]) const {
    for (int a = 0; a < 3; ++a) v[a] = (axis == wall_axis) ? cfg.wall_velocity[side][a] : 0.0;
  }

  void init(double rho, const double* u0, const double* rho_field = nullptr) {
    map_all(own);
    f.assign(19 * N, T(0.0));
    ft.assign(19 * N, T(0.0));
    fn.assign(19 * N, T(0.0));
    has_link.assign(N, 0);
    for (long c = 0; c < N; ++c) {
      if (own[c] >= 0) continue;
      T u[3];
      for (int a = 0; a < 3; ++a) u[a] = T(u0 ? u0[a * N + c] : 0.0);
      T feq[19];
      equilibrium(T(rho_field ? rho_field[c] : rho), u, feq);
      for (int q = 0; q < 19; ++q) f[q * N + c] = feq[q];
    }
    for (auto& s : sph) {
      for (int a = 0; a < 3; ++a) { s.a[a] = s.b[a] = 0.0; s.F[a] = s.T[a] = 0.0; }
      s.have_prev = 0;
    }
    steps = 0;
  }

  void collide_all(const std::vector<T>& src, std::vector<T>& dst) const {
#pragma omp parallel for schedule(static)
    for (long c = 0; c < N; ++c) {
      if (own[c] >= 0) continue;
      T a[19], b[19];
      for (int q = 0; q < 19; ++q) a[q] = src[q * N + c];
      if constexpr (std::is_same<T, double>::value) {
        if (mrt) collide_mrt(a, sp, sm, sb, F, b);
        else collide(a, sp, sm, F, b);
      } else {
        collide(a, sp, sm, F, b);
      }
      for (int q = 0; q < 19; ++q) dst[q * N + c] = b[q];
    }
  }

  // rigid-body velocity of sphere s at offset d from its centre
  static void body_velocity(const Sph& s, const double d[3], double v[3]) {
    v[0] = s.u[0] + (s.w[1] * d[2] - s.w[2] * d[1]);
    v[1] = s.u[1] + (s.w[2] * d[0] - s.w[0] * d[2]);
    v[2] = s.u[2] + (s.w[0] * d[1] - s.w[1] * d[0]);
  }

  // Incoming population q of fluid cell (x,y,z) at t+1.  If the source cell
  // x - c_q is fluid this is plain streaming; otherwise the link from x in
  // direction qq = opp(q) ends in a wall or a particle and Eq. 10 (CLI)
  // gives the value.  Returns the particle id for particle links (else -1)
  // and, for those, delta and the link velocity.
  T incoming(int x, int y, int z, int q, double* delta_out, double vb_out[3], int* pid) const {
    long c = idx(x, y, z);
    *pid = -1;
    if (q == 0) return ft[c];
    int qq = opposite(q);
    long src; int axis, side;
    const double w = weight(qq);
    if (!neighbour(x, y, z, -CX[q], -CY[q], -CZ[q], &src, &axis, &side)) {
      // domain wall, halfway: delta = 1/2 -> kappa0 = 0, alpha = 2
      double v[3];
      wall_velocity(axis, side, v);
      double cv = CX[qq] * v[0] + CY[qq] * v[1] + CZ[qq] * v[2];
      return ft[qq * N + c] - 3.0 * 2.0 * w * cv;
    }
    if (own[src] < 0) return ft[q * N + src];
    // particle link: x + c_qq = src is solid
    const Sph& s = sph[own[src]];
    *pid = own[src];
    double p[3] = {centre(x), centre(y), centre(z)}, d[3];
    offset(p, s, d);
    int cq[3] = {CX[qq], CY[qq], CZ[qq]};
    double delta = link_delta(d, cq, s.r);
    double rb[3] = {d[0] + delta * cq[0], d[1] + delta * cq[1], d[2] + delta * cq[2]};
    double v[3];
    body_velocity(s, rb, v);
    double kappa = (1.0 - 2.0 * delta) / (1.0 + 2.0 * delta);
    double alpha = 4.0 / (1.0 + 2.0 * delta);
    // second fluid node x - c_qq = x + c_q; reading: if it is not fluid,
    // fall back to kappa0 = 0, alpha = 2
    long second = c; int ax2 = 0, sd2 = 0;
    bool ok = neighbour(x, y, z, CX[q], CY[q], CZ[q], &second, &ax2, &sd2);
    if (!ok || own[second] >= 0) { kappa = 0.0; alpha = 2.0; }
    double cv = cq[0] * v[0] + cq[1] * v[1] + cq[2] * v[2];
    T val = ft[qq * N + c] - 3.0 * alpha * w * cv;
    if (kappa != 0.0) val = val + kappa * (ft[qq * N + second] - ft[q * N + c]);
    *delta_out = delta;
    for (int a = 0; a < 3; ++a) vb_out[a] = v[a];
    return val;
  }

  void stream_all() {
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          long c = idx(x, y, z);
          has_link[c] = 0;
          if (own[c] >= 0) continue;
          for (int q = 0; q < 19; ++q) {
            double delta, vb[3];
            int pid;
            fn[q * N + c] = incoming(x, y, z, q, &delta, vb, &pid);
            if (pid >= 0) has_link[c] = 1;
          }
        }
  }

  // Eqs. 11-12: link forces and their sums, sequential in (z, y, x, q) order
  void sum_forces() {
    using A = typename Acc<T>::type;
    std::vector<A> Fs(3 * sph.size(), A(0.0)), Ts(3 * sph.size(), A(0.0));
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          long c = idx(x, y, z);
          if (!has_link[c]) continue;
          for (int q = 1; q < 19; ++q) {
            double delta, vb[3];
            int pid;
            T fin = incoming(x, y, z, q, &delta, vb, &pid);
            if (pid < 0) continue;
            int qq = opposite(q);
            const Sph& s = sph[pid];
            double p[3] = {centre(x), centre(y), centre(z)}, d[3];
            offset(p, s, d);
            double rb[3] = {d[0] + delta * CX[qq], d[1] + delta * CY[qq], d[2] + delta * CZ[qq]};
            const int cqq[3] = {CX[qq], CY[qq], CZ[qq]};
            const int cq[3] = {CX[q], CY[q], CZ[q]};
            T Fl[3];
            for (int a = 0; a < 3; ++a)
              Fl[a] = (cqq[a] - vb[a]) * ft[qq * N + c] - (cq[a] - vb[a]) * fin;
            T Tl[3] = {rb[1] * Fl[2] - rb[2] * Fl[1], rb[2] * Fl[0] - rb[0] * Fl[2],
                       rb[0] * Fl[1] - rb[1] * Fl[0]};
            for (int a = 0; a < 3; ++a) {
              Fs[3 * pid + a] = Fs[3 * pid + a] + A(Fl[a]);
              Ts[3 * pid + a] = Ts[3 * pid + a] + A(Tl[a]);
            }
          }
        }
    last_F.assign(3 * sph.size(), T(0.0));
    last_T.assign(3 * sph.size(), T(0.0));
    for (size_t i = 0; i < Fs.size(); ++i) { last_F[i] = T(to_double(Fs[i])); last_T[i] = T(to_double(Ts[i])); }
  }
  std::vector<T> last_F, last_T;
};

// ---------------------------------------------------------------------------
// refill of a newly uncovered cell (Sec. 2.3, after Dorschner et al.):
// reading: rho is the mean density of the D3Q19 neighbours that held fluid
// before the re-mapping; the velocity is the rigid-body velocity of the
// particle that uncovered the cell; the strain rate comes from central
// differences over the six axis neighbours (fluid velocity where the
// neighbour held fluid, rigid-body or wall velocity otherwise); the
// populations are f^eq(rho, v) - 3 w_q / s+ (c_q c_q - I/3) : S.
// ---------------------------------------------------------------------------
void refill_cell(Grid<double>& G, const std::vector<int>& old_own, int x, int y, int z, int pid) {
  const long N = G.N;
  long c = G.idx(x, y, z);
  auto cell_rho = [&](long k) { double r = 0.0; for (int q = 0; q < 19; ++q) r += G.fn[q * N + k]; return r; };
  auto cell_u = [&](long k, double u[3]) {
    double j[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < 19; ++q) { j[0] += CX[q] * G.fn[q * N + k]; j[1] += CY[q] * G.fn[q * N + k]; j[2] += CZ[q] * G.fn[q * N + k]; }
    for (int a = 0; a < 3; ++a) u[a] = j[a] + 0.5 * G.cfg.body_force[a];
  };
  double rsum = 0.0;
  int cnt = 0;
  for (int q = 1; q < 19; ++q) {
    long k; int ax, sd;
    if (!G.neighbour(x, y, z, CX[q], CY[q], CZ[q], &k, &ax, &sd)) continue;
    if (old_own[k] >= 0) continue;
    rsum += cell_rho(k);
    ++cnt;
  }
  double rho = cnt ? rsum / cnt : 1.0;
  const Sph& s = G.sph[pid];
  double p[3] = {G.centre(x), G.centre(y), G.centre(z)}, d[3];
  G.offset(p, s, d);
  double v[3];
  Grid<double>::body_velocity(s, d, v);
  // velocity at the six axis neighbours
  double Vn[3][2][3];
  for (int a = 0; a < 3; ++a)
    for (int side = 0; side < 2; ++side) {
      int o[3] = {0, 0, 0};
      o[a] = side ? 1 : -1;
      long k; int ax, sd;
      double* V = Vn[a][side];
      if (!G.neighbour(x, y, z, o[0], o[1], o[2], &k, &ax, &sd)) {
        G.wall_velocity(ax, sd, V);
      } else if (old_own[k] < 0) {
        cell_u(k, V);
      } else {
        const Sph& t = G.sph[old_own[k]];
        double pk[3] = {p[0] + o[0], p[1] + o[1], p[2] + o[2]}, dk[3];
        G.offset(pk, t, dk);
        Grid<double>::body_velocity(t, dk, V);
      }
    }
  double grad[3][3];  // grad[a][b] = d u_b / d x_a
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) grad[a][b] = 0.5 * (Vn[a][1][b] - Vn[a][0][b]);
  double S[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) S[a][b] = 0.5 * (grad[a][b] + grad[b][a]);
  double out[19];
  refill_populations(rho, v, S, G.cfg.omega, out);
  for (int q = 0; q < 19; ++q) G.fn[q * N + c] = out[q];
}

// one full step of Algorithm 1 on the plain-FP64 grid
void step_double(Grid<double>& G) {
  G.collide_all(G.f, G.ft);
  G.stream_all();
  G.sum_forces();
  bool moving = false;
  for (size_t p = 0; p < G.sph.size(); ++p) {
    Sph& s = G.sph[p];
    for (int a = 0; a < 3; ++a) { s.F[a] = G.last_F[3 * p + a]; s.T[a] = G.last_T[3 * p + a]; }
    if (s.fixed != 1) {
      update_particle(s, G.cfg.gravity, G.cfg.n, G.cfg.periodic);
      moving = moving || s.fixed == 0;
    }
    for (int a = 0; a < 3; ++a) { s.Fprev[a] = s.F[a]; s.Tprev[a] = s.T[a]; }
    s.have_prev = 1;
  }
  if (moving) {
    std::vector<int> old_own = G.own, new_own;
    G.map_all(new_own);
    for (int z = 0; z < G.nz; ++z)
      for (int y = 0; y < G.ny; ++y)
        for (int x = 0; x < G.nx; ++x) {
          long c = G.idx(x, y, z);
          if (old_own[c] >= 0 && new_own[c] < 0) refill_cell(G, old_own, x, y, z, old_own[c]);
        }
    G.own = new_own;
    // reading: newly covered cells drop their populations
    for (long c = 0; c < G.N; ++c)
      if (G.own[c] >= 0)
        for (int q = 0; q < 19; ++q) G.fn[q * G.N + c] = 0.0;
  }
  std::swap(G.f, G.fn);
  G.steps += 1;
}

// forward map in any scalar type (fixed spheres only)
template <class T>
void step_fixed(Grid<T>& G) {
  G.collide_all(G.f, G.ft);
  G.stream_all();
  G.sum_forces();
  std::swap(G.f, G.fn);
  G.steps += 1;
}

template <class T>
T drag_average(const ora_config* cfg, const ora_sphere* spheres, int ns, int n_steps, int avg_from,
               const T& fmag, const T& omega) {
  ora_config c = *cfg;
  Grid<T> G(c);
  G.sp = omega;
  G.sm = s_minus(omega, c.magic);
  G.F[0] = T(0.0); G.F[1] = T(0.0); G.F[2] = fmag;
  for (int i = 0; i < ns; ++i) {
    Sph s{};
    for (int a = 0; a < 3; ++a) { s.x[a] = spheres[i].x[a]; s.u[a] = 0.0; s.w[a] = 0.0; }
    s.r = spheres[i].radius; s.rho = spheres[i].density_ratio; s.cv = spheres[i].cv; s.cvw = spheres[i].cv_omega;
    s.fixed = 1;
    G.sph.push_back(s);
  }
  G.init(1.0, nullptr);
  T acc(0.0);
  for (int n = 0; n < n_steps; ++n) {
    step_fixed(G);
    if (n >= avg_from) acc = acc + G.last_F[2];
  }
  return acc / double(n_steps - avg_from);
}

}  // namespace

// ---------------------------------------------------------------------------
// C API
// ---------------------------------------------------------------------------
extern "C" {

void ora_lattice(int c[19][3], double w[19], int opp[19]) {
  for (int q = 0; q < 19; ++q) {
    c[q][0] = CX[q]; c[q][1] = CY[q]; c[q][2] = CZ[q];
    w[q] = weight(q);
    opp[q] = opposite(q);
  }
}

void ora_collide_cell(const double f[19], double omega, double magic, const double F[3], double out[19]) {
  double sp = omega, sm = s_minus(sp, magic);
  collide(f, sp, sm, F, out);
}

void ora_equilibrium(double rho, const double u[3], double out[19]) { equilibrium(rho, u, out); }

void ora_collide_cell_mrt(const double f[19], double omega, double magic, double bulk_factor, const double F[3],
                          double out[19]) {
  collide_mrt(f, omega, s_minus(omega, magic), s_bulk(omega, bulk_factor), F, out);
}

void ora_mrt_basis(double e[19][19], double norm[19]) {
  const MrtBasis& B = mrt_basis();
  for (int a = 0; a < 19; ++a) {
    norm[a] = B.norm[a];
    for (int q = 0; q < 19; ++q) e[a][q] = B.e[a][q];
  }
}

void ora_refill_populations(double rho, const double v[3], const double S[9], double omega, double out[19]) {
  double M[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) M[a][b] = S[3 * a + b];
  refill_populations(rho, v, M, omega, out);
}

double ora_link_delta(const double d[3], const int c[3], double radius) { return link_delta(d, c, radius); }

void* ora_create(const ora_config* cfg) {
  if (!cfg) return nullptr;
  for (int a = 0; a < 3; ++a) if (cfg->n[a] <= 0) return nullptr;
  return new Grid<double>(*cfg);
}

int ora_add_sphere(void* h, const ora_sphere* s) {
  auto* G = static_cast<Grid<double>*>(h);
  if (!G || !s || s->radius <= 0.0) return -1;
  Sph p{};
  for (int a = 0; a < 3; ++a) { p.x[a] = s->x[a]; p.u[a] = s->u[a]; p.w[a] = s->w[a]; }
  p.r = s->radius; p.rho = s->density_ratio; p.cv = s->cv; p.cvw = s->cv_omega; p.fixed = s->fixed;
  p.scheme = s->vm_scheme;
  p.nvel = 1;
  if (p.fixed < 0 || p.fixed > 2 || p.scheme < 0 || p.scheme > 2) return -1;
  for (int a = 0; a < 3; ++a) {
    if (p.fixed) p.u[a] = 0.0;
    if (p.fixed == 1) p.w[a] = 0.0;
  }
  G->sph.push_back(p);
  return (int)G->sph.size() - 1;
}

// new velocities and hold mode of sphere id (position unchanged); the
// accelerations and the previous step's F/T are kept
int ora_set_sphere_motion(void* h, int id, const double u[3], const double w[3], int fixed) {
  auto* G = static_cast<Grid<double>*>(h);
  if (!G || id < 0 || id >= (int)G->sph.size() || fixed < 0 || fixed > 2) return -1;
  Sph& s = G->sph[id];
  s.fixed = fixed;
  for (int a = 0; a < 3; ++a) {
    s.u[a] = fixed ? 0.0 : u[a];
    s.w[a] = fixed == 1 ? 0.0 : w[a];
  }
  return 0;
}

// the refill of one cell on a given pre-collision state and old mapping
// (test entry point for the gradient estimate)
int ora_refill_cell(void* h, const double* f_pre, const int* old_owner, int x, int y, int z, int pid,
                    double out[19]) {
  auto* G = static_cast<Grid<double>*>(h);
  if (!G || !f_pre || !old_owner || !out || pid < 0 || pid >= (int)G->sph.size()) return -1;
  if (x < 0 || y < 0 || z < 0 || x >= G->nx || y >= G->ny || z >= G->nz) return -1;
  G->fn.assign(f_pre, f_pre + 19 * G->N);
  std::vector<int> old_own(old_owner, old_owner + G->N);
  refill_cell(*G, old_own, x, y, z, pid);
  const long c = G->idx(x, y, z);
  for (int q = 0; q < 19; ++q) out[q] = G->fn[q * G->N + c];
  return 0;
}

int ora_init(void* h, double rho, const double* u0) {
  auto* G = static_cast<Grid<double>*>(h);
  if (!G) return -1;
  G->init(rho, u0);
  return 0;
}

int ora_init_fields(void* h, const double* rho, const double* u0) {
  auto* G = static_cast<Grid<double>*>(h);
  if (!G || !rho) return -1;
  G->init(1.0, u0, rho);
  return 0;
}

int ora_step(void* h, int nsteps) {
  auto* G = static_cast<Grid<double>*>(h);
  if (!G || nsteps < 0) return -1;
  for (int i = 0; i < nsteps; ++i) step_double(*G);
  return 0;
}

int ora_post_collision(void* h, double* out) {
  auto* G = static_cast<Grid<double>*>(h);
  if (!G || !out) return -1;
  std::vector<double> ft(19 * G->N, 0.0);
  G->collide_all(G->f, ft);
  for (long c = 0; c < G->N; ++c)
    for (int q = 0; q < 19; ++q) out[q * G->N + c] = G->own[c] >= 0 ? 0.0 : ft[q * G->N + c];
  return 0;
}

int ora_pre_collision(void* h, double* out) {
  auto* G = static_cast<Grid<double>*>(h);
  if (!G || !out) return -1;
  for (long c = 0; c < G->N; ++c)
    for (int q = 0; q < 19; ++q) out[q * G->N + c] = G->own[c] >= 0 ? 0.0 : G->f[q * G->N + c];
  return 0;
}

int ora_owner(void* h, int* out) {
  auto* G = static_cast<Grid<double>*>(h);
  if (!G || !out) return -1;
  for (long c = 0; c < G->N; ++c) out[c] = G->own[c];
  return 0;
}

int ora_force_torque(void* h, int id, double F[3], double T[3]) {
  auto* G = static_cast<Grid<double>*>(h);
  if (!G || id < 0 || id >= (int)G->sph.size()) return -1;
  for (int a = 0; a < 3; ++a) { F[a] = G->sph[id].F[a]; T[a] = G->sph[id].T[a]; }
  return 0;
}

int ora_particle(void* h, int id, double x[3], double u[3], double w[3]) {
  auto* G = static_cast<Grid<double>*>(h);
  if (!G || id < 0 || id >= (int)G->sph.size()) return -1;
  for (int a = 0; a < 3; ++a) { x[a] = G->sph[id].x[a]; u[a] = G->sph[id].u[a]; w[a] = G->sph[id].w[a]; }
  return 0;
}

int ora_fields(void* h, double* rho, double* u) {
  auto* G = static_cast<Grid<double>*>(h);
  if (!G) return -1;
  const long N = G->N;
  for (long c = 0; c < N; ++c) {
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    if (G->own[c] < 0)
      for (int q = 0; q < 19; ++q) {
        double v = G->f[q * N + c];
        r += v; j[0] += CX[q] * v; j[1] += CY[q] * v; j[2] += CZ[q] * v;
      }
    if (rho) rho[c] = r;
    if (u)
      for (int a = 0; a < 3; ++a) u[a * N + c] = G->own[c] < 0 ? j[a] + 0.5 * G->cfg.body_force[a] : 0.0;
  }
  return 0;
}

int ora_totals(void* h, double* mass, double mom[3]) {
  auto* G = static_cast<Grid<double>*>(h);
  if (!G) return -1;
  long double m = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (long c = 0; c < G->N; ++c) {
    if (G->own[c] >= 0) continue;
    for (int q = 0; q < 19; ++q) {
      long double v = G->f[q * G->N + c];
      m += v; j[0] += CX[q] * v; j[1] += CY[q] * v; j[2] += CZ[q] * v;
    }
  }
  *mass = (double)m;
  for (int a = 0; a < 3; ++a) mom[a] = (double)j[a];
  return 0;
}

int ora_steps_done(void* h) {
  auto* G = static_cast<Grid<double>*>(h);
  return G ? G->steps : -1;
}

void ora_destroy(void* h) { delete static_cast<Grid<double>*>(h); }

int ora_drag_gradient(const ora_config* cfg, const ora_sphere* spheres, int nspheres, int n_steps,
                      int avg_from, double* J, double grad[2]) {
  if (!cfg || n_steps <= avg_from || avg_from < 0) return -1;
  if (cfg->bulk_factor > 0.0 && cfg->bulk_factor != 1.0) return -1;   // TRT only
  D2 fmag(cfg->body_force[2]);
  fmag.d[0] = 1.0;
  D2 om(cfg->omega);
  om.d[1] = 1.0;
  D2 r = drag_average<D2>(cfg, spheres, nspheres, n_steps, avg_from, fmag, om);
  *J = r.v;
  grad[0] = r.d[0];
  grad[1] = r.d[1];
  return 0;
}

int ora_drag_value(const ora_config* cfg, const ora_sphere* spheres, int nspheres, int n_steps,
                   int avg_from, double* J) {
  if (!cfg || n_steps <= avg_from || avg_from < 0) return -1;
  *J = drag_average<double>(cfg, spheres, nspheres, n_steps, avg_from, cfg->body_force[2], cfg->omega);
  return 0;
}

int ora_vm_trajectory(const ora_sphere* s0, const double F[3], const double dF[3], const double T[3],
                      const double g[3], int nsteps, double* out) {
  if (!s0 || nsteps < 0 || !out) return -1;
  Sph s{};
  for (int a = 0; a < 3; ++a) { s.x[a] = s0->x[a]; s.u[a] = s0->u[a]; s.w[a] = s0->w[a]; s.a[a] = s.b[a] = 0.0; }
  s.r = s0->radius; s.rho = s0->density_ratio; s.cv = s0->cv; s.cvw = s0->cv_omega;
  s.fixed = s0->fixed == 2 ? 2 : 0;
  s.scheme = s0->vm_scheme;
  s.nvel = 1;
  s.have_prev = 0;
  const int n[3] = {1, 1, 1}, periodic[3] = {0, 0, 0};
  for (int k = 0; k < nsteps; ++k) {
    for (int a = 0; a < 3; ++a) { s.F[a] = F[a] + k * dF[a]; s.T[a] = T[a]; }
    update_particle(s, g, n, periodic);
    for (int a = 0; a < 3; ++a) { s.Fprev[a] = s.F[a]; s.Tprev[a] = s.T[a]; }
    s.have_prev = 1;
    double* o = out + 15 * k;
    for (int a = 0; a < 3; ++a) { o[a] = s.x[a]; o[3 + a] = s.u[a]; o[6 + a] = s.w[a]; o[9 + a] = s.a[a]; o[12 + a] = s.b[a]; }
  }
  return 0;
}

int ora_num_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
