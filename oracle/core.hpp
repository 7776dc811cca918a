// Core arithmetic of the CPU oracle (test infrastructure only): lattice,
// collision, equilibrium, sphere geometry, particle update and refill
// populations.  Shared by the uniform-grid and the refined-grid oracle.
#pragma once

#include <cmath>
#include <vector>

namespace ora {

// ---------------------------------------------------------------------------
// D3Q19 lattice (Sec. 2.1).  The paper does not print the set; this is the
// textbook D3Q19 in the order: rest, 6 axis, then the xy, xz, yz diagonals.
// ---------------------------------------------------------------------------
const int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 0, 0, 0, 0};
const int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1};
const int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1};

inline double weight(int q) {
  int c2 = CX[q] * CX[q] + CY[q] * CY[q] + CZ[q] * CZ[q];
  if (c2 == 0) return 1.0 / 3.0;
  if (c2 == 1) return 1.0 / 18.0;
  return 1.0 / 36.0;
}

inline int opposite(int q) {
  for (int r = 0; r < 19; ++r)
    if (CX[r] == -CX[q] && CY[r] == -CY[q] && CZ[r] == -CZ[q]) return r;
  return -1;
}

// ---------------------------------------------------------------------------
// dual numbers: value plus N tangents, for the exact forward derivative
// ---------------------------------------------------------------------------
template <int N>
struct Dual {
  double v;
  double d[N];
  Dual() : v(0.0) { for (int i = 0; i < N; ++i) d[i] = 0.0; }
  Dual(double x) : v(x) { for (int i = 0; i < N; ++i) d[i] = 0.0; }
};
template <int N> Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v + b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
template <int N> Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v - b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
template <int N> Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r; r.v = -a.v; for (int i = 0; i < N; ++i) r.d[i] = -a.d[i]; return r; }
template <int N> Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v * b.v; for (int i = 0; i < N; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
template <int N> Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r; r.v = a.v / b.v;
  for (int i = 0; i < N; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r; }
template <int N> Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N> Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N> Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> Dual<N> operator*(const Dual<N>& a, double b) { return a * Dual<N>(b); }
template <int N> Dual<N> operator*(double a, const Dual<N>& b) { return Dual<N>(a) * b; }
template <int N> Dual<N> operator/(const Dual<N>& a, double b) { return a / Dual<N>(b); }
template <int N> Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }
template <int N> Dual<N>& operator+=(Dual<N>& a, const Dual<N>& b) { a = a + b; return a; }

using D2 = Dual<2>;


// accumulator for the force sums: extended precision for plain FP64
template <class T> struct Acc { using type = T; };
template <> struct Acc<double> { using type = long double; };
inline double to_double(long double x) { return (double)x; }
template <int N> inline Dual<N> to_double(const Dual<N>& x) { return x; }

// ---------------------------------------------------------------------------
// collision: TRT (MRT of Sec. 2.1 with Lambda_b = 1), incompressible
// equilibrium with rho0 = 1 (moments of Sec. 2.1), Guo forcing.
// reading: the paper gives no fluid body force; forcing follows Guo et al.
// with the velocity shifted by F/2, split into its even and odd parts.
// ---------------------------------------------------------------------------
template <class T>
void equilibrium(const T& rho, const T u[3], T feq[19]) {
  T uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int q = 0; q < 19; ++q) {
    T cu = CX[q] * u[0] + CY[q] * u[1] + CZ[q] * u[2];
    feq[q] = weight(q) * (rho + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
}

template <class T>
T s_minus(const T& s_plus, double magic) {
  // Lambda = (1/s+ - 1/2)(1/s- - 1/2)  ->  1/s- = 1/2 + Lambda / (1/s+ - 1/2)
  return 1.0 / (0.5 + magic / (1.0 / s_plus - 0.5));
}

template <class T>
void collide(const T f[19], const T& sp, const T& sm, const T F[3], T out[19]) {
  T rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int q = 0; q < 19; ++q) {
    rho = rho + f[q];
    j[0] = j[0] + CX[q] * f[q];
    j[1] = j[1] + CY[q] * f[q];
    j[2] = j[2] + CZ[q] * f[q];
  }
  T u[3];
  for (int a = 0; a < 3; ++a) u[a] = j[a] + 0.5 * F[a];
  T feq[19];
  equilibrium(rho, u, feq);
  T S[19];
  for (int q = 0; q < 19; ++q) {
    T cmu[3] = {CX[q] - u[0], CY[q] - u[1], CZ[q] - u[2]};
    T cu = CX[q] * u[0] + CY[q] * u[1] + CZ[q] * u[2];
    T cF = CX[q] * F[0] + CY[q] * F[1] + CZ[q] * F[2];
    S[q] = weight(q) * (3.0 * (cmu[0] * F[0] + cmu[1] * F[1] + cmu[2] * F[2]) + 9.0 * cu * cF);
  }
  for (int q = 0; q < 19; ++q) {
    int qb = opposite(q);
    T fp = 0.5 * (f[q] + f[qb]), fm = 0.5 * (f[q] - f[qb]);
    T ep = 0.5 * (feq[q] + feq[qb]), em = 0.5 * (feq[q] - feq[qb]);
    T Sp = 0.5 * (S[q] + S[qb]), Sm = 0.5 * (S[q] - S[qb]);
    out[q] = f[q] - sp * (fp - ep) - sm * (fm - em) + (1.0 - 0.5 * sp) * Sp + (1.0 - 0.5 * sm) * Sm;
  }
}

// ---------------------------------------------------------------------------
// MRT collision (Sec. 2.1): C = M^-1 S M.  Moments in a D3Q19 basis that is
// orthogonal with respect to the lattice weights (the basis of Duenweg,
// Schiller and Ladd): density; momentum (3); bulk c^2 - 1; shear 3cx^2 - c^2,
// cy^2 - cz^2, cx cy, cy cz, cz cx; odd ghosts (3c^2 - 5) c_a and
// (cy^2 - cz^2) cx, (cz^2 - cx^2) cy, (cx^2 - cy^2) cz; even ghosts
// 3c^4 - 6c^2 + 1, (2c^2 - 3)(3cx^2 - c^2), (2c^2 - 3)(cy^2 - cz^2).
// Relaxation as the paper assigns it: conserved moments 0; the isotropic
// pair (bulk and the isotropic even ghost) s_b; the shear moments and the
// two tensor even ghosts s_nu; the six odd ghosts s-.  Reading: the rates
// are shared within each isotropy sector, so the operator does not depend on
// which orthogonal basis spans the sectors.  Forcing enters in moment space
// with (I - S/2) (Guo).  s_b from the bulk factor:
// 1/s_b - 1/2 = Lambda_b (1/s_nu - 1/2).
// ---------------------------------------------------------------------------
struct MrtBasis {
  double e[19][19];   // e[a][q]: basis polynomial a at velocity q
  double norm[19];    // sum_q w_q e[a][q]^2
  int rate[19];       // 0 conserved, 1 s_b, 2 s_nu, 3 s-
  MrtBasis() {
    for (int q = 0; q < 19; ++q) {
      const double x = CX[q], y = CY[q], z = CZ[q], c2 = x * x + y * y + z * z;
      const double v[19] = {1.0, x, y, z, c2 - 1.0,
                            3.0 * x * x - c2, y * y - z * z, x * y, y * z, z * x,
                            (3.0 * c2 - 5.0) * x, (3.0 * c2 - 5.0) * y, (3.0 * c2 - 5.0) * z,
                            (y * y - z * z) * x, (z * z - x * x) * y, (x * x - y * y) * z,
                            3.0 * c2 * c2 - 6.0 * c2 + 1.0, (2.0 * c2 - 3.0) * (3.0 * x * x - c2),
                            (2.0 * c2 - 3.0) * (y * y - z * z)};
      for (int a = 0; a < 19; ++a) e[a][q] = v[a];
    }
    for (int a = 0; a < 19; ++a) {
      norm[a] = 0.0;
      for (int q = 0; q < 19; ++q) norm[a] += weight(q) * e[a][q] * e[a][q];
    }
    const int r[19] = {0, 0, 0, 0, 1, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 3, 1, 2, 2};
    for (int a = 0; a < 19; ++a) rate[a] = r[a];
  }
};

inline const MrtBasis& mrt_basis() {
  static const MrtBasis B;
  return B;
}

inline double s_bulk(double snu, double bulk_factor) { return 1.0 / (0.5 + bulk_factor * (1.0 / snu - 0.5)); }

inline void collide_mrt(const double f[19], double snu, double sm, double sb, const double F[3], double out[19]) {
  const MrtBasis& B = mrt_basis();
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int q = 0; q < 19; ++q) {
    rho += f[q];
    j[0] += CX[q] * f[q];
    j[1] += CY[q] * f[q];
    j[2] += CZ[q] * f[q];
  }
  double u[3];
  for (int a = 0; a < 3; ++a) u[a] = j[a] + 0.5 * F[a];
  double feq[19], S[19];
  equilibrium(rho, u, feq);
  for (int q = 0; q < 19; ++q) {
    const double cmu[3] = {CX[q] - u[0], CY[q] - u[1], CZ[q] - u[2]};
    const double cu = CX[q] * u[0] + CY[q] * u[1] + CZ[q] * u[2];
    const double cF = CX[q] * F[0] + CY[q] * F[1] + CZ[q] * F[2];
    S[q] = weight(q) * (3.0 * (cmu[0] * F[0] + cmu[1] * F[1] + cmu[2] * F[2]) + 9.0 * cu * cF);
  }
  const double rates[4] = {0.0, sb, snu, sm};
  double mpost[19];
  for (int a = 0; a < 19; ++a) {
    double m = 0.0, meq = 0.0, ms = 0.0;
    for (int q = 0; q < 19; ++q) {
      m += B.e[a][q] * f[q];
      meq += B.e[a][q] * feq[q];
      ms += B.e[a][q] * S[q];
    }
    const double s = rates[B.rate[a]];
    mpost[a] = m - s * (m - meq) + (1.0 - 0.5 * s) * ms;
  }
  // f = M^-1 m with (M^-1)_{q a} = w_q e_a(q) / norm_a
  for (int q = 0; q < 19; ++q) {
    double v = 0.0;
    for (int a = 0; a < 19; ++a) v += weight(q) * B.e[a][q] * mpost[a] / B.norm[a];
    out[q] = v;
  }
}

// ---------------------------------------------------------------------------
// sphere geometry (Sec. 2.3): a cell is solid iff its centre lies in the
// sphere (reading: |x_c - x_p|^2 <= r^2, minimum image on periodic axes);
// the boundary distance ratio delta_q is the exact ray-sphere root.
// ---------------------------------------------------------------------------
struct Sph {
  double x[3], u[3], w[3];
  double r, rho, cv, cvw;
  int fixed;                    // 0 free, 1 held (u = w = 0), 2 position held, rotation free
  int scheme;                   // virtual-force acceleration: 0 previous step's, 1 and 2 from three velocities
  double uh[2][3], wh[2][3];    // the two velocities before u, w (newest first)
  int nvel;                     // how many of u, uh[0], uh[1] are known (1..3)
  double a[3], b[3];            // accelerations of the previous step
  double Fprev[3], Tprev[3];    // raw hydrodynamic F/T of the previous step
  int have_prev;
  double F[3], T[3];            // raw F^n, T^n of the last step
};

inline double min_image(double d, int n, int periodic) {
  if (!periodic) return d;
  if (d > 0.5 * n) d -= n;
  else if (d < -0.5 * n) d += n;
  return d;
}

inline double link_delta(const double d[3], const int c[3], double r) {
  // |d + delta c|^2 = r^2, smallest root in (0, 1]
  double cc = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
  double dc = d[0] * c[0] + d[1] * c[1] + d[2] * c[2];
  double dd = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  double disc = dc * dc - cc * (dd - r * r);
  if (disc < 0.0) return -1.0;
  return (-dc - std::sqrt(disc)) / cc;
}

// ---------------------------------------------------------------------------
// particle update (FP64): Sec. 2.2 velocity Verlet, Algorithm 1 with the
// virtual force/torque of Sec. 3.3.
// reading: hydrodynamic F/T "averaged over two time steps" is the mean of the
// raw sums of this and the previous step (the first step uses its own);
// a_{t-1} and beta_{t-1} start at zero; rho_f = 1; V_p = 4/3 pi r^3.
// A sphere with fixed == 2 (the rotation test of Sec. 3.4.2: position held,
// rotation free) integrates only the angular part.
// The acceleration inside the virtual force is the previous step's (Sec. 3.3)
// or the alternative the paper attributes to Schwarz et al., the derivative
// of the quadratic through the three most recent velocities u_{n-1},
// u_{n-2}, u_{n-3} (unit steps).  The paper leaves open where it is taken:
// scheme 1 reads it at the new time level, 5/2 u_{n-1} - 4 u_{n-2}
// + 3/2 u_{n-3}; scheme 2 at the newest velocity, 3/2 u_{n-1} - 2 u_{n-2}
// + 1/2 u_{n-3}.  The previous step's acceleration stands in until three
// velocities are known.
// ---------------------------------------------------------------------------
inline void update_particle(Sph& s, const double g[3], const int n[3], const int periodic[3]) {
  double Fav[3], Tav[3];
  for (int a = 0; a < 3; ++a) {
    Fav[a] = s.have_prev ? 0.5 * (s.F[a] + s.Fprev[a]) : s.F[a];
    Tav[a] = s.have_prev ? 0.5 * (s.T[a] + s.Tprev[a]) : s.T[a];
  }
  const double PI = 3.14159265358979323846;
  double V = 4.0 / 3.0 * PI * s.r * s.r * s.r;
  double m = (s.rho + s.cv) * V;                           // virtually increased mass
  double I = 0.4 * (s.rho + s.cvw) * V * s.r * s.r;        // and moment of inertia
  double an[3], bn[3];
  const bool lagrange = s.scheme != 0 && s.nvel >= 3;
  // weights of u_{n-1}, u_{n-2}, u_{n-3}
  const double c0 = s.scheme == 1 ? 2.5 : 1.5, c1 = s.scheme == 1 ? -4.0 : -2.0, c2 = s.scheme == 1 ? 1.5 : 0.5;
  for (int a = 0; a < 3; ++a) {
    double a_est = s.a[a], b_est = s.b[a];
    if (lagrange) {
      a_est = c0 * s.u[a] + c1 * s.uh[0][a] + c2 * s.uh[1][a];
      b_est = c0 * s.w[a] + c1 * s.wh[0][a] + c2 * s.wh[1][a];
    }
    double Fg = (s.rho - 1.0) * g[a] * V;                  // gravity + buoyancy
    double Fv = s.cv * V * a_est;                          // virtual force, m_v a_{t-1}
    double Tv = 0.4 * s.cvw * V * s.r * s.r * b_est;       // virtual torque
    an[a] = (Fav[a] + Fg + Fv) / m;
    bn[a] = (Tav[a] + Tv) / I;
  }
  for (int a = 0; a < 3; ++a) {
    s.uh[1][a] = s.uh[0][a];
    s.uh[0][a] = s.u[a];
    s.wh[1][a] = s.wh[0][a];
    s.wh[0][a] = s.w[a];
  }
  s.nvel = s.nvel < 3 ? s.nvel + 1 : 3;
  for (int a = 0; a < 3; ++a) {
    s.w[a] = s.w[a] + 0.5 * (s.b[a] + bn[a]);
    s.b[a] = bn[a];
    if (s.fixed == 2) continue;
    s.u[a] = s.u[a] + 0.5 * (s.a[a] + an[a]);
    s.x[a] = s.x[a] + s.u[a] + 0.5 * an[a];
    if (periodic[a]) {
      if (s.x[a] < 0.0) s.x[a] += n[a];
      else if (s.x[a] >= n[a]) s.x[a] -= n[a];
    }
    s.a[a] = an[a];
  }
}

// Refill populations (Sec. 2.3, after Dorschner et al.): f^eq(rho, v) minus
// the first-order non-equilibrium part 3 w_q / s+ (c_q c_q - I/3) : S of a
// strain rate S.
inline void refill_populations(double rho, const double v[3], const double S[3][3], double omega, double out[19]) {
  double feq[19];
  equilibrium(rho, v, feq);
  double trS = S[0][0] + S[1][1] + S[2][2];
  for (int q = 0; q < 19; ++q) {
    const int cq[3] = {CX[q], CY[q], CZ[q]};
    double QS = 0.0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) QS += cq[a] * cq[b] * S[a][b];
    QS -= trS / 3.0;
    out[q] = feq[q] - 3.0 * weight(q) / omega * QS;
  }
}

}  // namespace ora
