/*
 * CPU oracle for the coupled lattice Boltzmann hot path -- TEST INFRASTRUCTURE.
 *
 * A plain, slow, FP64 implementation of what the GPU library computes, written
 * from the paper (Werner, Rettinger, Ruede: coupling fully resolved light
 * particles with the LBM on adaptively refined grids).  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg load it.  It shares no
 * code, header, table or helper with the GPU library.
 *
 * The refill of an uncovered cell follows a scheme the paper only cites; its
 * populations given a strain rate are pinned by their moments, and its
 * strain-rate estimate (central differences over the axis neighbours) by
 * linear velocity fields, which it must reproduce exactly.
 *
 * Conventions: lattice units of the finest level; cell (i,j,k) has its centre
 * at (i+1/2, j+1/2, k+1/2); population arrays are [19][nz][ny][nx] C order.
 * All functions return 0 on success and a negative value on error.
 */
#ifndef VMLBM_ORACLE_H
#define VMLBM_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int n[3];                 /* cells in x, y, z */
  int periodic[3];          /* 1 periodic, 0 halfway no-slip wall at both ends */
  double wall_velocity[2][3]; /* low/high wall of the first non-periodic axis */
  double omega;             /* s_nu (= s+ of TRT) */
  double magic;             /* Lambda */
  double body_force[3];     /* fluid force density (Guo forcing) */
  double gravity[3];        /* acts on particles only */
  double bulk_factor;       /* Lambda_b of the MRT collision; 0 or 1 = TRT */
} ora_config;

typedef struct {
  double x[3], u[3], w[3];
  double radius, density_ratio, cv, cv_omega;
  int fixed;                /* 0 free, 1 held (u = w = 0), 2 position held, rotation free */
  int vm_scheme;            /* acceleration in the virtual force: 0 previous step's (Sec. 3.3);
                               derivative of the quadratic through three velocities at the new
                               time level (1) or at the newest velocity (2) */
} ora_sphere;

/* lattice tables in the oracle's order */
void ora_lattice(int c[19][3], double w[19], int opp[19]);

/* single-cell TRT collision with Guo forcing on full populations f[19] */
void ora_collide_cell(const double f[19], double omega, double magic,
                      const double F[3], double out[19]);
/* single-cell MRT collision (explicit moment basis) with bulk factor Lambda_b */
void ora_collide_cell_mrt(const double f[19], double omega, double magic, double bulk_factor,
                          const double F[3], double out[19]);
/* the MRT moment basis: e[a][q] and the weighted norms sum_q w_q e[a][q]^2 */
void ora_mrt_basis(double e[19][19], double norm[19]);
/* incompressible equilibrium f^eq(rho, u) */
void ora_equilibrium(double rho, const double u[3], double out[19]);
/* populations of a refilled cell from density, velocity and a strain rate
 * S[3][3] (row-major): f^eq(rho, v) - 3 w_q / omega (c_q c_q - I/3) : S */
void ora_refill_populations(double rho, const double v[3], const double S[9], double omega, double out[19]);
/* boundary distance ratio along c from a fluid point at offset d from a
 * sphere centre; returns -1 if the segment does not enter the sphere */
double ora_link_delta(const double d[3], const int c[3], double radius);

/* ---- uniform grid ---- */
void* ora_create(const ora_config* cfg);
int ora_add_sphere(void* h, const ora_sphere* s);
int ora_init(void* h, double rho, const double* u0 /* [3][nz][ny][nx] or NULL */);
/* same with a density per cell ([nz][ny][nx]) */
int ora_init_fields(void* h, const double* rho, const double* u0);
int ora_step(void* h, int nsteps);
/* Refill of cell (x,y,z) uncovered by sphere pid (Sec. 2.3), computed on the
 * pre-collision state f_pre [19][cells] with the mapping before the
 * re-mapping old_owner [cells] (-1 fluid, else sphere id), with the spheres'
 * current states; out[19] = its pre-collision populations.  The grid's own
 * state is replaced by f_pre.  Test entry point. */
int ora_refill_cell(void* h, const double* f_pre, const int* old_owner, int x, int y, int z, int pid,
                    double out[19]);
int ora_post_collision(void* h, double* out);  /* f~(n), solid cells = 0 */
int ora_pre_collision(void* h, double* out);   /* f(n), solid cells = 0 */
int ora_owner(void* h, int* out);              /* -1 fluid, else sphere id */
int ora_force_torque(void* h, int id, double F[3], double T[3]); /* raw F^n of last step */
int ora_particle(void* h, int id, double x[3], double u[3], double w[3]);
/* new velocities and hold mode of a sphere, position unchanged (u = 0 when
 * held, w = 0 when fixed = 1); accelerations and last F/T are kept */
int ora_set_sphere_motion(void* h, int id, const double u[3], const double w[3], int fixed);
int ora_fields(void* h, double* rho, double* u /* [3][cells] */);
int ora_steps_done(void* h);
void ora_destroy(void* h);

/* total mass and momentum over fluid cells of the pre-collision state */
int ora_totals(void* h, double* mass, double mom[3]);

/* Exact derivative of the time-averaged drag
 *   J = 1/(n_steps-avg_from) * sum_{n=avg_from}^{n_steps-1} F_z^n
 * with respect to (body force magnitude along +z, omega), magic held fixed,
 * by forward propagation of dual numbers.  Fixed spheres only, start f = w. */
int ora_drag_gradient(const ora_config* cfg, const ora_sphere* spheres, int nspheres,
                      int n_steps, int avg_from, double* J, double grad[2]);
/* Same forward map, value only (for finite differences) */
int ora_drag_value(const ora_config* cfg, const ora_sphere* spheres, int nspheres,
                   int n_steps, int avg_from, double* J);

/* particle update alone (no fluid): nsteps updates with raw hydrodynamic
 * force F + k dF at update k and constant T; out[nsteps][15] = x, u, w, a,
 * beta after each step.  s->fixed = 2 integrates the rotation only; other
 * values move freely. */
int ora_vm_trajectory(const ora_sphere* s, const double F[3], const double dF[3], const double T[3],
                      const double g[3], int nsteps, double* out);

int ora_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
