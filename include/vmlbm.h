/*
 * vmlbm -- MI355X (gfx950) library for the coupled lattice Boltzmann hot path
 * of Werner, Rettinger & Ruede, "Coupling fully resolved light particles with
 * the lattice Boltzmann method on adaptively refined grids":
 *
 *   D3Q19 TRT stream-collide (Sec. 2.1), moving-wall CLI boundary on particle
 *   links (Sec. 2.3, Eq. 10), momentum-exchange link forces and their
 *   per-particle sums (Eqs. 11-12), virtual-mass particle update (Sec. 2.2,
 *   Sec. 3.3, Algorithm 1), cell re-mapping and refill of uncovered cells
 *   (Sec. 2.3), a 2:1 block-refined grid with explosion, coalescence and
 *   sub-cycling (Sec. 4.1-4.2), populations stored as FP64/FP32/FP16
 *   deviations from the lattice weights, and the adjoint of the
 *   fixed-sphere drag with respect to body force and relaxation rate.
 *
 * Units: lattice units of the FINEST level (cell size 1, time step 1,
 * rho0 = 1).  Cell (i,j,k) has its centre at (i+1/2, j+1/2, k+1/2).
 *
 * Every function returns an int status: VMLBM_OK (0) or a negative error.
 * No exception crosses the boundary.  vmlbm_last_error() returns a message
 * owned by the context, valid until its next call.  A context is used from
 * one host thread at a time.
 *
 * Memory: the caller owns the device workspace (vmlbm_required_bytes, then
 * vmlbm_bind_workspace with a device pointer that outlives the context) and
 * every host buffer.  The library never allocates or frees device memory
 * except a few bytes of pinned host memory for status read-back.
 * All device work is enqueued on the bound stream; read functions
 * synchronise that stream.
 */
#ifndef VMLBM_H
#define VMLBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif
#pragma GCC visibility push(default)

#define VMLBM_OK 0
#define VMLBM_EINVAL (-1)     /* bad argument */
#define VMLBM_ENOMEM (-2)     /* workspace too small / host allocation failed */
#define VMLBM_EDEVICE (-3)    /* HIP runtime error */
#define VMLBM_ESTATE (-4)     /* call out of order */
#define VMLBM_EUNSTABLE (-5)  /* non-finite population, force or torque seen */
#define VMLBM_ERANGE (-6)     /* geometry outside the supported range */

typedef struct vmlbm_ctx vmlbm_ctx;

typedef enum { VMLBM_F64 = 0, VMLBM_F32 = 1, VMLBM_F16 = 2 } vmlbm_storage;

typedef struct {
  int n[3];                   /* uniform grid: cells in x, y, z.
                                 refined grid: COARSEST-level cells */
  int block;                  /* 0 = one uniform grid; else cells per block edge
                                 (16) of the block-structured grid (Sec. 4.1) */
  int levels;                 /* refinement levels, 1..9 (block > 0) */
  int periodic[3];            /* 1 periodic, 0 halfway no-slip walls at both ends */
  double wall_velocity[2][3]; /* velocity of the low/high wall of the first
                                 non-periodic axis (other walls rest) */
  double omega;               /* s_nu = s+ of TRT on the finest level (Sec. 2.1);
                                 coarser levels follow acoustic scaling */
  double magic;               /* Lambda of Sec. 2.1 (3/16) */
  double body_force[3];       /* fluid force density, finest-level units */
  double gravity[3];          /* acts on particles only (Sec. 2.2) */
  int storage;                /* vmlbm_storage of the populations */
  int check_every;            /* refinement check period in coarse steps */
  int history;                /* per-step F/T/x/u ring buffer length (>= 1) */
  int adjoint_steps;          /* > 0: reserve workspace for vmlbm_forward_ckpt
                                 with this many steps */
  int ckpt_every;             /* checkpoint period of the adjoint forward pass */
  double bulk_factor;         /* Lambda_b of the MRT collision (Sec. 2.1):
                                 1/s_b - 1/2 = Lambda_b (1/s_nu - 1/2) on every
                                 level; 0 or 1 selects TRT.  The adjoint
                                 supports TRT only. */
  double curl_threshold;      /* refined grid: sigma_c of the curl sensor
                                 phi = |curl u| s^(3/2) (Sec. 4.2.2, Eq. 23;
                                 s the cell edge in finest cells); at every
                                 layout check a leaf block whose max phi
                                 exceeds sigma_c is refined, one below
                                 curl_coarsen * sigma_c coarsened.  0 = off */
  double curl_coarsen;        /* c of Sec. 4.2.2 (the paper advises c <= 0.35) */
  int max_blocks;             /* refined grid with the curl sensor: block
                                 slots per level (the flow decides how many
                                 it needs); 0 = every block position of the
                                 level.  A layout that needs more fails with
                                 VMLBM_ERANGE. */
} vmlbm_config;

typedef struct {
  double x[3], u[3], w[3];    /* centre, velocity, angular velocity */
  double radius;              /* r_p in cells */
  double density_ratio;       /* pi_p = rho_p / rho_f */
  double cv, cv_omega;        /* virtual mass coefficients C_v, C_v,omega (Sec. 3.3) */
  int fixed;                  /* 0: free; 1: held in place, surface velocity
                                 0; 2: position held, rotation free (the
                                 rotation test of Sec. 3.4.2) */
  int vm_scheme;              /* acceleration inside the virtual force and
                                 torque (Sec. 3.3): 0 the previous step's;
                                 1 / 2 the derivative of the quadratic
                                 through the three most recent velocities
                                 (the Lagrange alternative after Schwarz et
                                 al.) at the new time level / at the newest
                                 velocity; the previous step's until three
                                 velocities are known */
} vmlbm_sphere;

/* Create a context from a configuration (copied).  *out receives it. */
int vmlbm_create(const vmlbm_config* cfg, vmlbm_ctx** out);

/* Register a sphere (Sec. 2.2) before the workspace is bound.  *id receives
 * its index.  Spheres must lie at least 3 cells apart. */
int vmlbm_add_sphere(vmlbm_ctx* ctx, const vmlbm_sphere* s, int* id);

/* Block-structured grid: hold the blocks intersecting the coarse-cell box
 * [lo, hi) at level >= `level` (Sec. 4.2), before the workspace is bound. */
int vmlbm_add_refine_region(vmlbm_ctx* ctx, const int lo[3], const int hi[3], int level);

/* Device workspace size in bytes for the current configuration and spheres. */
int vmlbm_required_bytes(const vmlbm_ctx* ctx, size_t* bytes);

/* Bind caller-owned device memory of at least vmlbm_required_bytes (256-byte
 * aligned).  It must outlive the context; the library never frees it. */
int vmlbm_bind_workspace(vmlbm_ctx* ctx, void* dev_ptr, size_t bytes);

/* HIP stream (hipStream_t) for all device work; NULL = default stream. */
int vmlbm_set_stream(vmlbm_ctx* ctx, void* hip_stream);

/* Map the spheres (Sec. 2.3) and set f(0) = f^eq(rho, u0) on fluid cells
 * (Sec. 2.1 moments).  u0 is a host array [3][nz][ny][nx] of the finest
 * (uniform) grid, or NULL for rest. */
int vmlbm_init_equilibrium(vmlbm_ctx* ctx, double rho, const double* u0);

/* Advance n steps (coarse steps on a refined grid) following Algorithm 1.
 * Asynchronous on the bound stream. */
int vmlbm_step(vmlbm_ctx* ctx, int n);

/* Wait for the stream; returns VMLBM_EUNSTABLE if a non-finite density,
 * force or torque was flagged, VMLBM_ERANGE if a particle left its range. */
int vmlbm_sync(vmlbm_ctx* ctx);

/* Particle state after the last step: centre, velocity and angular velocity
 * from the virtual-mass update (Sec. 3.3, Eqs. 16-20; Algorithm 1). */
int vmlbm_get_particle(vmlbm_ctx* ctx, int id, double x[3], double u[3], double w[3]);

/* Change how sphere id moves from the next step on, its position unchanged
 * (Sec. 3.4.2 holds a sphere until the flow has developed, then lets it
 * rotate).  fixed as in vmlbm_sphere; u is read when fixed = 0, w when fixed
 * != 1 (else velocities are set to 0).  The previous accelerations and F/T
 * are kept, so a released sphere starts from its held state.  fixed = 0 is
 * refused (VMLBM_EINVAL) unless a sphere was added free, since only then are
 * the re-mapping paths active.  Synchronises the stream. */
int vmlbm_set_sphere_motion(vmlbm_ctx* ctx, int id, const double u[3], const double w[3], int fixed);

/* Raw hydrodynamic force and torque F^n, T^n (Eq. 12) of the last (finest)
 * step, before the two-step average of Algorithm 1. */
int vmlbm_get_force_torque(vmlbm_ctx* ctx, int id, double F[3], double T[3]);

/* Last n history records of sphere id, oldest first: out[n][15] =
 * F^n, T^n, x, u, w after each step.  n <= history and <= steps done. */
int vmlbm_get_history(vmlbm_ctx* ctx, int id, int n, double* out);

/* Post-collision populations f~(n) of a level (uniform grid: level 0): the
 * state the next step's streaming pulls from (Sec. 2.1, the collision and
 * streaming of Eq. 1).  The library stores only this state, not the
 * pre-collision f(n), which is one pull away.  FP64, host array
 * [19][cells] in the canonical D3Q19 order
 * (rest; +x,-x,+y,-y,+z,-z; xy, xz, yz diagonals).  Uniform grid: cells in
 * [nz][ny][nx] order.  Refined grid: [block][16][16][16] in the order of
 * vmlbm_level_blocks.  Solid cells read 0. */
int vmlbm_read_populations(vmlbm_ctx* ctx, int level, double* out);

/* Overwrite the post-collision populations of a level (same layout).  The
 * deviation f - w is rounded once to the storage precision, to nearest with
 * ties to even.  For tests and fault injection. */
int vmlbm_write_populations(vmlbm_ctx* ctx, int level, const double* in);

/* Particle owner per cell of a level (the mapping of Sec. 2.3: a cell is
 * solid for the sphere whose centre lies within r of the cell centre):
 * -1 fluid, else sphere id. */
int vmlbm_read_owner(vmlbm_ctx* ctx, int level, int* out);

/* Density and velocity per cell of a level (the moments of Sec. 2.1,
 * rho = sum f, u = sum c f + F / 2 with the forcing shift of the fluid body
 * force): rho [cells], u [3][cells], from the post-collision state; solid
 * cells read 0. */
int vmlbm_read_fields(vmlbm_ctx* ctx, int level, double* rho, double* u);

/* Cell updates performed and device seconds measured so far by vmlbm_step. */
int vmlbm_stats(vmlbm_ctx* ctx, double* cell_updates, double* seconds);

/* Kernel timing: when enabled, HIP events on the bound stream bracket every
 * launch of the interior stream-collide sweep kernel; vmlbm_sweep_time
 * returns their summed duration and launch count (synchronises). */
int vmlbm_profile(vmlbm_ctx* ctx, int enable);
int vmlbm_sweep_time(vmlbm_ctx* ctx, double* seconds, long long* launches);

/* Bandwidth reference, not part of the method: a plain device copy of
 * `bytes` (a multiple of 16) from src to dst, device pointers that must not
 * overlap, with one 16-byte load and one streaming 16-byte store per thread,
 * enqueued on `stream` (a hipStream_t; NULL = default stream).  The
 * sweeps' fraction of HBM bandwidth is read against what this copy
 * reaches.  VMLBM_EINVAL for a size that is not a multiple of 16. */
int vmlbm_stream_copy(void* dst, const void* src, size_t bytes, void* stream);

/* Bandwidth reference, not part of the method: the memory access pattern of
 * the interior stream-collide sweep (Sec. 2.1, the pull form of Eq. 1)
 * without its arithmetic.  src and dst hold 19 populations of a periodic
 * n[0] x n[1] x n[2] box in storage format `storage` (VMLBM_F64, VMLBM_F32
 * or VMLBM_F16) and in the uniform grid's population layout for that
 * format: element (q, x, y, z) at q n0 n1 + z 19 n0 n1 + y n0 + x for FP16
 * (the 19 populations of a z-plane side by side), at q n0 n1 n2 + z n0 n1 +
 * y n0 + x otherwise.  Every cell gets dst[q][x] = src[q][x - c_q], with
 * streaming stores, enqueued on `stream`.
 * Device pointers, not overlapping, each 19 n[0] n[1] n[2] elements.
 * VMLBM_EINVAL for null pointers or a bad storage, VMLBM_ERANGE for
 * n[1] or n[2] outside 1..65535 or n[0] < 1. */
int vmlbm_stream_pull(void* dst, const void* src, int storage, const int n[3], void* stream);

/* Bandwidth reference, not part of the method: the memory access pattern of
 * one level's sweep on the block-structured grid (Sec. 4.1; the pull form
 * of Eq. 1 in 16^3-cell blocks) without its arithmetic.  Every cell of the
 * level's leaf blocks takes population q from x - c_q (periodic, through the
 * level's blocks as the sweep reads them; a source in a block the level does
 * not store gives 0) and stores it unchanged, with the sweep's workgroup
 * numbering and streaming stores; no flags, collision or rounding.  The
 * pulled state becomes the level's current state; `reps` such pulls are
 * enqueued on the context's stream (asynchronous, like vmlbm_step).  On a
 * single-level periodic grid one pull is the exact periodic shift of each
 * population by c_q.  VMLBM_ESTATE on a uniform grid, without a workspace or
 * before vmlbm_init_equilibrium; VMLBM_EINVAL for a level outside 0..L or
 * reps < 1. */
int vmlbm_level_pull(vmlbm_ctx* ctx, int level, int reps);

/* Totals of the post-collision state over fluid cells: mass sum f~ and
 * momentum sum c f~, the conserved moments of Sec. 2.1 (refined grid: every
 * level weighted by its cell volume 8^-l in coarse units, the volume scaling
 * of Sec. 4.1).  Deterministic device reduction; synchronises. */
int vmlbm_totals(vmlbm_ctx* ctx, double* mass, double mom[3]);

/* vmlbm_totals for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * sums, bit for bit, with the per-workgroup partials in a file-scope device
 * array of 1024 x 8 doubles (64 KiB) instead of the workspace, read back
 * into a stack buffer; no allocation routine is called.  Each GPU the
 * library runs on holds its own copy of the array until the process ends;
 * its address is looked up when a workspace is bound on that GPU.  The
 * array does not grow with the grid (the reduction strides over the
 * cells), so no grid is too large for it.  All calls on one GPU share the
 * array: calls that overlap on one GPU (on other host threads or streams)
 * race.  Every partial is written before it is read, so nothing needs
 * clearing between calls.  Synchronises the context's stream;
 * VMLBM_ESTATE if no workspace is bound. */
int vmlbm_totals_static(vmlbm_ctx* ctx, double* mass, double mom[3]);

/* Uniform grid: post-collision populations f~(n) (as vmlbm_read_populations,
 * Sec. 2.1) of the cells of a box (periodic wrap), FP64 host array
 * [19][size2][size1][size0]; solid cells read 0. */
int vmlbm_read_box(vmlbm_ctx* ctx, const int lo[3], const int size[3], double* out);

/* Cells of a level that are fluid, and fluid cells without any wall or
 * particle link (those the interior sweep updates; link cells are those with
 * a lattice link into a solid cell or a wall, Sec. 2.3). */
int vmlbm_cell_counts(vmlbm_ctx* ctx, int level, long long* fluid, long long* interior);

/* Block list of a refined level (the leaf blocks of that level in the
 * block-structured grid of Sec. 4.1): *count blocks; if origin != NULL it
 * gets [count][3] block origins in that level's cell units. */
int vmlbm_level_blocks(vmlbm_ctx* ctx, int level, int* count, int* origin);

/* Number of re-refinements performed so far (Sec. 4.2). */
int vmlbm_refinements(vmlbm_ctx* ctx, int* count);

/* Of those, the number whose host tables were built ahead on a host thread
 * (the block ranges of the next layout change predicted from the spheres'
 * velocities while the device stepped) rather than at the layout check.
 * The tables are the same either way; this counts where the build ran. */
int vmlbm_prebuilt_layouts(vmlbm_ctx* ctx, int* count);

/* Set the differentiable parameters: body force magnitude along +z and
 * omega (Lambda held fixed, so s- follows omega).  Checkpoints of an earlier
 * vmlbm_forward_ckpt no longer count: vmlbm_adjoint then needs a new forward
 * pass. */
int vmlbm_set_params(vmlbm_ctx* ctx, double body_force_z, double omega);

/* Forward pass for the time-averaged drag of a fixed sphere:
 *   J = 1/(n_steps - avg_from) * sum_{n=avg_from}^{n_steps-1} F_z^n
 * from f(0) = w, storing a checkpoint every ckpt_every steps.  Requires
 * config.adjoint_steps >= n_steps and ckpt_every == config.ckpt_every. */
int vmlbm_forward_ckpt(vmlbm_ctx* ctx, int sphere, int n_steps, int avg_from, int ckpt_every,
                       double* J);

/* Reverse pass of the last vmlbm_forward_ckpt: grad = dJ * (dJ/dF_z, dJ/domega)
 * by the discrete adjoint with segment recomputation.  VMLBM_ESTATE if no
 * forward pass ran since the parameters were last set. */
int vmlbm_adjoint(vmlbm_ctx* ctx, double dJ, double grad[2]);

/* Destroy the context (the workspace stays the caller's). */
int vmlbm_destroy(vmlbm_ctx* ctx);

const char* vmlbm_last_error(const vmlbm_ctx* ctx);

#pragma GCC visibility pop
#ifdef __cplusplus
}
#endif
#endif
