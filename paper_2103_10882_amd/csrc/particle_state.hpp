// Particle record shared by the sweep's boundary pass, the mapping kernels
// and the particle update.
#pragma once

namespace vm {

// ---------------------------------------------------------------------------
// particle record (FP64), one per sphere, in device memory
// ---------------------------------------------------------------------------
struct DevParticle {
  double x[3], u[3], w[3];
  double xold[3];              // position the mapping in place was made with (before the last update)
  double a[3], b[3];           // translational / angular acceleration of the previous step
  double F[3], T[3];           // raw hydrodynamic F^n, T^n of the last step
  double Fprev[3], Tprev[3];   // of the step before
  double uh[2][3], wh[2][3];   // the two velocities before u, w (newest first)
  double r, rho, cv, cvw;
  int fixed, have_prev;        // fixed: 0 free, 1 held (u = w = 0), 2 position held, rotation free
  int scheme, nvel;            // virtual-force acceleration scheme; known velocities of u, uh (1..3)
  int box_lo[3];               // box of the coming sweep (holds every link cell)
  int remap_lo[3];             // re-mapping region origin (old and new position)
};

}  // namespace vm
