"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds workload parameters and random draws only.  It contains none
of the lattice Boltzmann / coupling arithmetic: both the CPU oracle and the GPU
library receive what is produced here as plain inputs.

Workloads (lattice units of the finest level, cell (i,j,k) has its centre at
(i+1/2, j+1/2, k+1/2)):

* ``tiny``      periodic 32^3 box, fixed sphere r=6 in the centre, body force
                1e-5 along z, equilibrium start perturbed by U(-1e-3, 1e-3).
* ``rising``    256^3, x/y periodic, no-slip walls at z=0 and z=256, one light
                sphere (density ratio 0.5, r=12, C_v=0.5) released at rest at
                (128,128,64); Galileo number 150 (Eq. 13 with u_g=0.01).
* ``refined``   3-level block grid (16^3 blocks), coarse 128x128x512, periodic,
                sphere r=16 finest cells, density ratio 0.1, C_v=0.5, Ga=250,
                centre (64.3, 63.8, 63.0) in coarse cells (off block faces).
* ``precision`` 512^3 periodic, 8 fixed spheres r=20 at seeded positions,
                body force 1e-5 along z.
* ``adjoint``   128^3 periodic, fixed sphere r=10 in the centre, body force
                1e-5 along z, omega=1.6; drag averaged over steps 1500..1999.

Validation workloads of Sec. 3 (MRT with bulk factor 100, the paper's default):

* ``light_box`` periodic (6.4, 6.4, 12.8) d_p box, sphere of diameter d_p at
                (3.2, 3.2, 0.6) d_p released at rest, gravity along -z at a
                Galileo number (Sec. 3.1 and 3.4.1).  Gravity and buoyancy
                act on the sphere only; the fluid is unforced.
* ``amr_box``   refinement validation of Sec. 4.3 at a smaller sphere: periodic
                (7.68, 7.68, 53.76) d_p box, sphere of diameter d_p released at
                (3.84, 3.84, 0.6) d_p, Ga 300, density ratio 0.5, plain MEM;
                either the uniform finest grid or 3 levels of 16^3 blocks.
* ``rotation_box`` (12.8, 6.4, 4.8) d_p, walls at z = 0 (rest) and z = 4.8 d_p
                (moving at u_w = 0.1 along x), periodic in x and y, Couette
                start, sphere of diameter d_p held at the centre (Sec. 3.4.2);
                Re_p = (u_w / 2) d_p / nu.

Galileo-number parameterisation (Eq. 13): u_g = sqrt(|pi_p-1| g d_p) = 0.01,
Ga = u_g d_p / nu, and nu = (1/omega - 1/2)/3 in lattice units.  The derived
numbers are written out below next to the inputs they come from.
"""
import numpy as np

U_G = 0.01          # gravitational velocity in lattice units (Sec. 3.1)
MAGIC = 3.0 / 16.0  # TRT magic parameter (Sec. 2.1)


def _ga_params(ga, density_ratio, d_p):
    """Viscosity, omega and gravity for a Galileo number (Eq. 13)."""
    nu = U_G * d_p / ga
    omega = 1.0 / (3.0 * nu + 0.5)
    g = U_G * U_G / (abs(density_ratio - 1.0) * d_p)
    return nu, omega, g


def base_config(n, periodic=(1, 1, 1), omega=1.6, body_force=(0.0, 0.0, 0.0),
                gravity=(0.0, 0.0, 0.0), wall_velocity=((0.0, 0.0, 0.0), (0.0, 0.0, 0.0))):
    return {
        "n": tuple(int(v) for v in n),
        "periodic": tuple(int(v) for v in periodic),
        "omega": float(omega),
        "magic": MAGIC,
        "body_force": tuple(float(v) for v in body_force),
        "gravity": tuple(float(v) for v in gravity),
        "wall_velocity": tuple(tuple(float(v) for v in w) for w in wall_velocity),
    }


def sphere(x, radius, density_ratio=1.0, cv=0.0, cv_omega=None, fixed=True,
           u=(0.0, 0.0, 0.0), w=(0.0, 0.0, 0.0), vm_scheme=0):
    """fixed: True held in place, False free, 2 position held with free
    rotation.  vm_scheme: acceleration inside the virtual force, 0 the
    previous step's, 1 / 2 the derivative of the quadratic through the three
    most recent velocities at the new time level / at the newest velocity."""
    return {
        "x": tuple(float(v) for v in x),
        "u": tuple(float(v) for v in u),
        "w": tuple(float(v) for v in w),
        "radius": float(radius),
        "density_ratio": float(density_ratio),
        "cv": float(cv),
        "cv_omega": float(cv if cv_omega is None else cv_omega),
        "fixed": 2 if (fixed == 2 and fixed is not True) else int(bool(fixed)),
        "vm_scheme": int(vm_scheme),
    }


def velocity_perturbation(n, seed=0, amplitude=1e-3):
    """One draw of U(-a, a) for the full C-order [3][nz][ny][nx] array."""
    nx, ny, nz = n
    rng = np.random.default_rng(seed)
    return rng.uniform(-amplitude, amplitude, size=(3, nz, ny, nx))


def vortex_tube(n, centre, core, amplitude):
    """Gaussian vortex tube along y through (x0, z0) = centre (cell-centre
    coordinates): u_x = -A dz g, u_z = A dx g with g = exp(-(dx^2 + dz^2) /
    core^2), minimum-image offsets in the periodic box; [3][nz][ny][nx]."""
    nx, ny, nz = n
    x = np.arange(nx) + 0.5 - centre[0]
    z = np.arange(nz) + 0.5 - centre[1]
    x -= nx * np.round(x / nx)
    z -= nz * np.round(z / nz)
    dz, dx = np.meshgrid(z, x, indexing="ij")
    g = np.exp(-(dx * dx + dz * dz) / (core * core))
    u = np.zeros((3, nz, ny, nx))
    u[0] = (-amplitude * dz * g)[:, None, :]
    u[2] = (amplitude * dx * g)[:, None, :]
    return u


def place_spheres(n, count, radius, gap, seed=0):
    """Centres uniform in the periodic box, rejected when the minimum-image
    centre distance to an accepted one is below 2r + gap; accepted in draw
    order."""
    rng = np.random.default_rng(seed)
    box = np.array(n, dtype=np.float64)
    out = []
    min_d = 2.0 * radius + gap
    tries = 0
    while len(out) < count:
        tries += 1
        if tries > 100000:
            raise RuntimeError("sphere placement did not converge")
        c = rng.uniform(0.0, 1.0, size=3) * box
        ok = True
        for o in out:
            d = c - o
            d -= box * np.round(d / box)
            if np.sqrt(np.dot(d, d)) < min_d:
                ok = False
                break
        if ok:
            out.append(c)
    return [tuple(float(v) for v in c) for c in out]


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------

def tiny(n=32, radius=6.0):
    c = n / 2.0
    cfg = base_config((n, n, n), omega=1.6, body_force=(0.0, 0.0, 1e-5))
    return {
        "name": f"tiny{n}",
        "config": cfg,
        "spheres": [sphere((c, c, c), radius, fixed=True)],
        "u0": velocity_perturbation((n, n, n), seed=0),
        "steps": 200,
    }


def rising(n=(256, 256, 256), radius=12.0, height=64.0, ga=150.0, density_ratio=0.5, cv=0.5):
    _, omega, g = _ga_params(ga, density_ratio, 2.0 * radius)
    cfg = base_config(n, periodic=(1, 1, 0), omega=omega, gravity=(0.0, 0.0, -g))
    return {
        "name": "rising%dx%dx%d" % tuple(n),
        "config": cfg,
        "spheres": [sphere((n[0] / 2.0, n[1] / 2.0, height), radius, density_ratio=density_ratio,
                           cv=cv, fixed=False)],
        "u0": None,
        "steps": 2000,
    }


def precision(n=512, count=8, radius=20.0, seed=0):
    cfg = base_config((n, n, n), omega=1.6, body_force=(0.0, 0.0, 1e-5))
    centres = place_spheres((n, n, n), count, radius, gap=4.0, seed=seed)
    return {
        "name": f"precision{n}",
        "config": cfg,
        "spheres": [sphere(c, radius, fixed=True) for c in centres],
        "u0": None,
        "steps": 1000,
    }


def adjoint(n=128, radius=10.0, steps=2000, avg_from=1500, ckpt_every=50):
    c = n / 2.0
    cfg = base_config((n, n, n), omega=1.6, body_force=(0.0, 0.0, 1e-5))
    return {
        "name": f"adjoint{n}",
        "config": cfg,
        "spheres": [sphere((c, c, c), radius, fixed=True)],
        "u0": None,
        "steps": steps,
        "avg_from": avg_from,
        "ckpt_every": ckpt_every,
    }


def refined(coarse=(128, 128, 512), levels=3, block=16, radius=16.0, ga=250.0,
            density_ratio=0.1, cv=0.5, centre_coarse=(64.3, 63.8, 63.0)):
    """Rising light sphere on a 3-level grid.  The centre sits off block
    boundaries: with r + b a whole number of blocks, a centre on a block face
    makes the refinement box flip with round-off-sized lateral motion."""
    _, omega_f, g = _ga_params(ga, density_ratio, 2.0 * radius)
    scale = 2 ** (levels - 1)
    cfg = base_config(coarse, omega=omega_f, gravity=(0.0, 0.0, -g))
    cfg["levels"] = levels
    cfg["block"] = block
    return {
        "name": "refined%dx%dx%d_L%d" % (coarse + (levels,)),
        "config": cfg,
        "spheres": [sphere(tuple(v * scale for v in centre_coarse), radius,
                           density_ratio=density_ratio, cv=cv, fixed=False)],
        "u0": None,
        "steps": 500,
    }


def light_box(d_p, density_ratio, ga=100.0, cv=0.0, bulk_factor=100.0, compensate=False, vm_scheme=0):
    """Rising (or settling) sphere in a periodic box (Sec. 3.1, Table 1 and
    Sec. 3.4.1, Table 2).  d_p a multiple of 5 keeps the box whole.  The
    fluid is unforced, so the box gains the sphere's net weight as momentum
    (the reading whose Re_p matches Table 2); compensate=True adds a uniform
    fluid force that cancels it instead."""
    n = (int(round(6.4 * d_p)), int(round(6.4 * d_p)), int(round(12.8 * d_p)))
    nu, omega, g = _ga_params(ga, density_ratio, float(d_p))
    r = 0.5 * d_p
    vol = 4.0 / 3.0 * np.pi * r ** 3
    f_ext = (density_ratio - 1.0) * vol * (-g)        # net weight on the sphere, along z
    fz = -f_ext / (n[0] * n[1] * n[2] - vol) if compensate else 0.0   # per fluid cell, opposite
    cfg = base_config(n, omega=omega, body_force=(0.0, 0.0, fz), gravity=(0.0, 0.0, -g))
    cfg["bulk_factor"] = float(bulk_factor)
    return {
        "name": "lightbox_d%d_pi%g_ga%g_cv%g_s%d" % (d_p, density_ratio, ga, cv, vm_scheme),
        "config": cfg,
        "spheres": [sphere((3.2 * d_p, 3.2 * d_p, 0.6 * d_p), r, density_ratio=density_ratio, cv=cv,
                           fixed=False, vm_scheme=vm_scheme)],
        "u0": None,
        "nu": nu,
        "t_g": d_p / U_G,
    }


def rotation_box(d_p, density_ratio, cv=0.0, re_p=110.0, u_w=0.1, bulk_factor=100.0):
    """Couette-driven sphere held at the centre, later free to rotate
    (Sec. 3.4.2).  d_p a multiple of 5 keeps the box whole."""
    n = (int(round(12.8 * d_p)), int(round(6.4 * d_p)), int(round(4.8 * d_p)))
    u_p = 0.5 * u_w
    nu = u_p * d_p / re_p
    omega = 1.0 / (3.0 * nu + 0.5)
    cfg = base_config(n, periodic=(1, 1, 0), omega=omega, wall_velocity=((0.0, 0.0, 0.0), (u_w, 0.0, 0.0)))
    cfg["bulk_factor"] = float(bulk_factor)
    H = n[2]
    z = np.arange(H) + 0.5
    u0 = np.zeros((3, H, n[1], n[0]))
    u0[0] = (u_w * z / H)[:, None, None]
    return {
        "name": "rotation_d%d_pi%g_cv%g" % (d_p, density_ratio, cv),
        "config": cfg,
        "spheres": [sphere((6.4 * d_p, 3.2 * d_p, 2.4 * d_p), 0.5 * d_p, density_ratio=density_ratio, cv=cv,
                           fixed=True)],
        "u0": u0,
        "nu": nu,
        "t_c": d_p / u_p,
        "omega_c": u_p / d_p,
    }


def amr_box(d_p=25, refined=False, ga=300.0, density_ratio=0.5, levels=3, bulk_factor=100.0,
            curl_threshold=0.0, curl_coarsen=0.2):
    """Rising sphere of Sec. 4.3 (uniform against adaptively refined grid).
    The finest grid has (7.68, 7.68, 53.76) d_p cells; d_p = 25 makes that
    (192, 192, 1344), whole 16^3 blocks of the coarsest of 3 levels.  The
    refined grid holds the finest level around the sphere (and, with a curl
    threshold, wherever the flow asks for it)."""
    scale = 2 ** (levels - 1)
    n = (int(round(7.68 * d_p)), int(round(7.68 * d_p)), int(round(53.76 * d_p)))
    _, omega, g = _ga_params(ga, density_ratio, float(d_p))
    centre = (3.84 * d_p, 3.84 * d_p, 0.6 * d_p)
    if refined:
        if any(v % (16 * scale) for v in n):
            raise ValueError("the finest grid must hold whole coarsest blocks")
        cfg = base_config(tuple(v // scale for v in n), omega=omega, gravity=(0.0, 0.0, -g))
        cfg["levels"] = levels
        cfg["block"] = 16
        cfg["curl_threshold"] = float(curl_threshold)
        cfg["curl_coarsen"] = float(curl_coarsen)
    else:
        cfg = base_config(n, omega=omega, gravity=(0.0, 0.0, -g))
    cfg["bulk_factor"] = float(bulk_factor)
    return {
        "name": "amr_d%d_%s" % (d_p, "refined" if refined else "uniform"),
        "config": cfg,
        "spheres": [sphere(centre, 0.5 * d_p, density_ratio=density_ratio, cv=0.0, fixed=False)],
        "finest": n,
        "t_g": d_p / U_G,
    }
