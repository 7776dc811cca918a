"""CPU oracle for the coupled LBM hot path -- TEST INFRASTRUCTURE ONLY.

A plain FP64 C++ implementation (``oracle.cpp``, ``refine.cpp``) reached
through ctypes.  Only ``tests/``, the smoke check and the benchmark's
CPU-baseline leg import this package; the GPU library never does, and the two
share no code.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["oracle.cpp", "refine.cpp"]
_lib = None


def build(verbose=False):
    """Compile the oracle with g++ (FP64, no FMA contraction, OpenMP)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES if os.path.exists(os.path.join(_HERE, s))]
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
           "-Wall", "-o", _LIB_PATH + ".tmp"] + srcs
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class Config(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("periodic", ctypes.c_int * 3),
                ("wall_velocity", (ctypes.c_double * 3) * 2), ("omega", ctypes.c_double),
                ("magic", ctypes.c_double), ("body_force", ctypes.c_double * 3),
                ("gravity", ctypes.c_double * 3), ("bulk_factor", ctypes.c_double)]


class Sphere(ctypes.Structure):
    _fields_ = [("x", ctypes.c_double * 3), ("u", ctypes.c_double * 3), ("w", ctypes.c_double * 3),
                ("radius", ctypes.c_double), ("density_ratio", ctypes.c_double),
                ("cv", ctypes.c_double), ("cv_omega", ctypes.c_double), ("fixed", ctypes.c_int),
                ("vm_scheme", ctypes.c_int)]


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        L.ora_create.restype = ctypes.c_void_p
        L.ora_create.argtypes = [ctypes.POINTER(Config)]
        vp = ctypes.c_void_p
        for name, args in [
            ("ora_add_sphere", [vp, ctypes.POINTER(Sphere)]),
            ("ora_set_sphere_motion", [vp, ctypes.c_int, vp, vp, ctypes.c_int]),
            ("ora_init", [vp, ctypes.c_double, ctypes.c_void_p]),
            ("ora_init_fields", [vp, ctypes.c_void_p, ctypes.c_void_p]),
            ("ora_step", [vp, ctypes.c_int]),
            ("ora_refill_cell", [vp, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_void_p]),
            ("ora_post_collision", [vp, ctypes.c_void_p]),
            ("ora_pre_collision", [vp, ctypes.c_void_p]),
            ("ora_owner", [vp, ctypes.c_void_p]),
            ("ora_force_torque", [vp, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
            ("ora_particle", [vp, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
            ("ora_fields", [vp, ctypes.c_void_p, ctypes.c_void_p]),
            ("ora_totals", [vp, ctypes.c_void_p, ctypes.c_void_p]),
            ("ora_steps_done", [vp]),
            ("ora_drag_gradient", [ctypes.POINTER(Config), ctypes.POINTER(Sphere), ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]),
            ("ora_drag_value", [ctypes.POINTER(Config), ctypes.POINTER(Sphere), ctypes.c_int,
                                ctypes.c_int, ctypes.c_int, ctypes.c_void_p]),
            ("ora_vm_trajectory", [ctypes.POINTER(Sphere), ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
            ("ora_num_threads", []),
        ]:
            fn = getattr(L, name)
            fn.restype = ctypes.c_int
            fn.argtypes = args
        L.ora_destroy.restype = None
        L.ora_destroy.argtypes = [vp]
        L.ora_link_delta.restype = ctypes.c_double
        L.ora_link_delta.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double]
        L.ora_collide_cell.restype = None
        L.ora_collide_cell.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_void_p, ctypes.c_void_p]
        L.ora_equilibrium.restype = None
        L.ora_equilibrium.argtypes = [ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]
        L.ora_collide_cell_mrt.restype = None
        L.ora_collide_cell_mrt.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_void_p, ctypes.c_void_p]
        L.ora_mrt_basis.restype = None
        L.ora_mrt_basis.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        L.ora_refill_populations.restype = None
        L.ora_refill_populations.argtypes = [ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                             ctypes.c_void_p]
        L.ora_lattice.restype = None
        L.ora_lattice.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        if hasattr(L, "orf_create"):
            _bind_refine(L)
        _lib = L
    return _lib


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle call {what} failed with {rc}")


def make_config(cfg):
    c = Config()
    for a in range(3):
        c.n[a] = int(cfg["n"][a])
        c.periodic[a] = int(cfg["periodic"][a])
        c.body_force[a] = float(cfg["body_force"][a])
        c.gravity[a] = float(cfg["gravity"][a])
        for s in range(2):
            c.wall_velocity[s][a] = float(cfg["wall_velocity"][s][a])
    c.omega = float(cfg["omega"])
    c.magic = float(cfg["magic"])
    c.bulk_factor = float(cfg.get("bulk_factor", 1.0))
    return c


def make_sphere(s):
    o = Sphere()
    for a in range(3):
        o.x[a] = s["x"][a]
        o.u[a] = s["u"][a]
        o.w[a] = s["w"][a]
    o.radius = s["radius"]
    o.density_ratio = s["density_ratio"]
    o.cv = s["cv"]
    o.cv_omega = s["cv_omega"]
    o.fixed = int(s["fixed"])
    o.vm_scheme = int(s.get("vm_scheme", 0))
    return o


def lattice():
    c = np.zeros((19, 3), dtype=np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, dtype=np.int32)
    lib().ora_lattice(c.ctypes.data, w.ctypes.data, opp.ctypes.data)
    return c, w, opp


def collide_cell(f, omega, magic, F):
    f = np.ascontiguousarray(f, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    out = np.zeros(19)
    lib().ora_collide_cell(f.ctypes.data, omega, magic, F.ctypes.data, out.ctypes.data)
    return out


def equilibrium(rho, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(19)
    lib().ora_equilibrium(float(rho), u.ctypes.data, out.ctypes.data)
    return out


def refill_populations(rho, v, S, omega):
    v = np.ascontiguousarray(v, dtype=np.float64)
    S = np.ascontiguousarray(S, dtype=np.float64).reshape(9)
    out = np.zeros(19)
    lib().ora_refill_populations(float(rho), v.ctypes.data, S.ctypes.data, float(omega), out.ctypes.data)
    return out


def collide_cell_mrt(f, omega, magic, bulk_factor, F):
    f = np.ascontiguousarray(f, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.float64)
    out = np.zeros(19)
    lib().ora_collide_cell_mrt(f.ctypes.data, float(omega), float(magic), float(bulk_factor), F.ctypes.data,
                               out.ctypes.data)
    return out


def mrt_basis():
    e = np.zeros((19, 19))
    norm = np.zeros(19)
    lib().ora_mrt_basis(e.ctypes.data, norm.ctypes.data)
    return e, norm


def link_delta(d, c, radius):
    d = np.ascontiguousarray(d, dtype=np.float64)
    c = np.ascontiguousarray(c, dtype=np.int32)
    return lib().ora_link_delta(d.ctypes.data, c.ctypes.data, float(radius))


def vm_trajectory(sph, F, T, g, nsteps, dF=(0.0, 0.0, 0.0)):
    """Particle update alone: raw force F + k dF at update k, torque T;
    [nsteps][15] = x, u, w, a, beta after each update."""
    s = make_sphere(sph)
    F = np.ascontiguousarray(F, dtype=np.float64)
    dF = np.ascontiguousarray(dF, dtype=np.float64)
    T = np.ascontiguousarray(T, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    out = np.zeros((nsteps, 15))
    _check(lib().ora_vm_trajectory(ctypes.byref(s), F.ctypes.data, dF.ctypes.data, T.ctypes.data, g.ctypes.data,
                                   nsteps, out.ctypes.data), "vm_trajectory")
    return out


class Uniform:
    """Uniform-grid oracle: one periodic/walled box with spheres."""

    def __init__(self, cfg, spheres=()):
        self.cfg = cfg
        self._c = make_config(cfg)
        self.h = lib().ora_create(ctypes.byref(self._c))
        if not self.h:
            raise RuntimeError("ora_create failed")
        self.n = tuple(cfg["n"])
        self.N = self.n[0] * self.n[1] * self.n[2]
        for s in spheres:
            o = make_sphere(s)
            if lib().ora_add_sphere(self.h, ctypes.byref(o)) < 0:
                raise RuntimeError("ora_add_sphere failed")
        self.nsph = len(spheres)

    def __del__(self):
        if getattr(self, "h", None):
            lib().ora_destroy(self.h)
            self.h = None

    def init(self, rho=1.0, u0=None):
        """Equilibrium start; rho a number or a per-cell [nz][ny][nx] field."""
        if u0 is not None:
            u0 = np.ascontiguousarray(u0, dtype=np.float64)
            assert u0.size == 3 * self.N
        up = u0.ctypes.data if u0 is not None else None
        if np.ndim(rho) > 0:
            r = np.ascontiguousarray(rho, dtype=np.float64)
            assert r.size == self.N
            _check(lib().ora_init_fields(self.h, r.ctypes.data, up), "init")
        else:
            _check(lib().ora_init(self.h, float(rho), up), "init")

    def step(self, n=1):
        _check(lib().ora_step(self.h, int(n)), "step")

    def refill_cell(self, f_pre, old_owner, cell, pid):
        """Refill of cell (x, y, z) uncovered by sphere pid, computed on the
        pre-collision state f_pre [19][nz][ny][nx] with the mapping before
        the re-mapping old_owner [nz][ny][nx] (-1 fluid); replaces the
        oracle's state by f_pre.  Returns the cell's 19 populations."""
        f = np.ascontiguousarray(f_pre, dtype=np.float64)
        o = np.ascontiguousarray(old_owner, dtype=np.int32)
        assert f.size == 19 * self.N and o.size == self.N
        out = np.zeros(19)
        x, y, z = (int(v) for v in cell)
        _check(lib().ora_refill_cell(self.h, f.ctypes.data, o.ctypes.data, x, y, z, int(pid), out.ctypes.data),
               "refill_cell")
        return out

    def _shape(self):
        nx, ny, nz = self.n
        return (19, nz, ny, nx)

    def post_collision(self):
        out = np.zeros(self._shape())
        _check(lib().ora_post_collision(self.h, out.ctypes.data), "post_collision")
        return out

    def pre_collision(self):
        out = np.zeros(self._shape())
        _check(lib().ora_pre_collision(self.h, out.ctypes.data), "pre_collision")
        return out

    def owner(self):
        nx, ny, nz = self.n
        out = np.zeros((nz, ny, nx), dtype=np.int32)
        _check(lib().ora_owner(self.h, out.ctypes.data), "owner")
        return out

    def force_torque(self, i=0):
        F = np.zeros(3)
        T = np.zeros(3)
        _check(lib().ora_force_torque(self.h, i, F.ctypes.data, T.ctypes.data), "force_torque")
        return F, T

    def particle(self, i=0):
        x, u, w = np.zeros(3), np.zeros(3), np.zeros(3)
        _check(lib().ora_particle(self.h, i, x.ctypes.data, u.ctypes.data, w.ctypes.data), "particle")
        return x, u, w

    def set_sphere_motion(self, i, u=(0.0, 0.0, 0.0), w=(0.0, 0.0, 0.0), fixed=0):
        """New velocities and hold mode (0 free, 1 held, 2 rotation only)."""
        u = np.ascontiguousarray(u, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        _check(lib().ora_set_sphere_motion(self.h, i, u.ctypes.data, w.ctypes.data, int(fixed)), "set_sphere_motion")

    def fields(self):
        nx, ny, nz = self.n
        rho = np.zeros((nz, ny, nx))
        u = np.zeros((3, nz, ny, nx))
        _check(lib().ora_fields(self.h, rho.ctypes.data, u.ctypes.data), "fields")
        return rho, u

    def totals(self):
        m = np.zeros(1)
        j = np.zeros(3)
        _check(lib().ora_totals(self.h, m.ctypes.data, j.ctypes.data), "totals")
        return float(m[0]), j


def drag_gradient(cfg, spheres, n_steps, avg_from):
    c = make_config(cfg)
    arr = (Sphere * len(spheres))(*[make_sphere(s) for s in spheres])
    J = np.zeros(1)
    g = np.zeros(2)
    _check(lib().ora_drag_gradient(ctypes.byref(c), arr, len(spheres), n_steps, avg_from,
                                   J.ctypes.data, g.ctypes.data), "drag_gradient")
    return float(J[0]), g


def drag_value(cfg, spheres, n_steps, avg_from):
    c = make_config(cfg)
    arr = (Sphere * len(spheres))(*[make_sphere(s) for s in spheres])
    J = np.zeros(1)
    _check(lib().ora_drag_value(ctypes.byref(c), arr, len(spheres), n_steps, avg_from,
                                J.ctypes.data), "drag_value")
    return float(J[0])


def num_threads():
    return lib().ora_num_threads()


class RConfig(ctypes.Structure):
    _fields_ = [("n0", ctypes.c_int * 3), ("block", ctypes.c_int), ("levels", ctypes.c_int),
                ("omega", ctypes.c_double), ("magic", ctypes.c_double), ("body_force", ctypes.c_double * 3),
                ("gravity", ctypes.c_double * 3), ("check_every", ctypes.c_int),
                ("bulk_factor", ctypes.c_double), ("curl_threshold", ctypes.c_double),
                ("curl_coarsen", ctypes.c_double)]


def _bind_refine(L):
    vp = ctypes.c_void_p
    L.orf_create.restype = vp
    L.orf_create.argtypes = [ctypes.POINTER(RConfig)]
    L.orf_destroy.restype = None
    L.orf_destroy.argtypes = [vp]
    for name, args in [
        ("orf_add_region", [vp, vp, vp, ctypes.c_int]),
        ("orf_add_sphere", [vp, ctypes.POINTER(Sphere)]),
        ("orf_set_sphere_motion", [vp, ctypes.c_int, vp, vp, ctypes.c_int]),
        ("orf_init", [vp, ctypes.c_double, vp]),
        ("orf_set_level_velocity", [vp, ctypes.c_int, ctypes.c_double, vp]),
        ("orf_step", [vp, ctypes.c_int]),
        ("orf_level_dims", [vp, ctypes.c_int, vp]),
        ("orf_block_grid", [vp, vp]),
        ("orf_leaf", [vp, vp]),
        ("orf_read_level", [vp, ctypes.c_int, vp, vp]),
        ("orf_mass", [vp, vp]),
        ("orf_force_torque", [vp, ctypes.c_int, vp, vp]),
        ("orf_particle", [vp, ctypes.c_int, vp, vp, vp]),
        ("orf_owner", [vp, vp]),
        ("orf_counters", [vp, vp, vp, vp]),
        ("orf_block_sensor", [vp, ctypes.c_int, vp]),
    ]:
        fn = getattr(L, name)
        fn.restype = ctypes.c_int
        fn.argtypes = args


class Refined:
    """Refined-grid oracle: periodic block-structured 2:1 grid.

    cfg: synth config with "levels" and "block"; n is the coarsest grid.
    regions: list of (lo, hi, level) coarse-cell boxes to hold at >= level.
    """

    def __init__(self, cfg, spheres=(), regions=(), check_every=0):
        c = RConfig()
        for a in range(3):
            c.n0[a] = int(cfg["n"][a])
            c.body_force[a] = float(cfg["body_force"][a])
            c.gravity[a] = float(cfg["gravity"][a])
        c.block = int(cfg["block"])
        c.levels = int(cfg["levels"])
        c.omega = float(cfg["omega"])
        c.magic = float(cfg["magic"])
        c.check_every = int(check_every)
        c.bulk_factor = float(cfg.get("bulk_factor", 1.0))
        c.curl_threshold = float(cfg.get("curl_threshold", 0.0))
        c.curl_coarsen = float(cfg.get("curl_coarsen", 0.2))
        self._c = c
        self.h = lib().orf_create(ctypes.byref(c))
        if not self.h:
            raise RuntimeError("orf_create failed")
        self.levels = c.levels
        for lo, hi, lev in regions:
            lo = np.ascontiguousarray(lo, dtype=np.int32)
            hi = np.ascontiguousarray(hi, dtype=np.int32)
            _check(lib().orf_add_region(self.h, lo.ctypes.data, hi.ctypes.data, int(lev)), "add_region")
        for s in spheres:
            o = make_sphere(s)
            if lib().orf_add_sphere(self.h, ctypes.byref(o)) < 0:
                raise RuntimeError("orf_add_sphere failed")

    def __del__(self):
        if getattr(self, "h", None):
            lib().orf_destroy(self.h)
            self.h = None

    def init(self, rho=1.0, u0=None):
        if u0 is not None:
            u0 = np.ascontiguousarray(u0, dtype=np.float64)
            _check(lib().orf_init(self.h, float(rho), u0.ctypes.data), "init")
        else:
            _check(lib().orf_init(self.h, float(rho), None), "init")

    def set_level_velocity(self, level, rho, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        _check(lib().orf_set_level_velocity(self.h, level, float(rho), u.ctypes.data), "set_level_velocity")

    def step(self, n=1):
        _check(lib().orf_step(self.h, int(n)), "step")

    def dims(self, level):
        n = np.zeros(3, dtype=np.int32)
        _check(lib().orf_level_dims(self.h, level, n.ctypes.data), "level_dims")
        return tuple(int(v) for v in n)

    def block_grid(self):
        n = np.zeros(3, dtype=np.int32)
        _check(lib().orf_block_grid(self.h, n.ctypes.data), "block_grid")
        return tuple(int(v) for v in n)

    def leaf(self):
        nx, ny, nz = self.block_grid()
        out = np.zeros((nz, ny, nx), dtype=np.int32)
        _check(lib().orf_leaf(self.h, out.ctypes.data), "leaf")
        return out

    def level(self, level):
        nx, ny, nz = self.dims(level)
        f = np.zeros((19, nz, ny, nx))
        k = np.zeros((nz, ny, nx), dtype=np.uint8)
        _check(lib().orf_read_level(self.h, level, f.ctypes.data, k.ctypes.data), "read_level")
        return f, k

    def mass(self):
        m = np.zeros(1)
        _check(lib().orf_mass(self.h, m.ctypes.data), "mass")
        return float(m[0])

    def force_torque(self, i=0):
        F, T = np.zeros(3), np.zeros(3)
        _check(lib().orf_force_torque(self.h, i, F.ctypes.data, T.ctypes.data), "force_torque")
        return F, T

    def particle(self, i=0):
        x, u, w = np.zeros(3), np.zeros(3), np.zeros(3)
        _check(lib().orf_particle(self.h, i, x.ctypes.data, u.ctypes.data, w.ctypes.data), "particle")
        return x, u, w

    def set_sphere_motion(self, i, u=(0.0, 0.0, 0.0), w=(0.0, 0.0, 0.0), fixed=0):
        u = np.ascontiguousarray(u, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        _check(lib().orf_set_sphere_motion(self.h, i, u.ctypes.data, w.ctypes.data, int(fixed)), "set_sphere_motion")

    def owner(self):
        nx, ny, nz = self.dims(self.levels - 1)
        out = np.zeros((nz, ny, nx), dtype=np.int32)
        _check(lib().orf_owner(self.h, out.ctypes.data), "owner")
        return out

    def block_sensor(self, level):
        """Curl sensor (Eq. 23) per block of the level: [bnz][bny][bnx], -1
        where the block is not a leaf of that level."""
        nx, ny, nz = self.dims(level)
        b = self._c.block
        out = np.zeros((nz // b, ny // b, nx // b))
        _check(lib().orf_block_sensor(self.h, int(level), out.ctypes.data), "block_sensor")
        return out

    def counters(self):
        a, b = ctypes.c_longlong(), ctypes.c_longlong()
        r = ctypes.c_int()
        _check(lib().orf_counters(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(r)), "counters")
        return a.value, b.value, r.value
