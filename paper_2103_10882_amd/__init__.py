"""Python binding of libvmlbm (gfx950 HIP library of the coupled LBM hot path).

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch supplies the device workspace (a uint8 tensor) and the stream.
The library must have been built (``paper_2103_10882_amd.build.build()``);
there is no fallback path.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvmlbm.so")

F64, F32, F16 = 0, 1, 2
STORAGE = {"f64": F64, "f32": F32, "f16": F16}
BYTES = {F64: 8, F32: 4, F16: 2}

ERRORS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ESTATE", -5: "EUNSTABLE", -6: "ERANGE"}

EXPORTS = [
    "vmlbm_create", "vmlbm_add_sphere", "vmlbm_add_refine_region", "vmlbm_required_bytes", "vmlbm_bind_workspace",
    "vmlbm_set_stream", "vmlbm_init_equilibrium", "vmlbm_step", "vmlbm_sync", "vmlbm_get_particle",
    "vmlbm_set_sphere_motion",
    "vmlbm_get_force_torque", "vmlbm_get_history", "vmlbm_read_populations",
    "vmlbm_write_populations", "vmlbm_read_owner", "vmlbm_read_fields", "vmlbm_stats",
    "vmlbm_profile", "vmlbm_sweep_time", "vmlbm_totals", "vmlbm_read_box", "vmlbm_cell_counts", "vmlbm_level_blocks",
    "vmlbm_refinements", "vmlbm_prebuilt_layouts", "vmlbm_level_pull",
    "vmlbm_set_params", "vmlbm_forward_ckpt", "vmlbm_adjoint", "vmlbm_destroy", "vmlbm_last_error",
    "vmlbm_stream_copy", "vmlbm_stream_pull", "vmlbm_totals_static",
]


class VmlbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int * 3), ("block", ctypes.c_int), ("levels", ctypes.c_int),
                ("periodic", ctypes.c_int * 3), ("wall_velocity", (ctypes.c_double * 3) * 2),
                ("omega", ctypes.c_double), ("magic", ctypes.c_double),
                ("body_force", ctypes.c_double * 3), ("gravity", ctypes.c_double * 3),
                ("storage", ctypes.c_int), ("check_every", ctypes.c_int), ("history", ctypes.c_int),
                ("adjoint_steps", ctypes.c_int), ("ckpt_every", ctypes.c_int),
                ("bulk_factor", ctypes.c_double), ("curl_threshold", ctypes.c_double),
                ("curl_coarsen", ctypes.c_double), ("max_blocks", ctypes.c_int)]


class Sphere(ctypes.Structure):
    _fields_ = [("x", ctypes.c_double * 3), ("u", ctypes.c_double * 3), ("w", ctypes.c_double * 3),
                ("radius", ctypes.c_double), ("density_ratio", ctypes.c_double),
                ("cv", ctypes.c_double), ("cv_omega", ctypes.c_double), ("fixed", ctypes.c_int),
                ("vm_scheme", ctypes.c_int)]


_lib = None


def lib():
    """Load libvmlbm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2103_10882_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        sig = {
            "vmlbm_create": [ctypes.POINTER(Config), ctypes.POINTER(vp)],
            "vmlbm_add_sphere": [vp, ctypes.POINTER(Sphere), ctypes.POINTER(ctypes.c_int)],
            "vmlbm_add_refine_region": [vp, vp, vp, ctypes.c_int],
            "vmlbm_required_bytes": [vp, ctypes.POINTER(ctypes.c_size_t)],
            "vmlbm_bind_workspace": [vp, vp, ctypes.c_size_t],
            "vmlbm_set_stream": [vp, vp],
            "vmlbm_init_equilibrium": [vp, ctypes.c_double, vp],
            "vmlbm_step": [vp, ctypes.c_int],
            "vmlbm_sync": [vp],
            "vmlbm_get_particle": [vp, ctypes.c_int, vp, vp, vp],
            "vmlbm_set_sphere_motion": [vp, ctypes.c_int, vp, vp, ctypes.c_int],
            "vmlbm_get_force_torque": [vp, ctypes.c_int, vp, vp],
            "vmlbm_get_history": [vp, ctypes.c_int, ctypes.c_int, vp],
            "vmlbm_read_populations": [vp, ctypes.c_int, vp],
            "vmlbm_write_populations": [vp, ctypes.c_int, vp],
            "vmlbm_read_owner": [vp, ctypes.c_int, vp],
            "vmlbm_read_fields": [vp, ctypes.c_int, vp, vp],
            "vmlbm_stats": [vp, vp, vp],
            "vmlbm_profile": [vp, ctypes.c_int],
            "vmlbm_sweep_time": [vp, vp, vp],
            "vmlbm_cell_counts": [vp, ctypes.c_int, vp, vp],
            "vmlbm_totals": [vp, vp, vp],
            "vmlbm_totals_static": [vp, vp, vp],
            "vmlbm_read_box": [vp, vp, vp, vp],
            "vmlbm_level_blocks": [vp, ctypes.c_int, vp, vp],
            "vmlbm_refinements": [vp, vp],
            "vmlbm_prebuilt_layouts": [vp, vp],
            "vmlbm_level_pull": [vp, ctypes.c_int, ctypes.c_int],
            "vmlbm_set_params": [vp, ctypes.c_double, ctypes.c_double],
            "vmlbm_forward_ckpt": [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp],
            "vmlbm_adjoint": [vp, ctypes.c_double, vp],
            "vmlbm_destroy": [vp],
            "vmlbm_stream_copy": [vp, vp, ctypes.c_size_t, vp],
            "vmlbm_stream_pull": [vp, vp, ctypes.c_int, vp, vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        L.vmlbm_last_error.argtypes = [vp]
        L.vmlbm_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def make_config(cfg, storage="f64", history=4, adjoint_steps=0, ckpt_every=0, check_every=4):
    c = Config()
    for a in range(3):
        c.n[a] = int(cfg["n"][a])
        c.periodic[a] = int(cfg["periodic"][a])
        c.body_force[a] = float(cfg["body_force"][a])
        c.gravity[a] = float(cfg["gravity"][a])
        for s in range(2):
            c.wall_velocity[s][a] = float(cfg["wall_velocity"][s][a])
    c.block = int(cfg.get("block", 0))
    c.levels = int(cfg.get("levels", 1))
    c.omega = float(cfg["omega"])
    c.magic = float(cfg["magic"])
    c.bulk_factor = float(cfg.get("bulk_factor", 1.0))
    c.curl_threshold = float(cfg.get("curl_threshold", 0.0))
    c.curl_coarsen = float(cfg.get("curl_coarsen", 0.2))
    c.max_blocks = int(cfg.get("max_blocks", 0))
    c.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    c.check_every = int(cfg.get("check_every", check_every))
    c.history = int(history)
    c.adjoint_steps = int(adjoint_steps)
    c.ckpt_every = int(ckpt_every)
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


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


class Sim:
    """One simulation context on the current CUDA (HIP) device."""

    def __init__(self, cfg, spheres=(), storage="f64", history=4, adjoint_steps=0, ckpt_every=0,
                 device="cuda", regions=(), check_every=None):
        import torch
        self.L = lib()
        self.cfg = cfg
        self._c = make_config(cfg, storage, history, adjoint_steps, ckpt_every)
        if check_every is not None:
            self._c.check_every = int(check_every)
        self.h = ctypes.c_void_p()
        self._check(self.L.vmlbm_create(ctypes.byref(self._c), ctypes.byref(self.h)), "create")
        for s in spheres:
            o = make_sphere(s)
            i = ctypes.c_int()
            self._check(self.L.vmlbm_add_sphere(self.h, ctypes.byref(o), ctypes.byref(i)), "add_sphere")
        self.nsph = len(spheres)
        for lo, hi, lev in regions:
            lo = np.ascontiguousarray(lo, dtype=np.int32)
            hi = np.ascontiguousarray(hi, dtype=np.int32)
            self._check(self.L.vmlbm_add_refine_region(self.h, _ptr(lo), _ptr(hi), int(lev)), "add_refine_region")
        nb = ctypes.c_size_t()
        self._check(self.L.vmlbm_required_bytes(self.h, ctypes.byref(nb)), "required_bytes")
        self.ws_bytes = nb.value
        self.ws = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=device)
        base = self.ws.data_ptr()
        aligned = (base + 255) & ~255
        self._check(self.L.vmlbm_bind_workspace(self.h, ctypes.c_void_p(aligned), self.ws_bytes), "bind")
        self.stream = torch.cuda.current_stream(self.ws.device)
        self._check(self.L.vmlbm_set_stream(self.h, ctypes.c_void_p(self.stream.cuda_stream)), "set_stream")
        self.block = int(cfg.get("block", 0))
        self.n = tuple(int(v) for v in cfg["n"])

    def _check(self, rc, what):
        if rc != 0:
            msg = self.L.vmlbm_last_error(self.h) if self.h else b""
            raise VmlbmError(rc, f"{what}: {msg.decode() if msg else ''}")

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            self.L.vmlbm_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- stepping -----------------------------------------------------------
    def init(self, rho=1.0, u0=None):
        if u0 is not None:
            u0 = np.ascontiguousarray(u0, dtype=np.float64)
            self._check(self.L.vmlbm_init_equilibrium(self.h, float(rho), _ptr(u0)), "init")
        else:
            self._check(self.L.vmlbm_init_equilibrium(self.h, float(rho), None), "init")

    def step(self, n=1):
        self._check(self.L.vmlbm_step(self.h, int(n)), "step")

    def sync(self):
        self._check(self.L.vmlbm_sync(self.h), "sync")

    # --- read-back ----------------------------------------------------------
    def cells(self, level=0):
        if self.block:
            return self.level_blocks(level).shape[0] * self.block ** 3
        return self.n[0] * self.n[1] * self.n[2]

    def _shape(self, level):
        if self.block:
            return (19, self.cells(level))
        nx, ny, nz = self.n
        return (19, nz, ny, nx)

    def populations(self, level=0):
        out = np.zeros(self._shape(level))
        self._check(self.L.vmlbm_read_populations(self.h, level, _ptr(out)), "read_populations")
        return out

    def write_populations(self, f, level=0):
        f = np.ascontiguousarray(f, dtype=np.float64)
        self._check(self.L.vmlbm_write_populations(self.h, level, _ptr(f)), "write_populations")

    def owner(self, level=0):
        shp = self._shape(level)[1:]
        out = np.zeros(shp, dtype=np.int32)
        self._check(self.L.vmlbm_read_owner(self.h, level, _ptr(out)), "read_owner")
        return out

    def fields(self, level=0):
        shp = self._shape(level)[1:]
        rho = np.zeros(shp)
        u = np.zeros((3,) + shp)
        self._check(self.L.vmlbm_read_fields(self.h, level, _ptr(rho), _ptr(u)), "read_fields")
        return rho, u

    def force_torque(self, i=0):
        F, T = np.zeros(3), np.zeros(3)
        self._check(self.L.vmlbm_get_force_torque(self.h, i, _ptr(F), _ptr(T)), "force_torque")
        return F, T

    def particle(self, i=0):
        x, u, w = np.zeros(3), np.zeros(3), np.zeros(3)
        self._check(self.L.vmlbm_get_particle(self.h, i, _ptr(x), _ptr(u), _ptr(w)), "particle")
        return x, u, w

    def set_sphere_motion(self, i, u=(0.0, 0.0, 0.0), w=(0.0, 0.0, 0.0), fixed=0):
        """Hold mode of sphere i from the next step on (0 free, 1 held, 2
        position held with free rotation) and its new velocities."""
        u = np.ascontiguousarray(u, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        self._check(self.L.vmlbm_set_sphere_motion(self.h, i, _ptr(u), _ptr(w), int(fixed)), "set_sphere_motion")

    def history(self, i, n):
        """[n][15]: F, T, x, u, w after each of the last n steps."""
        out = np.zeros((n, 15))
        self._check(self.L.vmlbm_get_history(self.h, i, n, _ptr(out)), "history")
        return out

    def stats(self):
        cu, sec = ctypes.c_double(), ctypes.c_double()
        self._check(self.L.vmlbm_stats(self.h, ctypes.byref(cu), ctypes.byref(sec)), "stats")
        return cu.value, sec.value

    def profile(self, enable=True):
        self._check(self.L.vmlbm_profile(self.h, int(enable)), "profile")

    def sweep_time(self):
        s, n = ctypes.c_double(), ctypes.c_longlong()
        self._check(self.L.vmlbm_sweep_time(self.h, ctypes.byref(s), ctypes.byref(n)), "sweep_time")
        return s.value, n.value

    def totals_static(self):
        """totals() through the entry point that allocates nothing."""
        m = np.zeros(1)
        j = np.zeros(3)
        self._check(self.L.vmlbm_totals_static(self.h, _ptr(m), _ptr(j)), "totals_static")
        return float(m[0]), j

    def totals(self):
        m = np.zeros(1)
        j = np.zeros(3)
        self._check(self.L.vmlbm_totals(self.h, _ptr(m), _ptr(j)), "totals")
        return float(m[0]), j

    def read_box(self, lo, size):
        lo = np.ascontiguousarray(lo, dtype=np.int32)
        size = np.ascontiguousarray(size, dtype=np.int32)
        out = np.zeros((19, int(size[2]), int(size[1]), int(size[0])))
        self._check(self.L.vmlbm_read_box(self.h, _ptr(lo), _ptr(size), _ptr(out)), "read_box")
        return out

    def cell_counts(self, level=0):
        f, i = ctypes.c_longlong(), ctypes.c_longlong()
        self._check(self.L.vmlbm_cell_counts(self.h, level, ctypes.byref(f), ctypes.byref(i)), "cell_counts")
        return f.value, i.value

    def level_blocks(self, level):
        cnt = ctypes.c_int()
        self._check(self.L.vmlbm_level_blocks(self.h, level, ctypes.byref(cnt), None), "level_blocks")
        org = np.zeros((cnt.value, 3), dtype=np.int32)
        self._check(self.L.vmlbm_level_blocks(self.h, level, ctypes.byref(cnt), _ptr(org)), "level_blocks")
        return org

    def refinements(self):
        c = ctypes.c_int()
        self._check(self.L.vmlbm_refinements(self.h, ctypes.byref(c)), "refinements")
        return c.value

    def prebuilt_layouts(self):
        c = ctypes.c_int()
        self._check(self.L.vmlbm_prebuilt_layouts(self.h, ctypes.byref(c)), "prebuilt_layouts")
        return c.value

    def level_pull(self, level, reps=1):
        """Block-structured grid: the level sweep's access pattern without
        arithmetic (a bandwidth reference), `reps` times on the context's
        stream; each pulled state becomes the level's current state."""
        self._check(self.L.vmlbm_level_pull(self.h, int(level), int(reps)), "level_pull")

    # --- differentiation ------------------------------------------------------
    def set_params(self, body_force_z, omega):
        self._check(self.L.vmlbm_set_params(self.h, float(body_force_z), float(omega)), "set_params")
        self._params = (float(body_force_z), float(omega))
        self._adj_run = None

    def forward_ckpt(self, sphere, n_steps, avg_from, ckpt_every):
        J = np.zeros(1)
        self._adj_run = None
        self._check(self.L.vmlbm_forward_ckpt(self.h, sphere, n_steps, avg_from, ckpt_every, _ptr(J)),
                    "forward_ckpt")
        params = getattr(self, "_params", None)
        if params is not None:
            self._adj_run = params + (sphere, n_steps, avg_from)
        return float(J[0])

    def adjoint_run(self):
        """(F_z, omega, sphere, n_steps, avg_from) of the forward run whose
        checkpoints the simulation holds, or None."""
        return getattr(self, "_adj_run", None)

    def adjoint(self, dJ=1.0):
        g = np.zeros(2)
        self._check(self.L.vmlbm_adjoint(self.h, float(dJ), _ptr(g)), "adjoint")
        return g


def _drag_grad_function():
    import torch

    class DragGrad(torch.autograd.Function):
        """J(F_z, omega): time-averaged z-drag of a fixed sphere after a
        forward run from rest; backward runs the library's discrete adjoint
        with checkpoint recomputation."""

        @staticmethod
        def forward(ctx, force_z, omega, sim, sphere, n_steps, avg_from, ckpt_every):
            sim.set_params(float(force_z), float(omega))
            J = sim.forward_ckpt(sphere, n_steps, avg_from, ckpt_every)
            ctx.sim = sim
            ctx.run = (float(force_z), float(omega), sphere, n_steps, avg_from, ckpt_every)
            return torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gJ):
            # the simulation's checkpoints belong to its last forward run;
            # another drag() on the same sim since this one replaced them,
            # so this run's trajectory is recomputed first
            F, om, sphere, n_steps, avg_from, ckpt_every = ctx.run
            if ctx.sim.adjoint_run() != (F, om, sphere, n_steps, avg_from):
                ctx.sim.set_params(F, om)
                ctx.sim.forward_ckpt(sphere, n_steps, avg_from, ckpt_every)
            g = ctx.sim.adjoint(float(gJ))
            return (torch.tensor(g[0], dtype=torch.float64), torch.tensor(g[1], dtype=torch.float64),
                    None, None, None, None, None)

    return DragGrad


def drag(force_z, omega, sim, sphere=0, n_steps=2000, avg_from=1500, ckpt_every=50):
    """Differentiable time-averaged drag (torch scalars in, torch scalar out)."""
    return _drag_grad_function().apply(force_z, omega, sim, sphere, n_steps, avg_from, ckpt_every)


def stream_copy(dst, src):
    """Plain device copy src -> dst (torch tensors of equal byte size, a
    multiple of 16) on torch's current stream: the bandwidth reference."""
    import torch
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes
    rc = lib().vmlbm_stream_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != 0:
        raise VmlbmError(rc, "stream_copy")


def stream_pull(dst, src, n, storage):
    """The interior sweep's access pattern without arithmetic on a periodic
    n = (nx, ny, nz) box: dst[q][x] = src[q][x - c_q] (torch tensors of 19
    nx ny nz elements of the storage format, in its population layout:
    [z][q][y][x] for f16, [q][z][y][x] otherwise) on torch's current
    stream."""
    import torch
    code = {"f64": 0, "f32": 1, "f16": 2}[storage]
    cells = 19 * n[0] * n[1] * n[2]
    assert src.numel() == cells and dst.numel() == cells
    assert src.element_size() == dst.element_size() == (8, 4, 2)[code]
    nn = (ctypes.c_int * 3)(*n)
    rc = lib().vmlbm_stream_pull(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), code, nn,
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != 0:
        raise VmlbmError(rc, "stream_pull")
