"""Checks at the full workload sizes, in the launch configuration the
benchmark times: sampled cells against the oracle's collision, and
properties that hold at any size (fluid momentum balance of the momentum
exchange, exact rest state on the full refined layout)."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    import oracle
    import paper_2103_10882_amd as pkg
    assert torch.cuda.is_available()
    pkg.lib()
    oracle.lib()
    return pkg, oracle


def far_box(n, spheres, size, rng, margin=3):
    """Origin of a box whose cells (plus one layer) are far from every sphere."""
    for _ in range(1000):
        lo = rng.integers(0, n, 3)
        ok = True
        c = lo + size / 2.0
        for s in spheres:
            d = c - np.array(s["x"])
            d -= n * np.round(d / n)
            if np.sqrt(d @ d) < s["radius"] + size + margin:
                ok = False
        if ok:
            return lo
    raise RuntimeError("no free box")


def sampled_step_parity(ora, pkg, cfg, sph, u0, lo, size, steps=2):
    """A fresh FP64 run from f(0) = f^eq(1, u0), `steps` steps, read back at
    the cells of a box far from spheres and walls, against the oracle
    computed from u0 alone, cell by cell.  The stored state after the start
    is the collision of f^eq(1, u0) at each cell's own velocity; each step
    pulls from the 19 upstream cells and collides again."""
    import torch
    c, _, _ = ora.lattice()
    F = np.array(cfg["body_force"])
    n = cfg["n"]
    sim = pkg.Sim(cfg, sph, storage="f64")
    sim.init(1.0, u0)
    sim.step(steps)
    new = sim.read_box(np.array(lo), np.array([size] * 3))
    sim.close()
    del sim
    torch.cuda.empty_cache()
    memo = {}

    def state(k, x, y, z):
        key = (k, x % n[0], y % n[1], z % n[2])
        if key not in memo:
            _, i, j, l = key
            if k == 0:
                f = ora.equilibrium(1.0, u0[:, l, j, i])
            else:
                f = np.array([state(k - 1, i - c[q, 0], j - c[q, 1], l - c[q, 2])[q] for q in range(19)])
            memo[key] = ora.collide_cell(f, cfg["omega"], cfg["magic"], F)
        return memo[key]

    worst = 0.0
    for k in range(size):
        for j in range(size):
            for i in range(size):
                out = state(steps, lo[0] + i, lo[1] + j, lo[2] + k)
                worst = max(worst, np.abs(new[:, k, j, i] - out).max() / np.abs(out).max())
    return worst


def test_precision512_full(env):
    """512^3, 8 fixed r=20 spheres, FP64: fluid momentum changes by N_f F
    minus the summed sphere forces every step (Eq. 11 with v = 0); sampled
    interior cells follow the oracle's collision to 1e-12."""
    import torch
    pkg, ora = env
    w = synth.precision()
    cfg, sph = w["config"], w["spheres"]
    say("case precision512 f64 full size")
    sim = pkg.Sim(cfg, sph, storage="f64")
    sim.init()
    sim.step(3)
    fluid, _ = sim.cell_counts()
    F = np.array(cfg["body_force"])
    _, j0 = sim.totals()
    for k in range(3):
        sim.step(1)
        _, j1 = sim.totals()
        Fh = sum(sim.force_torque(i)[0] for i in range(len(sph)))
        res = j1 - j0 - fluid * F + Fh
        say(f"  step {k}: momentum balance residual {np.abs(res).max():.2e} (N_f F = {fluid * F[2]:.1f})")
        assert np.abs(res).max() <= 1e-10 * fluid * np.abs(F).max()
        j0 = j1
    sim.close()
    del sim
    torch.cuda.empty_cache()
    rng = np.random.default_rng(0)
    lo = far_box(512, sph, 6, rng)
    u0 = synth.velocity_perturbation((512, 512, 512), seed=5, amplitude=0.02)
    rel = sampled_step_parity(ora, pkg, cfg, sph, u0, lo, 6)
    del u0
    say(f"  sampled cells at {lo} after two steps from a rough start: rel err {rel:.2e}")
    assert rel <= 1e-12


def test_rising256_full(env):
    """256^3 rising light sphere between walls, FP64 and FP32: sampled cells
    far from sphere and walls follow the oracle after two steps from a rough
    start; the two storage formats give the same rise."""
    import torch
    pkg, ora = env
    w = synth.rising()
    cfg, sph = w["config"], w["spheres"]
    say("case rising256 full size")
    u0 = synth.velocity_perturbation((256, 256, 256), seed=6, amplitude=0.02)
    lo = np.array([20, 200, 100])
    rel = sampled_step_parity(ora, pkg, cfg, sph, u0, lo, 6)
    del u0
    say(f"  sampled cells after two steps from a rough start: rel err {rel:.2e}")
    assert rel <= 1e-12
    traj = {}
    for st in ("f64", "f32"):
        sim = pkg.Sim(cfg, sph, storage=st, history=300)
        sim.init()
        sim.step(300)
        sim.sync()
        traj[st] = sim.history(0, 300)
        sim.close()
        del sim
        torch.cuda.empty_cache()
    uz64, uz32 = traj["f64"][:, 11], traj["f32"][:, 11]
    say(f"  u_z after 300 steps: f64 {uz64[-1]:.6e} f32 {uz32[-1]:.6e}")
    assert uz64[-1] > 0
    assert np.abs(uz32 - uz64).max() <= 1e-4 * np.abs(uz64).max()


def test_refined_full_comoving_and_rise(env):
    """Full refined layout (coarse 128x128x512, 3 levels, r=16 finest):
    (a) a heavy sphere moving with a uniform flow leaves every interior cell
    of every level at f^eq(1, U) after 20 coarse steps (explosion,
    coalescence weights, CLI, re-mapping and refill all preserve it);
    (b) the buoyant sphere rises, FP32 matching FP64."""
    import torch
    pkg, ora = env
    w = synth.refined()
    cfg, s = w["config"], w["spheres"][0]
    U = np.array([0.0, 0.0, 0.03])
    comove = dict(s, density_ratio=1e9, cv=0.0, cv_omega=0.0, u=tuple(U))
    rest = dict(cfg, gravity=(0.0, 0.0, 0.0))
    n0 = cfg["n"]
    u0 = np.zeros((3, n0[2], n0[1], n0[0]))
    u0[2] = U[2]
    say("case refined full size co-moving")
    sim = pkg.Sim(rest, [comove], storage="f64")
    sim.init(1.0, u0)
    counts = [sim.level_blocks(l).shape[0] for l in range(3)]
    say(f"  blocks per level {counts}")
    assert counts[2] >= 64 and counts[0] >= 2000
    sim.step(20)
    sim.sync()
    feq = ora.equilibrium(1.0, U)
    for l in range(3):
        f = sim.populations(l)
        fluid = np.abs(f).sum(axis=0) > 0
        err = np.abs(f[:, fluid] - feq[:, None]).max()
        say(f"  level {l}: {fluid.sum()} fluid cells, max |f - f^eq| {err:.2e}")
        assert err < 1e-14
        del f
    x, u, _ = sim.particle(0)
    assert np.abs(u - U).max() < 1e-14
    sim.close()
    del sim
    torch.cuda.empty_cache()
    say("case refined full size rise")
    uz = {}
    for st in ("f64", "f32"):
        sim = pkg.Sim(cfg, [s], storage=st, history=80)
        sim.init()
        sim.step(20)
        sim.sync()
        uz[st] = sim.history(0, 80)[:, 11]
        sim.close()
        del sim
        torch.cuda.empty_cache()
    say(f"  u_z after 80 finest steps: f64 {uz['f64'][-1]:.6e} f32 {uz['f32'][-1]:.6e}")
    assert uz["f64"][-1] > 0
    assert np.abs(uz["f32"] - uz["f64"]).max() <= 1e-4 * np.abs(uz["f64"]).max()


def test_rising256_parity_100_steps(env):
    """The rising-sphere workload at full size (256^3, no-slip walls at z = 0
    and 256, density ratio 0.5, r = 12, C_v = 0.5, Ga = 150, from rest),
    FP64, against the oracle for 100 steps: force and torque every step
    within 1e-10 (scale: the net weight, as the force starts from zero),
    the owner map every 10 steps, sphere state and populations at the end."""
    import torch
    pkg, oracle = env
    w = synth.rising()
    cfg, sph = w["config"], w["spheres"]
    s = sph[0]
    fscale = abs((s["density_ratio"] - 1.0) * cfg["gravity"][2] * 4.0 / 3.0 * np.pi * s["radius"] ** 3)
    say("case rising256 f64, 100 steps against the oracle")
    sim = pkg.Sim(cfg, sph, storage="f64", history=4)
    sim.init()
    ref = oracle.Uniform(cfg, sph)
    ref.init()
    worst = 0.0
    for k in range(1, 101):
        sim.step(1)
        ref.step(1)
        Fg, Tg = sim.force_torque(0)
        Fo, To = ref.force_torque(0)
        fs = max(np.abs(Fo).max(), fscale)
        e = max(np.abs(Fg - Fo).max() / fs, np.abs(Tg - To).max() / max(np.abs(To).max(), s["radius"] * fs))
        assert e <= 1e-10, (k, Fg, Fo, Tg, To)
        worst = max(worst, e)
        if k % 10 == 0:
            flips = int((sim.owner() != ref.owner()).sum())
            assert flips == 0, f"step {k}: {flips} mapping differences"
            say(f"  step {k}: worst F/T error so far {worst:.2e}")
    xg, ug, wg = sim.particle(0)
    xo, uo, wo = ref.particle(0)
    assert np.abs(xg - xo).max() < 1e-12 and np.abs(ug - uo).max() < 1e-14
    fg = sim.populations()
    rel = np.abs(fg - ref.post_collision()).max() / np.abs(fg).max()
    say(f"  u_z {ug[2]:.6e} vs {uo[2]:.6e}; population rel err {rel:.2e}")
    assert rel <= 1e-12
    sim.close()
    del sim, ref, fg
    torch.cuda.empty_cache()
