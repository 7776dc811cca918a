"""GPU parity of the block-structured refined grid against the refined-grid
oracle: block layouts, per-level post-collision populations (FP64 to 1e-12),
and a moving sphere on the finest level across a re-refinement."""
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


def cfg_of(n0, levels, omega=1.6, F=(0.0, 0.0, 0.0), gravity=(0.0, 0.0, 0.0)):
    c = synth.base_config(n0, omega=omega, body_force=F, gravity=gravity)
    c["levels"] = levels
    c["block"] = 16
    return c


def oracle_blocks(leaf, level, levels):
    """Origins (level cells) of the level's leaf blocks from the oracle's leaf
    field over finest block positions."""
    L = levels - 1
    s = 2 ** (L - level)
    nz, ny, nx = leaf.shape
    out = []
    for k in range(0, nz, s):
        for j in range(0, ny, s):
            for i in range(0, nx, s):
                if leaf[k, j, i] == level:
                    out.append((i // s * 16, j // s * 16, k // s * 16))
    return sorted(out)


def compare_levels(sim, ref, levels):
    worst = 0.0
    leaf = ref.leaf()
    for l in range(levels):
        org = sim.level_blocks(l)
        assert sorted(map(tuple, org.tolist())) == oracle_blocks(leaf, l, levels), f"layout of level {l}"
        if len(org) == 0:
            continue
        fg = sim.populations(l).reshape(19, len(org), 16, 16, 16)
        fo, kind = ref.level(l)
        assert (kind == 1).sum() == len(org) * 4096
        scale = np.abs(fo).max()
        for b, (x, y, z) in enumerate(org):
            worst = max(worst, np.abs(fg[:, b] - fo[:, z:z + 16, y:y + 16, x:x + 16]).max() / scale)
    return worst


REGIONS = [((8, 4, 6), (20, 14, 22), 1), ((12, 16, 16), (18, 22, 22), 2), ((0, 24, 0), (4, 28, 6), 1)]


@pytest.mark.parametrize("storage,tol,lb", [("f64", 1e-12, 1.0), ("f32", 2e-6, 1.0), ("f16", 2e-4, 1.0),
                                            ("f64", 1e-12, 100.0)])
def test_static_three_levels(env, storage, tol, lb):
    """Three static levels from a perturbed equilibrium: every level's
    interior populations against the FP64 oracle after each coarse step.
    FP16 stores deviations of about 1e-3 with a 2^-11 relative rounding, a
    few 1e-7 of the largest population per store; 2e-4 leaves room for the
    stores of three coarse steps (12 on the finest level)."""
    pkg, oracle = env
    n0 = (32, 32, 32)
    c = cfg_of(n0, 3, omega=1.7, F=(1e-5, -2e-5, 3e-5))
    c["bulk_factor"] = lb
    u0 = synth.velocity_perturbation(n0, seed=7)
    say(f"case refined32 L3 static {storage} bulk factor {lb}")
    sim = pkg.Sim(c, [], storage=storage, regions=REGIONS, check_every=0)
    sim.init(1.0, u0)
    ref = oracle.Refined(c, regions=REGIONS)
    ref.init(1.0, u0)
    rel = compare_levels(sim, ref, 3)
    say(f"  init rel {rel:.2e}")
    assert rel <= tol
    for k in range(3):
        sim.step(1)
        ref.step(1)
        sim.sync()
        rel = compare_levels(sim, ref, 3)
        say(f"  coarse step {k + 1}: rel {rel:.2e}")
        assert rel <= tol


@pytest.mark.parametrize("lb", [1.0, 100.0])
def test_moving_sphere_rerefinement(env, lb):
    """Sphere on the finest level moving across a finest-block boundary: the
    layout is re-checked every 4 coarse steps and changes; F/T, mapping,
    particle state and populations follow the oracle, with TRT and with the
    MRT collision (bulk factor 100)."""
    pkg, oracle = env
    n0 = (32, 32, 48)
    c = cfg_of(n0, 3, omega=1.8, gravity=(0.0, 0.0, -2e-4))
    c["bulk_factor"] = lb
    # top of the grown box (sphere box plus one finest block) just below the
    # boundary of a level-1 node (32 finest cells): the layout changes once
    # the heavy sphere has moved half a cell
    s = synth.sphere((64.2, 63.7, 63.5 - 5.5 - 16.0), 5.5, density_ratio=1e3, cv=0.5, fixed=False,
                     u=(0.0, 0.0, 0.1))
    u0 = synth.velocity_perturbation(n0, seed=9)
    say(f"case refined32x32x48 L3 moving f64, bulk factor {lb}")
    sim = pkg.Sim(c, [s], storage="f64", history=8, check_every=4)
    sim.init(1.0, u0)
    ref = oracle.Refined(c, spheres=[s], check_every=4)
    ref.init(1.0, u0)
    for k in range(1, 13):
        sim.step(1)
        ref.step(1)
        Fg, Tg = sim.force_torque(0)
        Fo, To = ref.force_torque(0)
        assert np.abs(Fg - Fo).max() <= 1e-10 * np.abs(Fo).max(), (k, Fg, Fo)
        assert np.abs(Tg - To).max() <= 1e-10 * max(np.abs(To).max(), 5.5 * np.abs(Fo).max()), (k, Tg, To)
    sim.sync()
    nref = sim.refinements()
    _, _, nref_o = ref.counters()
    say(f"  refinements gpu {nref} oracle {nref_o}")
    assert nref == nref_o and nref >= 1
    xg, ug, wg = sim.particle(0)
    xo, uo, wo = ref.particle(0)
    assert np.abs(xg - xo).max() < 1e-11
    rel = compare_levels(sim, ref, 3)
    say(f"  population rel err {rel:.2e}")
    assert rel <= 1e-12
    # finest-level mapping
    org = sim.level_blocks(2)
    og = sim.owner(2).reshape(len(org), 16, 16, 16)
    oo = ref.owner()
    for b, (x, y, z) in enumerate(org):
        assert (og[b] == oo[z:z + 16, y:y + 16, x:x + 16]).all()


def test_refined_layout_across_periodic_boundary(env):
    """Two-level grid, sphere near x = 0: its refined region wraps around the
    periodic boundary (coarse nodes 3 and 0 of 4 along x) and grows to node 1
    once the sphere's grown box crosses x = 48 (after 2 cells of motion);
    layouts, forces and populations follow the oracle throughout."""
    pkg, oracle = env
    n0 = (64, 32, 32)
    c = cfg_of(n0, 2, omega=1.7, F=(0.0, 0.0, 2e-6))
    s = synth.sphere((8.0, 31.3, 33.7), 6.0, density_ratio=2e3, cv=0.5, fixed=False, u=(0.05, 0.0, 0.01))
    u0 = synth.velocity_perturbation(n0, seed=12)
    say("case refined64x32x32 L2 periodic wrap f64")
    sim = pkg.Sim(c, [s], storage="f64", history=8, check_every=4)
    sim.init(1.0, u0)
    ref = oracle.Refined(c, spheres=[s], check_every=4)
    ref.init(1.0, u0)
    leaf = ref.leaf()
    assert leaf[:, :, 0].max() == 1 and leaf[:, :, -1].max() == 1 and leaf.min() == 0   # wraps
    for k in range(1, 25):
        sim.step(1)
        ref.step(1)
        Fg, Tg = sim.force_torque(0)
        Fo, To = ref.force_torque(0)
        assert np.abs(Fg - Fo).max() <= 1e-10 * np.abs(Fo).max(), (k, Fg, Fo)
        assert np.abs(Tg - To).max() <= 1e-10 * max(np.abs(To).max(), 6.0 * np.abs(Fo).max()), (k, Tg, To)
    sim.sync()
    assert sim.refinements() == ref.counters()[2] >= 1
    rel = compare_levels(sim, ref, 2)
    say(f"  refinements {sim.refinements()}; population rel err {rel:.2e}")
    assert rel <= 1e-12


def test_single_level_block_grid_equals_uniform(env):
    """levels = 1: every block is a level-0 leaf, no ghosts and no
    coalescence; 16^3 blocks must reproduce the uniform grid (FP64)."""
    pkg, oracle = env
    n0 = (48, 32, 16)
    c = cfg_of(n0, 1, omega=1.3, F=(1e-5, 0.0, 2e-5))
    u0 = synth.velocity_perturbation(n0, seed=13, amplitude=0.01)
    say("case block grid 48x32x16 L1 f64")
    sim = pkg.Sim(c, [], storage="f64", check_every=0)
    sim.init(1.0, u0)
    ref = oracle.Uniform(synth.base_config(n0, omega=1.3, body_force=(1e-5, 0.0, 2e-5)))
    ref.init(1.0, u0)
    sim.step(20)
    ref.step(20)
    sim.sync()
    org = sim.level_blocks(0)
    assert len(org) == 3 * 2 * 1
    fg = sim.populations(0).reshape(19, len(org), 16, 16, 16)
    fo = ref.post_collision()
    worst = 0.0
    for b, (x, y, z) in enumerate(org):
        worst = max(worst, np.abs(fg[:, b] - fo[:, z:z + 16, y:y + 16, x:x + 16]).max())
    say(f"  max abs diff {worst:.2e}")
    assert worst <= 1e-15


def test_static_four_levels(env):
    """Four levels (the deepest the dense oracle follows at this size), nested
    static regions."""
    pkg, oracle = env
    n0 = (64, 16, 16)
    c = cfg_of(n0, 4, omega=1.9, F=(0.0, 0.0, 1e-6))
    regions = [((0, 6, 6), (2, 9, 9), 3)]
    u0 = synth.velocity_perturbation(n0, seed=14, amplitude=0.01)
    say("case refined64x16x16 L4 static f64")
    sim = pkg.Sim(c, [], storage="f64", regions=regions, check_every=0)
    sim.init(1.0, u0)
    ref = oracle.Refined(c, regions=regions)
    ref.init(1.0, u0)
    leaf = ref.leaf()
    assert leaf.max() == 3 and leaf.min() == 0
    for k in range(2):
        sim.step(1)
        ref.step(1)
    sim.sync()
    rel = compare_levels(sim, ref, 4)
    say(f"  population rel err {rel:.2e}")
    assert rel <= 1e-12


def test_five_levels_static_oracle(env):
    """Five levels against the oracle on the smallest domain, one coarse
    16^3 block (finest level 256^3; the oracle's dense per-level arrays
    take about 8 GB): static nesting down to level 4 around one spot, a
    rough start and a body force, every level's populations after two coarse
    steps (32 finest steps) within 1e-12."""
    pkg, oracle = env
    n0 = (16, 16, 16)
    c = cfg_of(n0, 5, omega=1.8, F=(2e-7, -1e-7, 3e-7))
    regions = [((7, 7, 7), (9, 9, 9), 4)]
    u0 = synth.velocity_perturbation(n0, seed=21, amplitude=0.01)
    say("case refined16^3 L5 static f64 against the oracle")
    sim = pkg.Sim(c, [], storage="f64", regions=regions, check_every=0)
    sim.init(1.0, u0)
    ref = oracle.Refined(c, regions=regions)
    ref.init(1.0, u0)
    assert ref.leaf().max() == 4
    for k in range(2):
        sim.step(1)
        ref.step(1)
    sim.sync()
    rel = compare_levels(sim, ref, 5)
    say(f"  blocks per level {[int(sim.level_blocks(l).shape[0]) for l in range(5)]}; population rel err {rel:.2e}")
    assert rel <= 1e-12
    sim.close()


def test_five_levels_moving_sphere_oracle(env):
    """Five levels against the oracle with a heavy sphere moving on level 4
    (one coarse 16^3 block, finest 256^3): the particle criterion holds the
    finest level around it and the layout changes once its grown box crosses
    a finest-block face; force and torque every finest step, layouts,
    particle state and every level's populations after three coarse steps."""
    pkg, oracle = env
    n0 = (16, 16, 16)
    c = cfg_of(n0, 5, omega=1.7)
    # the grown box's lower face crosses z = 128, the boundary between two
    # pairs of sibling finest blocks, during the run
    s = synth.sphere((128.3, 127.8, 147.8), 5.5, density_ratio=1e3, cv=0.5, fixed=False, u=(0.0, 0.0, 0.05))
    u0 = synth.velocity_perturbation(n0, seed=22, amplitude=0.005)
    say("case refined16^3 L5 moving sphere f64 against the oracle")
    sim = pkg.Sim(c, [s], storage="f64", history=64, check_every=1)
    sim.init(1.0, u0)
    ref = oracle.Refined(c, spheres=[s], check_every=1)
    ref.init(1.0, u0)
    for k in range(1, 4):
        sim.step(1)
        ref.step(1)
        hg = sim.history(0, 16)
        Fo, To = ref.force_torque(0)
        Fg, Tg = hg[-1, 0:3], hg[-1, 3:6]
        assert np.abs(Fg - Fo).max() <= 1e-10 * np.abs(Fo).max(), (k, Fg, Fo)
        assert np.abs(Tg - To).max() <= 1e-10 * max(np.abs(To).max(), 5.5 * np.abs(Fo).max()), (k, Tg, To)
    sim.sync()
    nref = sim.refinements()
    _, _, nref_o = ref.counters()
    say(f"  refinements gpu {nref} oracle {nref_o} (tables built ahead: {sim.prebuilt_layouts()}); "
        f"blocks {[int(sim.level_blocks(l).shape[0]) for l in range(5)]}")
    assert nref == nref_o and nref >= 1
    # the change is the one predicted from the sphere's velocity after the
    # first check, so its tables come from the host thread
    assert sim.prebuilt_layouts() >= 1
    xg, ug, wg = sim.particle(0)
    xo, uo, wo = ref.particle(0)
    assert np.abs(xg - xo).max() < 1e-11 and np.abs(ug - uo).max() < 1e-12
    rel = compare_levels(sim, ref, 5)
    say(f"  population rel err {rel:.2e}")
    assert rel <= 1e-12
    sim.close()


def test_reversed_sphere_unpredicted_layout(env):
    """Layout tables are built ahead for the block ranges predicted from the
    spheres' velocities; a change that was not predicted is built at the
    check.  A heavy sphere moves up, is turned around after the first check
    (whose prediction was a crossing above), and its grown box then crosses
    a level-1 node boundary below: the re-refinement takes the check's own
    build, and F/T, layout, particle and populations follow the oracle."""
    pkg, oracle = env
    n0 = (32, 32, 48)
    c = cfg_of(n0, 3, omega=1.8)
    # lower face of the grown box (sphere box minus one finest block) 0.05
    # cells above the level-1 node boundary at z = 64; up 0.4 cells in the
    # first coarse step, down 0.6 in the second, so the crossing happens
    # before any check has seen the sphere move down
    s = synth.sphere((64.2, 63.7, 64.05 + 5.5 + 16.0), 5.5, density_ratio=1e3, cv=0.5, fixed=False,
                     u=(0.0, 0.0, 0.1))
    u0 = synth.velocity_perturbation(n0, seed=13)
    say("case refined32x32x48 L3 sphere reversed after the first check, f64")
    sim = pkg.Sim(c, [s], storage="f64", history=8, check_every=1)
    sim.init(1.0, u0)
    ref = oracle.Refined(c, spheres=[s], check_every=1)
    ref.init(1.0, u0)
    for k in range(1, 7):
        if k == 2:
            sim.set_sphere_motion(0, u=(0.0, 0.0, -0.15), fixed=0)
            ref.set_sphere_motion(0, u=(0.0, 0.0, -0.15), fixed=0)
        sim.step(1)
        ref.step(1)
        Fg, Tg = sim.force_torque(0)
        Fo, To = ref.force_torque(0)
        assert np.abs(Fg - Fo).max() <= 1e-10 * np.abs(Fo).max(), (k, Fg, Fo)
        assert np.abs(Tg - To).max() <= 1e-10 * max(np.abs(To).max(), 5.5 * np.abs(Fo).max()), (k, Tg, To)
    sim.sync()
    nref, npre = sim.refinements(), sim.prebuilt_layouts()
    _, _, nref_o = ref.counters()
    say(f"  refinements gpu {nref} oracle {nref_o}, of which tables built ahead {npre}")
    assert nref == nref_o and nref >= 1
    assert npre < nref
    xg, _, _ = sim.particle(0)
    xo, _, _ = ref.particle(0)
    assert np.abs(xg - xo).max() < 1e-11
    rel = compare_levels(sim, ref, 3)
    say(f"  population rel err {rel:.2e}")
    assert rel <= 1e-12
    sim.close()


def write_from_oracle(sim, ref, levels):
    """Copy the oracle's interior populations of every level into the GPU
    grid, block by block in the GPU's slot order (same layout on both)."""
    for l in range(levels):
        org = sim.level_blocks(l)
        if len(org) == 0:
            continue
        fo, _ = ref.level(l)
        f = np.empty((19, len(org), 16, 16, 16))
        for b, (x, y, z) in enumerate(org):
            f[:, b] = fo[:, z:z + 16, y:y + 16, x:x + 16]
        sim.write_populations(f.reshape(19, -1), l)


def shear_x_field(ref, level, levels, U, wavelength, phase):
    nx, ny, nz = ref.dims(level)
    s = 2 ** (levels - 1 - level)
    xf = (np.arange(nx) + 0.5) * s
    u = np.zeros((3, nz, ny, nx))
    u[2] = U * np.sin(2 * np.pi * xf / wavelength + phase)[None, None, :]
    return u


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 2e-6)])
def test_curl_refine_then_coarsen(env, storage, tol):
    """Curl-sensor criterion of Sec. 4.2.2 with check_every = 1: a shear
    field u_z = U sin(k x + pi/4) refines the level-0 blocks whose sensor
    exceeds sigma_c (two of four along x, margin > 2 %); the same field at
    5 % strength on both levels coarsens them again.  Layouts and
    populations follow the oracle after each check."""
    pkg, oracle = env
    n0 = (64, 16, 16)
    c = cfg_of(n0, 2, omega=1.6)
    U, lam = 1e-3, 128.0
    k = 2 * np.pi / lam
    c["curl_threshold"] = 0.8 * U * k * 2 ** 1.5
    c["curl_coarsen"] = 0.2
    say(f"case curl shear 64x16x16 L2 {storage}")
    sim = pkg.Sim(c, [], storage=storage, check_every=1)
    sim.init(1.0)
    ref = oracle.Refined(c, check_every=1)
    ref.init(1.0)
    ref.set_level_velocity(0, 1.0, shear_x_field(ref, 0, 2, U, lam, np.pi / 4))
    write_from_oracle(sim, ref, 2)
    sim.step(1)
    ref.step(1)
    sim.sync()
    leaf = ref.leaf()
    assert leaf.max() == 1 and leaf.min() == 0
    rel = compare_levels(sim, ref, 2)
    say(f"  refined: {len(sim.level_blocks(1))} level-1 blocks, population rel err {rel:.2e}")
    assert rel <= tol
    for l in range(2):
        ref.set_level_velocity(l, 1.0, shear_x_field(ref, l, 2, 0.05 * U, lam, np.pi / 4))
    write_from_oracle(sim, ref, 2)
    sim.step(1)
    ref.step(1)
    sim.sync()
    assert ref.leaf().max() == 0
    rel = compare_levels(sim, ref, 2)
    say(f"  coarsened: population rel err {rel:.2e}")
    assert rel <= tol
    assert sim.refinements() == ref.counters()[2] == 2


@pytest.mark.parametrize("storage,tol", [("f64", 1e-12), ("f32", 2e-6)])
def test_curl_vortex_tube_three_levels(env, storage, tol):
    """A Gaussian vortex tube (plus small noise) on an all-level-0 start:
    the curl sensor refines the core to level 1 at the first check and to
    level 2 at the second (sensors on all three levels, blocks next to level
    interfaces, fluid-only differences); layouts and populations follow the
    oracle over four coarse steps, each followed by a check."""
    pkg, oracle = env
    n0 = (64, 32, 32)
    c = cfg_of(n0, 3, omega=1.7, F=(1e-5, 0.0, 0.0))
    u0 = synth.vortex_tube(n0, (24.3, 15.2), 4.0, 1e-3) + synth.velocity_perturbation(n0, seed=21, amplitude=1e-5)
    c["curl_threshold"] = 9.3e-4
    c["curl_coarsen"] = 0.2
    say(f"case curl vortex 64x32x32 L3 {storage}")
    sim = pkg.Sim(c, [], storage=storage, check_every=1)
    sim.init(1.0, u0)
    ref = oracle.Refined(c, check_every=1)
    ref.init(1.0, u0)
    for k in range(1, 5):
        sim.step(1)
        ref.step(1)
        sim.sync()
        rel = compare_levels(sim, ref, 3)
        say(f"  step {k}: blocks per level {[len(sim.level_blocks(l)) for l in range(3)]}, rel err {rel:.2e}")
        assert rel <= tol
    assert ref.leaf().max() == 2
    assert sim.refinements() == ref.counters()[2] == 2


@pytest.mark.parametrize("levels", [5, 6])
def test_deep_hierarchy_conservation(env, levels):
    """Five and six levels (the paper runs up to 9): the oracle's dense
    per-level arrays are too large here, so the checks are properties that
    hold at any depth.  Static nested refinement down to the finest level
    around one spot: volume-weighted mass stays constant and momentum grows
    by V 2^L F per coarse step (every level forced with its acoustically
    scaled F); the 2:1 shape holds between touching leaves."""
    pkg, oracle = env
    n0 = (64, 64, 64) if levels == 5 else (128, 128, 128)   # room for a level-0 leaf
    F = np.array([1e-6, -2e-6, 3e-6])
    c = cfg_of(n0, levels, omega=1.7, F=tuple(F))
    regions = [((5, 6, 7), (7, 8, 9), levels - 1)]
    u0 = synth.velocity_perturbation(n0, seed=15, amplitude=0.01)
    say(f"case deep hierarchy {n0[0]}^3 coarse, {levels} levels, f64")
    sim = pkg.Sim(c, [], storage="f64", regions=regions, check_every=0)
    sim.init(1.0, u0)
    counts = [int(sim.level_blocks(l).shape[0]) for l in range(levels)]
    say(f"  blocks per level {counts}")
    assert min(counts) > 0
    # 2:1 between touching leaves, on finest block positions
    L = levels - 1
    nb = n0[0] // 16 * 2 ** L
    leaf = np.full((nb, nb, nb), -1, dtype=np.int8)
    for l in range(levels):
        s = 2 ** (L - l)
        for x, y, z in sim.level_blocks(l).tolist():
            i, j, k = x // 16 * s, y // 16 * s, z // 16 * s
            assert (leaf[k:k + s, j:j + s, i:i + s] == -1).all()
            leaf[k:k + s, j:j + s, i:i + s] = l
    assert (leaf >= 0).all()
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                nbr = np.roll(leaf, (dz, dy, dx), axis=(0, 1, 2))
                assert np.abs(leaf.astype(int) - nbr).max() <= 1
    V = n0[0] * n0[1] * n0[2]
    m0, J0 = sim.totals()
    for s in range(1, 4):
        sim.step(1)
        m, J = sim.totals()
        say(f"  coarse step {s}: mass drift {m - m0:.2e}, momentum error {np.abs(J - J0 - s * V * 2 ** L * F).max():.2e}")
        assert abs(m - m0) < s * V * 1e-13
        assert np.abs(J - J0 - s * V * 2 ** L * F).max() < s * V * 1e-13
    sim.close()


def test_deep_hierarchy_comoving_sphere(env):
    """Five levels, a heavy sphere moving with a uniform flow across finest
    blocks (re-refinement included): every interior cell of every level
    stays at f^eq(1, U), and the sphere keeps U."""
    pkg, oracle = env
    n0 = (32, 32, 32)
    U = np.array([0.02, -0.01, 0.03])
    c = cfg_of(n0, 5, omega=1.6)
    s = synth.sphere((250.3, 262.8, 243.1), 5.5, density_ratio=1e9, cv=0.0, fixed=False, u=tuple(U))
    u0 = np.broadcast_to(U[:, None, None, None], (3,) + n0[::-1]).copy()
    say("case deep hierarchy co-moving sphere, 5 levels, f64")
    sim = pkg.Sim(c, [s], storage="f64", check_every=1)
    sim.init(1.0, u0)
    sim.step(6)
    sim.sync()
    say(f"  refinements {sim.refinements()}, blocks {[int(sim.level_blocks(l).shape[0]) for l in range(5)]}")
    assert sim.refinements() >= 1
    feq = oracle.equilibrium(1.0, U)
    for l in range(5):
        f = sim.populations(l)
        fluid = np.abs(f).sum(axis=0) > 0
        if fluid.sum() == 0:
            continue
        err = np.abs(f[:, fluid] - feq[:, None]).max()
        say(f"  level {l}: {int(fluid.sum())} fluid cells, max |f - f^eq| {err:.2e}")
        assert err < 1e-14
    _, u, _ = sim.particle(0)
    assert np.abs(u - U).max() < 1e-14
    sim.close()


def test_nine_levels_comoving_sphere(env):
    """Nine levels, the depth of the paper's Table 3 setups, on one coarse
    16^3 block (finest level 4096^3 cells, of which only the blocks around
    the sphere are stored): a heavy sphere moving with a uniform flow crosses
    finest blocks over two coarse steps (512 finest steps), re-refining on
    the way; every interior cell of every level stays at f^eq(1, U)."""
    pkg, oracle = env
    n0 = (16, 16, 16)
    U = np.array([0.012, -0.008, 0.015])
    c = cfg_of(n0, 9, omega=1.6)
    # the grown box's lower z face crosses 2048, between two pairs of
    # sibling finest blocks, during the run
    s = synth.sphere((2050.3, 2045.8, 2064.0), 4.5, density_ratio=1e9, cv=0.0, fixed=False, u=tuple(U))
    u0 = np.broadcast_to(U[:, None, None, None], (3,) + n0[::-1]).copy()
    say("case deep hierarchy co-moving sphere, 9 levels, f64")
    sim = pkg.Sim(c, [s], storage="f64", check_every=1)
    sim.init(1.0, u0)
    sim.step(2)
    sim.sync()
    blocks = [int(sim.level_blocks(l).shape[0]) for l in range(9)]
    say(f"  refinements {sim.refinements()}, blocks {blocks}")
    assert sim.refinements() >= 1 and blocks[8] > 0
    feq = oracle.equilibrium(1.0, U)
    for l in range(9):
        if blocks[l] == 0:
            continue
        f = sim.populations(l)
        fluid = np.abs(f).sum(axis=0) > 0
        err = np.abs(f[:, fluid] - feq[:, None]).max()
        say(f"  level {l}: {int(fluid.sum())} fluid cells, max |f - f^eq| {err:.2e}")
        assert err < 1e-14
    _, u, _ = sim.particle(0)
    assert np.abs(u - U).max() < 1e-14
    sim.close()


def test_two_spheres_refined(env):
    """Two spheres on the finest level of a 3-level grid, one held and one
    moving through the layout: per-sphere link lists, force slots and
    refinement boxes; F/T of both every step and populations at the end
    follow the oracle."""
    pkg, oracle = env
    n0 = (64, 32, 32)
    c = cfg_of(n0, 3, omega=1.7, F=(2e-6, 0.0, 1e-6))
    held = synth.sphere((40.6, 62.2, 58.9), 6.5, fixed=True)
    # the moving sphere's refinement box reaches the next finest block
    # after about 2.5 cells of motion along x
    moving = synth.sphere((168.2, 66.1, 70.3), 5.5, density_ratio=50.0, cv=0.5, fixed=False,
                          u=(0.08, -0.02, 0.05))
    u0 = synth.velocity_perturbation(n0, seed=16)
    say("case refined64x32x32 L3 two spheres f64")
    sim = pkg.Sim(c, [held, moving], storage="f64", history=8, check_every=4)
    sim.init(1.0, u0)
    ref = oracle.Refined(c, spheres=[held, moving], check_every=4)
    ref.init(1.0, u0)
    for k in range(1, 13):
        sim.step(1)
        ref.step(1)
        for i, r in ((0, 6.5), (1, 5.5)):
            Fg, Tg = sim.force_torque(i)
            Fo, To = ref.force_torque(i)
            assert np.abs(Fg - Fo).max() <= 1e-10 * np.abs(Fo).max(), (k, i, Fg, Fo)
            assert np.abs(Tg - To).max() <= 1e-10 * max(np.abs(To).max(), r * np.abs(Fo).max()), (k, i, Tg, To)
    sim.sync()
    assert sim.refinements() == ref.counters()[2] >= 1
    for i in range(2):
        xg, ug, _ = sim.particle(i)
        xo, uo, _ = ref.particle(i)
        assert np.abs(xg - xo).max() < 1e-11 and np.abs(ug - uo).max() < 1e-12
    rel = compare_levels(sim, ref, 3)
    say(f"  refinements {sim.refinements()}; population rel err {rel:.2e}")
    assert rel <= 1e-12


def test_rotation_only_sphere_refined(env):
    """Hold modes on the refined grid: a sphere held in a shear wave, then
    switched to rotation-only (Sec. 3.4.2 protocol) with the Lagrange
    virtual-force scheme; F/T every step and the angular velocity follow
    the oracle, the position stays put."""
    pkg, oracle = env
    n0 = (32, 16, 32)
    c = cfg_of(n0, 2, omega=1.5)
    s = synth.sphere((31.3, 15.6, 33.2), 5.0, density_ratio=0.8, cv=1.0, fixed=True, vm_scheme=2)
    z = np.arange(n0[2]) + 0.5
    u0 = np.zeros((3, n0[2], n0[1], n0[0]))
    u0[0] = (0.02 * np.sin(2 * np.pi * z / n0[2]))[:, None, None]
    say("case refined32x16x32 L2 hold then rotate f64")
    sim = pkg.Sim(c, [s], storage="f64", history=8, check_every=4)
    sim.init(1.0, u0)
    ref = oracle.Refined(c, spheres=[s], check_every=4)
    ref.init(1.0, u0)
    for k in range(1, 9):
        if k == 3:
            for o in (sim, ref):
                o.set_sphere_motion(0, fixed=2)
        sim.step(1)
        ref.step(1)
        Fg, Tg = sim.force_torque(0)
        Fo, To = ref.force_torque(0)
        assert np.abs(Fg - Fo).max() <= 1e-10 * np.abs(Fo).max(), (k, Fg, Fo)
        assert np.abs(Tg - To).max() <= 1e-10 * max(np.abs(To).max(), 5.0 * np.abs(Fo).max()), (k, Tg, To)
    sim.sync()
    xg, ug, wg = sim.particle(0)
    xo, uo, wo = ref.particle(0)
    assert (xg == np.array(s["x"])).all() and (ug == 0.0).all()
    assert np.abs(wg - wo).max() <= 1e-12 * np.abs(wo).max() and np.abs(wo).max() > 0
    rel = compare_levels(sim, ref, 2)
    say(f"  w {wg}, population rel err {rel:.2e}")
    assert rel <= 1e-12


def test_large_sphere_refined(env):
    """A sphere of radius 27 on the finest level of a 2-level grid: more link
    cells than the finest level's link-cell pass takes in one round (256
    workgroups of 32 cells), so its later rounds run; F/T every coarse step,
    the particle and the populations follow the oracle."""
    pkg, oracle = env
    n0 = (96, 64, 64)          # room for level-0 leaves beyond the sphere's box in x
    r = 27.0
    centre = (64.3, 63.8, 64.4)
    c = cfg_of(n0, 2, omega=1.7, F=(1e-6, -2e-6, 3e-6))
    s = synth.sphere(centre, r, density_ratio=20.0, cv=0.5, fixed=False, u=(0.01, -0.005, 0.02))
    # link cells: fluid cells with a D3Q19 neighbour inside the sphere
    Z, Y, X = np.meshgrid(np.arange(128) + 0.5, np.arange(128) + 0.5, np.arange(192) + 0.5, indexing="ij")
    inside = (X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2 <= r * r
    near = np.zeros_like(inside)
    for q in range(1, 19):
        cx, cy, cz = oracle.lattice()[0][q]
        near |= np.roll(inside, (-int(cz), -int(cy), -int(cx)), axis=(0, 1, 2))
    n_links = int((near & ~inside).sum())
    assert n_links > 256 * 32, n_links
    u0 = synth.velocity_perturbation(n0, seed=23)
    say(f"case refined96x64x64 L2 large sphere r={r} ({n_links} link cells) f64")
    sim = pkg.Sim(c, [s], storage="f64", history=8, check_every=4)
    sim.init(1.0, u0)
    ref = oracle.Refined(c, spheres=[s], check_every=4)
    ref.init(1.0, u0)
    assert 0 < len(sim.level_blocks(0)) and 0 < len(sim.level_blocks(1))
    for k in range(1, 5):
        sim.step(1)
        ref.step(1)
        Fg, Tg = sim.force_torque(0)
        Fo, To = ref.force_torque(0)
        assert np.abs(Fg - Fo).max() <= 1e-10 * np.abs(Fo).max(), (k, Fg, Fo)
        assert np.abs(Tg - To).max() <= 1e-10 * max(np.abs(To).max(), r * np.abs(Fo).max()), (k, Tg, To)
    sim.sync()
    xg, ug, _ = sim.particle(0)
    xo, uo, _ = ref.particle(0)
    assert np.abs(xg - xo).max() < 1e-11 and np.abs(ug - uo).max() < 1e-12
    rel = compare_levels(sim, ref, 2)
    say(f"  population rel err {rel:.2e}")
    assert rel <= 1e-12



def _level_field(sim, level, n):
    """A level's interior populations on its full cell grid (0 outside its
    leaf blocks) and the mask of its leaf cells."""
    org = sim.level_blocks(level)
    f = sim.populations(level).reshape(19, len(org), 16, 16, 16)
    full = np.zeros((19, n[2], n[1], n[0]))
    mask = np.zeros((n[2], n[1], n[0]), dtype=bool)
    for b, (x, y, z) in enumerate(org):
        full[:, z:z + 16, y:y + 16, x:x + 16] = f[:, b]
        mask[z:z + 16, y:y + 16, x:x + 16] = True
    return full, mask


def _blocks_of(full, org):
    """Populations of a full level grid in the level's slot order."""
    f = np.empty((19, len(org), 16, 16, 16))
    for b, (x, y, z) in enumerate(org):
        f[:, b] = full[:, z:z + 16, y:y + 16, x:x + 16]
    return f.reshape(19, -1)


def _shift(a, c, k=1):
    """a moved by k c along (x, y, z): out[x] = a[x - k c], periodic."""
    return np.roll(a, shift=(k * int(c[2]), k * int(c[1]), k * int(c[0])), axis=(0, 1, 2))


@pytest.mark.parametrize("storage", ["f64", "f32", "f16"])
def test_level_pull_reference(env, storage):
    """The bandwidth reference with the level sweep's access pattern moves
    population q of every leaf cell from x - c_q through the level's blocks,
    bit for bit: on a single-level grid one pull is the periodic shift of
    each population by c_q and two pulls the shift by 2 c_q; on the coarse
    level of a 3-level grid a source inside the refined region, which the
    level does not store, gives 0."""
    pkg, oracle = env
    c_lat, _, _ = oracle.lattice()
    rng = np.random.default_rng(11)

    say(f"case level pull single level 48x32x16 {storage}")
    n0 = (48, 32, 16)
    sim = pkg.Sim(cfg_of(n0, 1), [], storage=storage, check_every=0)
    sim.init()
    org = sim.level_blocks(0)
    sim.write_populations(rng.uniform(-0.02, 0.02, size=(19, len(org) * 4096)), 0)
    f0, mask = _level_field(sim, 0, n0)
    assert mask.all()
    for reps in (1, 2):
        sim.write_populations(_blocks_of(f0, org), 0)
        sim.level_pull(0, reps)
        sim.sync()
        got, _ = _level_field(sim, 0, n0)
        want = np.stack([_shift(f0[q], c_lat[q], reps) for q in range(19)])
        assert np.array_equal(got, want), f"{reps} pull(s)"
    # a level the grid does not have, and no pull at all, are refused
    for level, reps in ((1, 1), (-1, 1), (0, 0)):
        with pytest.raises(pkg.VmlbmError):
            sim.level_pull(level, reps)
    sim.close()

    say(f"case level pull coarse level of 3, 32^3 {storage}")
    n0 = (32, 32, 32)
    sim = pkg.Sim(cfg_of(n0, 3), [], storage=storage, regions=REGIONS, check_every=0)
    sim.init()
    org = sim.level_blocks(0)
    sim.write_populations(rng.uniform(-0.02, 0.02, size=(19, len(org) * 4096)), 0)
    f0, mask = _level_field(sim, 0, n0)
    assert not mask.all()
    sim.level_pull(0, 1)
    sim.sync()
    got, _ = _level_field(sim, 0, n0)
    want = np.stack([np.where(_shift(mask, c_lat[q]), _shift(f0[q], c_lat[q]), 0.0) for q in range(19)])
    assert np.array_equal(got[:, mask], want[:, mask])
    sim.close()
