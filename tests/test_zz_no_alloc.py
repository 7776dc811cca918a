"""The entry point that allocates nothing (vmlbm_totals_static) against the
one it stands in for (vmlbm_totals), through the C ABI: the same sums, bit
for bit, on two calls in a row, the second on a smaller grid, and on a
refined grid."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pkg():
    import torch
    import paper_2103_10882_amd as pkg
    assert torch.cuda.is_available()
    pkg.lib()
    return pkg


def same_totals(sim):
    m0, j0 = sim.totals()
    m1, j1 = sim.totals_static()
    say(f"  mass {m0!r} / {m1!r}, momentum {j0} / {j1}")
    assert m1 == m0 and np.array_equal(j1, j0)
    return m1, j1


def test_static_totals_two_calls(pkg):
    say("case totals without allocation: 40x36x48 moving sphere f32, then 12^3 f64")
    cfg = synth.base_config((40, 36, 48), periodic=(1, 1, 0), omega=1.7, gravity=(0.0, 0.0, -4e-4))
    s = synth.sphere((20.3, 17.8, 16.2), 5.2, density_ratio=0.5, cv=0.5, fixed=False, u=(0.004, -0.003, 0.0))
    big = pkg.Sim(cfg, [s], storage="f32")
    big.init(1.0, synth.velocity_perturbation((40, 36, 48), seed=3, amplitude=0.01))
    big.step(30)
    m_big, _ = same_totals(big)
    big.close()
    small_cfg = synth.base_config((12, 12, 12), omega=1.3, body_force=(1e-5, 0.0, 2e-5))
    small = pkg.Sim(small_cfg, [], storage="f64")
    small.init(1.0, synth.velocity_perturbation((12, 12, 12), seed=4, amplitude=0.01))
    small.step(5)
    m_small, j_small = same_totals(small)
    # what the smaller grid holds, not what the larger one left behind
    assert abs(m_small - 12 ** 3) < 1e-9 * 12 ** 3 and abs(m_small - m_big) > 1.0
    small.close()


def test_static_totals_refined(pkg):
    say("case totals without allocation: two-level block grid f64")
    cfg = synth.base_config((32, 32, 32), omega=1.6, body_force=(0.0, 0.0, 1e-5))
    cfg["levels"] = 2
    cfg["block"] = 16
    sim = pkg.Sim(cfg, [], storage="f64", regions=[((0, 0, 0), (2, 2, 2), 1)], check_every=0)
    sim.init(1.0, synth.velocity_perturbation((32, 32, 32), seed=5, amplitude=0.01))
    sim.step(3)
    same_totals(sim)
    sim.close()
