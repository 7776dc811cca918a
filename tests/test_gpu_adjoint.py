"""GPU adjoint of the fixed-sphere drag against the dual-number oracle
gradient and central finite differences."""
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


def small_case():
    n = 24
    cfg = synth.base_config((n, n, n), omega=1.6, body_force=(0, 0, 1e-5))
    sph = [synth.sphere((12.3, 11.8, 12.1), 4.2)]
    return cfg, sph, 120, 80, 20


@pytest.mark.parametrize("storage,tol", [("f64", 1e-9), ("f32", 1e-3)])
def test_adjoint_vs_dual(env, storage, tol):
    pkg, oracle = env
    cfg, sph, N, A, K = small_case()
    say(f"case adjoint24 {storage}")
    J_o, g_o = oracle.drag_gradient(cfg, sph, N, A)
    sim = pkg.Sim(cfg, sph, storage=storage, history=N - A, adjoint_steps=N, ckpt_every=K)
    J = sim.forward_ckpt(0, N, A, K)
    g = sim.adjoint(1.0)
    say(f"  J {J:.12e} vs {J_o:.12e}; grad {g} vs {g_o}")
    assert abs(J - J_o) <= (1e-11 if storage == "f64" else 1e-4) * abs(J_o)
    assert np.abs(g - g_o).max() <= tol * np.abs(g_o).max() * 1.0
    assert abs(g[0] - g_o[0]) <= tol * abs(g_o[0])
    assert abs(g[1] - g_o[1]) <= tol * abs(g_o[1])


def test_autograd_function(env):
    import torch
    pkg, oracle = env
    cfg, sph, N, A, K = small_case()
    say("case autograd24 f64")
    sim = pkg.Sim(cfg, sph, storage="f64", history=N - A, adjoint_steps=N, ckpt_every=K)
    F = torch.tensor(1e-5, dtype=torch.float64, requires_grad=True)
    w = torch.tensor(1.6, dtype=torch.float64, requires_grad=True)
    J = pkg.drag(F, w, sim, 0, N, A, K)
    J.backward()
    _, g_o = oracle.drag_gradient(cfg, sph, N, A)
    assert abs(F.grad.item() - g_o[0]) <= 1e-9 * abs(g_o[0])
    assert abs(w.grad.item() - g_o[1]) <= 1e-9 * abs(g_o[1])


def test_drag_twice_before_backward(env):
    """Two drag evaluations on one simulation before the first one's
    backward (a finite-difference probe in between): the first gradient
    still belongs to its own parameters.  The library refuses an adjoint
    whose checkpoints were taken with other parameters."""
    import torch
    pkg, oracle = env
    cfg, sph, N, A, K = small_case()
    say("case drag-twice24 f64")
    sim = pkg.Sim(cfg, sph, storage="f64", history=N - A, adjoint_steps=N, ckpt_every=K)
    F = torch.tensor(1e-5, dtype=torch.float64, requires_grad=True)
    w = torch.tensor(1.6, dtype=torch.float64, requires_grad=True)
    J = pkg.drag(F, w, sim, 0, N, A, K)
    with torch.no_grad():
        pkg.drag(torch.tensor(1.1e-5, dtype=torch.float64), torch.tensor(1.55, dtype=torch.float64), sim, 0, N, A, K)
    J.backward()
    _, g_o = oracle.drag_gradient(cfg, sph, N, A)
    assert abs(F.grad.item() - g_o[0]) <= 1e-9 * abs(g_o[0])
    assert abs(w.grad.item() - g_o[1]) <= 1e-9 * abs(g_o[1])
    sim.set_params(1e-5, 1.6)
    with pytest.raises(pkg.VmlbmError) as e:
        sim.adjoint(1.0)
    assert e.value.code == -4


def test_adjoint_full_size_fd(env):
    """128^3, r = 10, 2000 steps, window 1500..1999, checkpoints every 50:
    FP32 adjoint vs FP64 adjoint, and FP64 adjoint vs central differences of
    the FP64 forward (h = 1e-4 relative)."""
    pkg, _ = env
    w = synth.adjoint()
    cfg, sph = w["config"], w["spheres"]
    N, A, K = w["steps"], w["avg_from"], w["ckpt_every"]
    say("case adjoint128 f64/f32")
    s64 = pkg.Sim(cfg, sph, storage="f64", history=N - A, adjoint_steps=N, ckpt_every=K)
    J64 = s64.forward_ckpt(0, N, A, K)
    g64 = s64.adjoint(1.0)
    s32 = pkg.Sim(cfg, sph, storage="f32", history=N - A, adjoint_steps=N, ckpt_every=K)
    J32 = s32.forward_ckpt(0, N, A, K)
    g32 = s32.adjoint(1.0)
    say(f"  J64 {J64:.10e} J32 {J32:.10e} g64 {g64} g32 {g32}")
    assert np.abs(g32 - g64).max() <= 1e-3 * np.abs(g64).max()
    assert abs(g32[0] - g64[0]) <= 1e-3 * abs(g64[0]) and abs(g32[1] - g64[1]) <= 1e-3 * abs(g64[1])
    s32.close()
    F0, w0 = cfg["body_force"][2], cfg["omega"]
    for k, (base, setp) in enumerate([(F0, lambda v: s64.set_params(v, w0)), (w0, lambda v: s64.set_params(F0, v))]):
        h = 1e-4 * base
        setp(base + h)
        Jp = s64.forward_ckpt(0, N, A, K)
        setp(base - h)
        Jm = s64.forward_ckpt(0, N, A, K)
        setp(base)
        fd = (Jp - Jm) / (2 * h)
        say(f"  theta{k}: adjoint {g64[k]:.8e} fd {fd:.8e}")
        assert abs(fd - g64[k]) <= 1e-5 * abs(g64[k])
