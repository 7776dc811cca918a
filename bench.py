"""Benchmark of the coupled LBM hot path on one MI355X.

Headline workload (precision sweep): 512^3 periodic D3Q19 TRT grid, omega 1.6,
body force 1e-5 along z, 8 fixed spheres of radius 20 at seeded positions,
populations stored as FP64, FP32 or FP16 deviations f - w (FP32 collision for
the reduced formats, FP64 forces).  One step = one time step of Algorithm 1:
stream-collide sweep with CLI boundary and momentum-exchange link forces,
per-sphere force/torque reduction and particle update.

For each storage format: W warm-up steps, then K timed steps between HIP
events on the library's stream (MLUPS over all 512^3 cells), then untimed
steps up to 1000 to measure the drag against the library's FP64 run (mean
F_z over steps 800-999, max over spheres).  The drag error against the FP64
oracle is measured on a reduced instance of the same workload (128^3, one
fixed r = 20 sphere, 1000 steps), whose oracle run is stored in
tests/golden/reference_runs.json.  `value` is the MLUPS of the fastest
format whose drag error against the oracle is below 1e-3.

Also reported: the roofline of the interior sweep kernel (algorithmic bytes
per launch / event-timed launch duration vs 8 TB/s), the moving-sphere
workload (256^3 throughput; trajectory error of each format against the
stored oracle run of a reduced 64 x 64 x 128 instance), the refined
workload with its roofline (all levels' cell updates x bytes per update per
coarse step), the adjoint cost, and the CPU oracle timed on a bounded
sample on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS & %HBM roofline, FP16/FP32-store vs FP64 at drag err<1e-3; adjoint cost"
PEAK_GBS = 8000.0
BYTES = {"f64": 8, "f32": 4, "f16": 2}
# sources of the interior sweep kernel; the HBM counter figures in
# TRAFFIC_FILE hold for the build whose sources hash to its source_sha256
SWEEP_SOURCES = ["paper_2103_10882_amd/csrc/common.hpp", "paper_2103_10882_amd/csrc/stencil.hpp",
                 "paper_2103_10882_amd/csrc/uniform.hpp", "paper_2103_10882_amd/csrc/uniform.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_traffic_precision512.md")
GOLDEN_FILE = os.path.join(ROOT, "tests", "golden", "reference_runs.json")
COPY_BYTES = 1 << 30


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def timed_steps(sim, steps):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(sim.stream)
    sim.step(steps)
    e1.record(sim.stream)
    sim.sync()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e-3


def run_precision(pkg, w, storage, warmup, steps, drag_steps, drag_window):
    import torch
    cfg, sph = w["config"], w["spheres"]
    N = cfg["n"][0] * cfg["n"][1] * cfg["n"][2]
    sim = pkg.Sim(cfg, sph, storage=storage, history=drag_window)
    sim.init()
    sim.step(warmup)
    sim.sync()
    sim.profile(True)
    t = timed_steps(sim, steps)
    sweep_s, launches = sim.sweep_time()
    sim.profile(False)
    fluid, interior = sim.cell_counts()
    rest = drag_steps - warmup - steps
    if rest > 0:
        sim.step(rest)
        sim.sync()
    drag = [float(sim.history(i, drag_window)[:, 2].mean()) for i in range(len(sph))]
    sim.close()
    del sim
    torch.cuda.empty_cache()
    avg = sweep_s / max(launches, 1)
    alg_bytes = interior * (38 * BYTES[storage] + 1)      # 19 loads + 19 stores + flag byte
    return {
        "mlups": N * steps / t / 1e6,
        "mlups_fluid": fluid * steps / t / 1e6,
        "ms_per_step": 1e3 * t / steps,
        "sweep_ms": 1e3 * avg,
        "sweep_launches": launches,
        "sweep_bytes": alg_bytes,
        "sweep_gbs": alg_bytes / avg / 1e9,
        "drag": drag,
        "cells": N,
        "fluid_cells": fluid,
        "interior_cells": interior,
    }


def run_mrt(pkg, w, storages, warmup, steps, bulk_factor=100.0):
    """The headline workload with the paper's default collision: MRT with
    bulk factor 100 (Sec. 2.1).  Throughput only."""
    w2 = dict(w, config=dict(w["config"], bulk_factor=bulk_factor))
    out = {"bulk_factor": bulk_factor}
    for st in storages:
        r = run_precision(pkg, w2, st, warmup, steps, warmup + steps, 1)
        out[st] = {"mlups": round(r["mlups"], 1), "sweep_gbs": round(r["sweep_gbs"], 1),
                   "hbm_frac": round(r["sweep_gbs"] / PEAK_GBS, 4)}
    return out


def golden():
    with open(GOLDEN_FILE) as f:
        return json.load(f)


def drag_vs_oracle(pkg, storages):
    """Drag error of each storage format against the stored FP64 oracle run
    of the reduced precision-sweep instance (128^3, one fixed r = 20 sphere,
    1000 steps): |<F_z> - <F_z>_oracle| / |<F_z>_oracle| over steps 800-999."""
    g = golden()["drag128"]
    lo, hi = g["window"]
    out = {"workload": "128^3 periodic, one fixed r=20 sphere, omega 1.6, F 1e-5 z; mean F_z over steps %d-%d" %
           (lo, hi - 1), "oracle_fz_mean": g["Fz_mean"]}
    for st in storages:
        sim = pkg.Sim(g["config"], g["spheres"], storage=st, history=hi - lo)
        sim.init()
        sim.step(g["steps"])
        sim.sync()
        fz = float(sim.history(0, hi - lo)[:, 2].mean())
        sim.close()
        out[st] = {"fz_mean": fz, "drag_err": abs(fz - g["Fz_mean"]) / abs(g["Fz_mean"])}
    return out


def trajectory_vs_oracle(pkg, storages):
    """Trajectory error of each storage format against the stored FP64
    oracle run of the reduced rising-sphere instance (64 x 64 x 128 between
    walls, r = 8, density ratio 0.5, C_v 0.5, Ga 150, 1000 steps): the
    error measures of Sec. 3.4.1 on u_z,n = u_z / u_g sampled every step."""
    import numpy as np
    g = golden()["rising64"]
    n = g["steps"]
    uo = np.array(g["uz"]) / 0.01
    out = {"workload": "64x64x128, walls at z=0,128; r=8, density ratio 0.5, C_v 0.5, Ga 150; %d steps" % n}
    for st in storages:
        sim = pkg.Sim(g["config"], g["spheres"], storage=st, history=n)
        sim.init()
        sim.step(n)
        sim.sync()
        h = sim.history(0, n)
        sim.close()
        ug = h[:, 11] / 0.01
        out[st] = {"eps_sq": float(np.mean((ug - uo) ** 2)),
                   "eps_rel": float(np.mean((ug[uo != 0] - uo[uo != 0]) / uo[uo != 0])),
                   "eps_term_rel": float((ug[-1] - uo[-1]) / uo[-1]),
                   "z_err": float(np.abs(h[:, 8] - np.array(g["z"])).max())}
    return out


def run_rising(pkg, steps):
    """Moving light sphere between walls at full size: throughput of FP64
    and FP32 (their trajectory errors are measured against the oracle on
    the reduced instance, trajectory_vs_oracle)."""
    import numpy as np
    import synth
    w = synth.rising()
    out = {}
    for st in ("f64", "f32"):
        sim = pkg.Sim(w["config"], w["spheres"], storage=st, history=steps)
        sim.init()
        t = timed_steps(sim, steps)
        N = np.prod(w["config"]["n"])
        out[st] = {"mlups": float(N * steps / t / 1e6)}
        if st == "f64":
            out["uz_n_final_f64"] = float(sim.history(0, 1)[0, 11] / 0.01)
        sim.close()
        del sim
    out["steps"] = steps
    return out


def run_refined(pkg, coarse_steps=500):
    """Adaptive refinement workload: coarse 128x128x512, 3 levels (16^3
    blocks), light sphere r=16 finest cells (density ratio 0.1, C_v 0.5,
    Ga 250) rising from rest; layout checked every 4 coarse steps.  MLUPS
    counts cell updates of all levels (2^l per coarse step on level l)."""
    import torch
    import synth
    w = synth.refined()
    out = {}
    for st in ("f64", "f32", "f16"):
        sim = pkg.Sim(w["config"], w["spheres"], storage=st, history=4 * coarse_steps)
        sim.init()
        blocks = [int(sim.level_blocks(l).shape[0]) for l in range(3)]
        sim.step(2)
        sim.sync()
        cu0, _ = sim.stats()
        t = timed_steps(sim, coarse_steps)
        cu1, _ = sim.stats()
        h = sim.history(0, 4 * coarse_steps)
        upd = (cu1 - cu0) / coarse_steps
        # all levels' cell updates per coarse step (sum_l 2^l N_l) x bytes per
        # update (19 loads, 19 stores, the flag byte)
        gbs = upd * (38 * BYTES[st] + 1) / (t / coarse_steps) / 1e9
        out[st] = {"mlups": (cu1 - cu0) / t / 1e6, "ms_per_coarse_step": 1e3 * t / coarse_steps,
                   "cell_updates_per_coarse_step": upd, "blocks_at_start": blocks,
                   "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_GBS, "unit": "GB/s",
                                "frac": round(gbs / PEAK_GBS, 4),
                                "bytes_per_coarse_step": upd * (38 * BYTES[st] + 1)},
                   "refinements": sim.refinements(), "prebuilt_layouts": sim.prebuilt_layouts(),
                   "z_rise": float(h[-1, 8] - w["spheres"][0]["x"][2]),
                   "uz_final": float(h[-1, 11])}
        # the coarse level's access pattern without arithmetic (vmlbm_level_pull:
        # 19 pulls and 19 streaming stores per leaf cell), after the run
        nb0 = int(sim.level_blocks(0).shape[0])
        sim.level_pull(0, 2)
        sim.sync()
        reps = 50
        t0 = time.perf_counter()
        sim.level_pull(0, reps)
        sim.sync()
        tp = (time.perf_counter() - t0) / reps
        out[st]["coarse_level_pull"] = {"blocks": nb0, "us": round(1e6 * tp, 1),
                                        "gbs": round(nb0 * 4096 * 38 * BYTES[st] / tp / 1e9, 1)}
        sim.close()
        del sim
        torch.cuda.empty_cache()
    out["coarse_steps"] = coarse_steps
    # rise of the reduced formats against FP64 over the run
    for st in ("f32", "f16"):
        out[st]["z_rise_rel_err"] = abs(out[st]["z_rise"] - out["f64"]["z_rise"]) / abs(out["f64"]["z_rise"])
    return out


def run_adjoint(pkg, storage="f32"):
    """Drag gradient on a fixed sphere (128^3, r=10, 2000 steps, window
    1500..1999, checkpoints every 50): forward-with-checkpoints time vs
    reverse time (segment recomputation + adjoint sweeps)."""
    import torch
    import synth
    w = synth.adjoint()
    N, A, K = w["steps"], w["avg_from"], w["ckpt_every"]
    sim = pkg.Sim(w["config"], w["spheres"], storage=storage, history=N - A, adjoint_steps=N, ckpt_every=K)
    sim.forward_ckpt(0, N, A, K)          # warm-up
    sim.adjoint(1.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = sim.forward_ckpt(0, N, A, K)
    t1 = time.perf_counter()
    g = sim.adjoint(1.0)
    t2 = time.perf_counter()
    sim.close()
    return {"storage": storage, "steps": N, "J": J, "dJ_dF": float(g[0]), "dJ_domega": float(g[1]),
            "forward_s": t1 - t0, "reverse_s": t2 - t1, "cost_ratio": (t2 - t1) / (t1 - t0)}


# ---------------------------------------------------------------------------
# validation workloads of Sec. 3 (run with --validate; not part of the
# headline line).  The paper's printed figures are kept here as context.
# ---------------------------------------------------------------------------
PAPER_TABLE1_PI_MIN = {10: 0.13, 15: 0.09, 20: 0.066, 30: 0.045, 40: 0.034, 50: 0.03, 80: 0.02}   # Table 1, Ga 100
PAPER_TABLE2 = {   # Sec. 3.4.1, Table 2: VM-MEM (C_v = 1) against MEM, d_p = 40
    0.1: {"ga": 100.0, "re_p": 113.08, "eps_sq": 15.48e-9, "eps_rel": 0.28e-3, "eps_term_rel": 0.04e-3},
    1.1: {"ga": 100.0, "re_p": 111.77, "eps_sq": 1.85e-9, "eps_rel": 0.15e-3, "eps_term_rel": 0.06e-3},
    0.001: {"ga": 170.0, "re_p": 225.64},
}
PAPER_ROTATION = {0.1: {"eps_rel": 0.46e-3, "eps_term_rel": 0.01e-3},   # Sec. 3.4.2, VM-MEM vs MEM
                  1.1: {"eps_rel": 0.15e-3, "eps_term_rel": 0.0}}


def _run_chunks(pkg, sim, steps, chunk, speed_limit, tag):
    """Step in chunks; a run is unstable once the library flags a non-finite
    or runaway state, or the sphere's speed passes speed_limit.  Returns
    (status, steps done)."""
    import numpy as np
    done = 0
    while done < steps:
        k = min(chunk, steps - done)
        sim.step(k)
        try:
            sim.sync()
        except pkg.VmlbmError as e:
            log(f"  {tag}: unstable at step <= {done + k} ({e})")
            return "unstable", done
        done += k
        _, u, w = sim.particle(0)
        if not (np.all(np.isfinite(u)) and np.all(np.isfinite(w))) or max(np.abs(u).max(), 0.0) > speed_limit:
            log(f"  {tag}: unstable at step {done} (u = {u})")
            return "unstable", done
        log(f"  {tag}: step {done}/{steps}, u = {u[2]:.5f}, w = {w[1]:.3e}")
    return "stable", done


def run_light_sphere(pkg, d_p, pi_p, ga=100.0, cv=0.0, t_n=10.0, storage="f64", compensate=False, vm_scheme=0):
    """One rising/settling sphere run of Sec. 3.1 / 3.4.1 up to t_n = t u_g / d_p."""
    import numpy as np
    import torch
    import synth
    w = synth.light_box(d_p, pi_p, ga=ga, cv=cv, compensate=compensate, vm_scheme=vm_scheme)
    steps = int(round(t_n * w["t_g"]))
    tag = w["name"]
    sim = pkg.Sim(w["config"], w["spheres"], storage=storage, history=steps)
    sim.init()
    t0 = time.time()
    status, done = _run_chunks(pkg, sim, steps, max(500, steps // 20), 10.0 * synth.U_G, tag)
    h = sim.history(0, done) if done > 0 else np.zeros((0, 15))
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return {"status": status, "steps": done, "of": steps, "seconds": time.time() - t0,
            "uz_n": h[:, 11] / synth.U_G, "nu": w["nu"], "t_g": w["t_g"]}


def _errors(u, ref, every):
    """Mean squared and mean relative error and the terminal relative error
    of a series against a reference (Sec. 3.4.1), sampled every `every`
    steps from the first sample on."""
    import numpy as np
    a = np.abs(u[every - 1::every])
    b = np.abs(ref[every - 1::every])
    return {"m": int(len(a)), "eps_sq": float(np.mean((a - b) ** 2)), "eps_rel": float(np.mean((a - b) / b)),
            "eps_term_rel": float((a[-1] - b[-1]) / b[-1])}


def validate_stability(pkg, diameters=(10, 15, 20, 30), storage="f64", bisections=4, factors=None):
    """Table 1: lowest density ratio at Ga 100 for which plain MEM stays
    stable up to t_n = 10, bracketed by bisection in log(pi_p) from the
    paper's value x {1/2, 2}; VM-MEM (C_v = 1) run at the unstable end.
    With factors, MEM runs only at those multiples of the paper's value
    (VM-MEM at the smallest), for diameters where a bisection costs too
    much."""
    import math
    out = {}
    for d in diameters:
        ref = PAPER_TABLE1_PI_MIN[d]
        runs = {}

        def stable(pi_p, cv=0.0):
            r = run_light_sphere(pkg, d, pi_p, cv=cv, storage=storage)
            runs["%.5g cv%g" % (pi_p, cv)] = {"status": r["status"], "steps": r["steps"], "of": r["of"]}
            return r["status"] == "stable"

        if factors:
            for fct in sorted(factors, reverse=True):
                stable(fct * ref)
            out[d] = {"paper": ref, "vm_mem_stable_at_smallest": stable(min(factors) * ref, cv=1.0), "runs": runs}
            continue

        lo, hi = 0.5 * ref, 2.0 * ref
        if not stable(hi):
            hi *= 2.0
            stable(hi)
        if stable(lo):
            out[d] = {"paper": ref, "pi_min_at_most": lo, "runs": runs}
            continue
        for _ in range(bisections):
            mid = math.exp(0.5 * (math.log(lo) + math.log(hi)))
            if stable(mid):
                hi = mid
            else:
                lo = mid
        vm_ok = stable(lo, cv=1.0)
        out[d] = {"paper": ref, "pi_min_bracket": [round(lo, 5), round(hi, 5)], "vm_mem_stable_at_lo": vm_ok,
                  "runs": runs}
    return out


def validate_extrapolation(pkg, d_p=40, storage="f64", schemes=(1, 2), densities=(0.1, 1.1)):
    """VM-MEM (C_v = 1) with the acceleration from three velocities
    (schemes 1 and 2) in the Table 2 cases, against MEM."""
    out = {}
    for pi_p in densities:
        ga = PAPER_TABLE2[pi_p]["ga"]
        mem = run_light_sphere(pkg, d_p, pi_p, ga=ga, cv=0.0, storage=storage)
        for sc in schemes:
            lag = run_light_sphere(pkg, d_p, pi_p, ga=ga, cv=1.0, storage=storage, vm_scheme=sc)
            r = {"status_mem": mem["status"], "status_vm": lag["status"], "steps_vm": lag["steps"]}
            if mem["status"] == lag["status"] == "stable":
                r.update(_errors(lag["uz_n"], mem["uz_n"], 100))
                r["re_p_vm"] = float(abs(lag["uz_n"][-1]) * 0.01 * d_p / lag["nu"])
            out["%g scheme %d" % (pi_p, sc)] = r
    return out


def validate_translation(pkg, d_p=40, storage="f64", compensated=False):
    """Table 2: VM-MEM (C_v = 1) against MEM for pi_p = 0.1 and 1.1 at Ga 100,
    and VM-MEM alone at pi_p = 0.001, Ga 170 (MEM is expected to fail).
    compensated: also MEM with a fluid force cancelling the net weight
    (Re_p only), the other reading of the setup."""
    out = {}
    for pi_p in (0.1, 1.1):
        ga = PAPER_TABLE2[pi_p]["ga"]
        mem = run_light_sphere(pkg, d_p, pi_p, ga=ga, cv=0.0, storage=storage)
        vm = run_light_sphere(pkg, d_p, pi_p, ga=ga, cv=1.0, storage=storage)
        r = {"status_mem": mem["status"], "status_vm": vm["status"], "paper": PAPER_TABLE2[pi_p]}
        if mem["status"] == vm["status"] == "stable":
            r.update(_errors(vm["uz_n"], mem["uz_n"], 100))
            for k, run in (("mem", mem), ("vm", vm)):
                r["re_p_" + k] = float(abs(run["uz_n"][-1]) * 0.01 * d_p / run["nu"])
        if compensated:
            cm = run_light_sphere(pkg, d_p, pi_p, ga=ga, cv=0.0, storage=storage, compensate=True)
            if cm["status"] == "stable":
                r["re_p_mem_compensated"] = float(abs(cm["uz_n"][-1]) * 0.01 * d_p / cm["nu"])
        out[pi_p] = r
    vm = run_light_sphere(pkg, d_p, 0.001, ga=170.0, cv=1.0, storage=storage)
    mem = run_light_sphere(pkg, d_p, 0.001, ga=170.0, cv=0.0, storage=storage)
    r = {"status_vm": vm["status"], "status_mem": mem["status"], "steps_mem": mem["steps"],
         "paper": PAPER_TABLE2[0.001]}
    if vm["status"] == "stable":
        r["re_p_vm"] = float(abs(vm["uz_n"][-1]) * 0.01 * d_p / vm["nu"])
    out[0.001] = r
    return out


def run_rotation(pkg, d_p, pi_p, cv, hold_tc=20.0, free_tc=20.0, storage="f64"):
    """Sec. 3.4.2: Couette-driven sphere held for hold_tc t_c, then free to
    rotate (position held) for free_tc t_c; omega_n = omega_y / omega_c."""
    import numpy as np
    import torch
    import synth
    w = synth.rotation_box(d_p, pi_p, cv=cv)
    hold = int(round(hold_tc * w["t_c"]))
    free = int(round(free_tc * w["t_c"]))
    tag = w["name"]
    sim = pkg.Sim(w["config"], w["spheres"], storage=storage, history=free)
    sim.init(1.0, w["u0"])
    t0 = time.time()
    status, done = _run_chunks(pkg, sim, hold, 2000, 1.0, tag + " held")
    fdone = 0
    if status == "stable":
        sim.set_sphere_motion(0, fixed=2)
        status, fdone = _run_chunks(pkg, sim, free, 2000, 1.0, tag + " rotating")
    h = sim.history(0, fdone) if fdone > 0 else np.zeros((0, 15))
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return {"status": status, "steps_free": fdone, "of": free, "seconds": time.time() - t0,
            "omega_n": h[:, 13] / w["omega_c"], "t_c": w["t_c"]}


def validate_rotation(pkg, d_p=40, storage="f64"):
    """Sec. 3.4.2 table: VM-MEM (C_v = C_v,omega = 1) against MEM for pi_p =
    0.1 and 1.1, and both at pi_p = 0.001."""
    out = {}
    for pi_p in (0.1, 1.1, 0.001):
        mem = run_rotation(pkg, d_p, pi_p, 0.0, storage=storage)
        vm = run_rotation(pkg, d_p, pi_p, 1.0, storage=storage)
        r = {"status_mem": mem["status"], "status_vm": vm["status"], "paper": PAPER_ROTATION.get(pi_p)}
        if mem["status"] == vm["status"] == "stable":
            r.update(_errors(vm["omega_n"], mem["omega_n"], 80))
        for k, run in (("mem", mem), ("vm", vm)):
            if run["status"] == "stable":
                r["omega_n_term_" + k] = float(run["omega_n"][-1])
        out[pi_p] = r
    return out


def run_amr(pkg, refined, t_n, storage="f64", curl_threshold=0.0, check_every=4, ga=300.0):
    """The rising sphere of Sec. 4.3 (d_p = 25, density ratio 0.5, MEM) on
    the uniform finest grid or on 3 refined levels, up to t_n."""
    import numpy as np
    import torch
    import synth
    w = synth.amr_box(refined=refined, curl_threshold=curl_threshold, ga=ga)
    steps = int(round(t_n * w["t_g"]))                      # finest-level steps
    per = 4 if refined else 1                               # finest steps per call unit
    tag = w["name"] + (" curl" if curl_threshold > 0 else "")
    sim = pkg.Sim(w["config"], w["spheres"], storage=storage, history=steps, check_every=check_every)
    sim.init()
    sim.sync()
    cu0, _ = sim.stats()
    torch.cuda.synchronize()
    t0 = time.time()
    done, status = 0, "stable"
    chunk = 2000
    while done < steps:
        k = min(chunk, steps - done)
        sim.step(k // per)
        try:
            sim.sync()
        except pkg.VmlbmError as e:
            status = "failed: %s" % e
            log(f"  {tag}: {status}")
            break
        done += k
        x, u, _ = sim.particle(0)
        extra = (" blocks " + str([int(sim.level_blocks(l).shape[0]) for l in range(3)])) if refined else ""
        log(f"  {tag}: step {done}/{steps}, z = {x[2]:.2f}, u = {u}{extra}")
    wall = time.time() - t0
    cu1, _ = sim.stats()
    h = sim.history(0, done) if done else np.zeros((0, 15))
    out = {"status": status, "steps": done, "seconds": wall, "cell_updates": cu1 - cu0,
           "refinements": sim.refinements() if refined else 0, "hist": h, "d_p": 25.0,
           "x0": np.array(w["spheres"][0]["x"])}
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def validate_amr(pkg, t_n=12.0, storage="f64", curl_threshold=0.0, ga=300.0):
    """Sec. 4.3: trajectory on 3 refined levels against the uniform finest
    grid; u_z,n compared every 100 finest steps from t_n = 0.5 on."""
    import numpy as np
    import synth
    uni = run_amr(pkg, False, t_n, storage, ga=ga)
    ref = run_amr(pkg, True, t_n, storage, curl_threshold=curl_threshold, ga=ga)
    out = {"t_n": t_n, "ga": ga, "storage": storage, "curl_threshold": curl_threshold,
           "status": [uni["status"], ref["status"]]}
    m = min(len(uni["hist"]), len(ref["hist"]))
    out["steps"] = [uni["steps"], ref["steps"]]
    if m < 400:
        return out
    d = uni["d_p"]
    ug = synth.U_G
    s = slice(int(0.5 * d / ug) - 1, m, 100)
    uu, ur = uni["hist"][s, 11] / ug, ref["hist"][s, 11] / ug
    lat = {}
    for k, r in (("uniform", uni), ("refined", ref)):
        dx = r["hist"][:m, 6:8] - r["x0"][None, :2]
        lat[k] = float(np.sqrt((dx ** 2).sum(axis=1)).max() / d)
    out.update({
        "samples": int(len(uu)),
        "uz_n_mean_rel_err": float(np.mean(np.abs(ur - uu) / np.abs(uu))),
        "uz_n_max_abs_diff": float(np.abs(ur - uu).max()),
        "uz_n_end": [float(uu[-1]), float(ur[-1])],
        "z_n_end": [float(uni["hist"][m - 1, 8] / d), float(ref["hist"][m - 1, 8] / d)],
        "max_lateral_displacement_n": [lat["uniform"], lat["refined"]],
        "cell_updates": [uni["cell_updates"], ref["cell_updates"]],
        "seconds": [round(uni["seconds"], 1), round(ref["seconds"], 1)],
        "refinements": ref["refinements"],
    })
    return out


def sweep_source_hash():
    import hashlib
    h = hashlib.sha256()
    for p in SWEEP_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(storage):
    """HBM bytes per launch of the interior sweep from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE per dispatch, each scaled by what the
    counter reads for a plain copy of known size), or None if there is none
    for this storage or the kernel sources changed since it was taken."""
    try:
        text = open(TRAFFIC_FILE).read()
        blob = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if blob.get("source_sha256") != sweep_source_hash() or storage not in blob.get("kernels", {}):
        return None
    k = blob["kernels"][storage]
    return k["fetch_kib"] * 1024 * blob["fetch_scale"] + k["write_kib"] * 1024 * blob["write_scale"]


def copy_reference():
    """The library's plain device copy of COPY_BYTES, five times: the
    reference whose FETCH_SIZE / WRITE_SIZE readings scale the sweep's
    counters."""
    import torch
    import paper_2103_10882_amd as pkg
    n = COPY_BYTES // 4
    x = torch.ones(n, device="cuda", dtype=torch.float32)
    y = torch.empty_like(x)
    for _ in range(5):
        pkg.stream_copy(y, x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": COPY_BYTES, "copies": 5}), flush=True)


def stream_reference(nbytes=4 << 30, reps=10):
    """Streaming rates on this GPU, GB/s of bytes moved: the library's plain
    16-byte-per-lane copy (vmlbm_stream_copy), and PyTorch's read (sum) and
    write (fill) of nbytes.  A 1:1 read/write stream such as the interior
    sweep is bounded by the copy figure."""
    import torch
    import paper_2103_10882_amd as pkg
    n = nbytes // 4
    x = torch.ones(n, device="cuda", dtype=torch.float32)
    y = torch.empty_like(x)
    out = {}
    for name, fn, moved in (("read", lambda: x.sum(), nbytes), ("write", lambda: y.fill_(1.5), nbytes),
                            ("copy", lambda: pkg.stream_copy(y, x), 2 * nbytes)):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[name + "_gbs"] = round(moved * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    del x, y
    torch.cuda.empty_cache()
    return out


def pull_reference(n, storages, reps=5):
    """GB/s of the interior sweep's access pattern without its arithmetic
    (vmlbm_stream_pull: 19 pulled loads and 19 streaming stores per cell of
    a periodic n^3 box), per storage format: the rate a sweep with no
    arithmetic and no flags would reach."""
    import torch
    import paper_2103_10882_amd as pkg
    out = {}
    for st in storages:
        dt = {"f64": torch.float64, "f32": torch.float32, "f16": torch.float16}[st]
        cells = n ** 3
        x = torch.zeros(19 * cells, device="cuda", dtype=dt)
        y = torch.empty_like(x)
        pkg.stream_pull(y, x, (n, n, n), st)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            pkg.stream_pull(y, x, (n, n, n), st)
        e1.record()
        torch.cuda.synchronize()
        out[st] = round(2 * 19 * cells * x.element_size() * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
        del x, y
        torch.cuda.empty_cache()
    return out


def cpu_baseline(n=512, target_s=12.0):
    """The oracle on a bounded sample of the headline workload itself: the
    n^3 box with its eight fixed r=20 spheres (omega 1.6, body force 1e-5
    along z), one untimed step, then timed steps until about target_s
    seconds have passed (set-up excluded).  At 512^3 the oracle holds three
    FP64 population arrays, about 61 GB of host memory."""
    import oracle
    import synth
    oracle.build()
    w = synth.precision(n=n)
    o = oracle.Uniform(w["config"], w["spheres"])
    o.init()
    o.step(1)
    t0 = time.perf_counter()
    k = 0
    while True:
        o.step(1)
        k += 1
        if time.perf_counter() - t0 > target_s and k >= 2:
            break
    t = time.perf_counter() - t0
    del o
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": n ** 3 * k / t / 1e6, "unit": "MLUPS", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"the headline workload itself ({n}^3, eight fixed r=20 spheres, omega 1.6, F=1e-5 z), "
                      f"{k} steps after one untimed step, {t:.1f} s", "cpu": model}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--drag-steps", type=int, default=1000)
    ap.add_argument("--storages", default="f64,f32,f16")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--copy-ref", action="store_true",
                    help="only run the plain copy used to scale HBM byte counters")
    ap.add_argument("--validate", default="",
                    help="only run validation workloads of Sec. 3 and 4.3: any of stability,translation,"
                         "rotation,extrapolation,amr")
    ap.add_argument("--validate-diameters", default="10,15,20,30",
                    help="sphere diameters of the stability bracket (Table 1)")
    ap.add_argument("--validate-factors", default="",
                    help="stability: run only these multiples of the paper's lowest density ratio")
    ap.add_argument("--validate-schemes", default="1,2", help="extrapolation: virtual-force schemes to run")
    ap.add_argument("--validate-tn", type=float, default=12.0, help="amr: run length in t_n = t u_g / d_p")
    ap.add_argument("--validate-curl", type=float, default=0.0, help="amr: curl-sensor threshold (0 = particle only)")
    ap.add_argument("--validate-ga", type=float, default=150.0, help="amr: Galileo number (the paper's 300 needs "
                    "more than 25 cells per diameter)")
    ap.add_argument("--validate-densities", default="0.1,1.1", help="extrapolation: density ratios to run")
    ap.add_argument("--validate-compensated", action="store_true",
                    help="translation: also run MEM with a fluid force that cancels the net weight")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (no halo exchange, "
              "all-reduce or load balancing across GPUs)", file=sys.stderr)
        sys.exit(2)

    import torch
    torch.cuda.set_device(0)
    if args.copy_ref:
        copy_reference()
        return
    if args.validate:
        import paper_2103_10882_amd as pkg
        pkg.lib()
        runs = {"stability": lambda: validate_stability(
                    pkg, tuple(int(v) for v in args.validate_diameters.split(",")),
                    factors=tuple(float(v) for v in args.validate_factors.split(",")) if args.validate_factors else None),
                "translation": lambda: validate_translation(pkg, compensated=args.validate_compensated),
                "rotation": lambda: validate_rotation(pkg),
                "amr": lambda: validate_amr(pkg, t_n=args.validate_tn, curl_threshold=args.validate_curl,
                                            ga=args.validate_ga),
                "extrapolation": lambda: validate_extrapolation(
                    pkg, schemes=tuple(int(v) for v in args.validate_schemes.split(",")),
                    densities=tuple(float(v) for v in args.validate_densities.split(",")))}
        for name in args.validate.split(","):
            log(f"validation: {name}")
            print(json.dumps({"validation": name, "result": runs[name]()}, default=str), flush=True)
        return
    import synth
    import paper_2103_10882_amd as pkg
    pkg.lib()
    log("stream reference")
    sref = stream_reference()
    log(f"  {sref}")
    pref = pull_reference(args.n, args.storages.split(","))
    log(f"  sweep access pattern without arithmetic: {pref}")
    w = synth.precision(n=args.n)
    drag_window = 200
    drag_steps = max(args.drag_steps, args.warmup + args.steps + drag_window)
    res = {}
    for st in args.storages.split(","):
        log(f"precision sweep: {st}")
        res[st] = run_precision(pkg, w, st, args.warmup, args.steps, drag_steps, drag_window)
        log(f"  {res[st]['mlups']:.0f} MLUPS, sweep {res[st]['sweep_ms']:.3f} ms, {res[st]['sweep_gbs']:.0f} GB/s")
    ref = res.get("f64")
    for st, r in res.items():
        r["drag_err_vs_fp64"] = None if ref is None else max(abs(a - b) / abs(b) for a, b in zip(r["drag"], ref["drag"]))
    log("drag against the stored FP64 oracle run (128^3)")
    dvo = drag_vs_oracle(pkg, list(res))
    ok = [st for st in res if dvo[st]["drag_err"] < 1e-3]
    best = max(ok, key=lambda s: res[s]["mlups"]) if ok else max(res, key=lambda s: res[s]["mlups"])
    b = res[best]
    traffic = measured_traffic(best) if args.n == 512 else None
    line = {
        "metric": METRIC,
        "value": round(b["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(b["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if best == "f64" else "f32",
        "data": "synthetic",
        "config": {
            "workload": f"precision sweep: {args.n}^3 periodic D3Q19 TRT (omega 1.6, Lambda 3/16), 8 fixed "
                        f"spheres r=20 at seeded positions, body force 1e-5 z; CLI + MEM coupling",
            "storage": best,
            "storage_meets_drag_bar": best in ok,
            "cells": b["cells"],
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": f"interior stream-collide sweep ({best} storage)",
            "achieved": round(b["sweep_gbs"], 1),
            "peak": PEAK_GBS,
            "unit": "GB/s",
            "frac": round(b["sweep_gbs"] / PEAK_GBS, 4),
            "traffic": None if traffic is None else round(traffic),
            "traffic_over_algorithmic": None if traffic is None else round(traffic / b["sweep_bytes"], 3),
            "stream_reference_gbs": sref,
            "frac_of_copy": round(b["sweep_gbs"] / sref["copy_gbs"], 3),
            "pull_pattern_gbs": pref,
            "frac_of_pull_pattern": round(b["sweep_gbs"] / pref[best], 3),
            "bytes_per_launch": b["sweep_bytes"],
            "launch_ms": round(b["sweep_ms"], 4),
        },
        "precision_sweep": {st: {"mlups": round(r["mlups"], 1), "mlups_fluid": round(r["mlups_fluid"], 1),
                                 "sweep_gbs": round(r["sweep_gbs"], 1),
                                 "hbm_frac": round(r["sweep_gbs"] / PEAK_GBS, 4),
                                 "drag_err_vs_oracle": dvo[st]["drag_err"],
                                 "drag_err_vs_fp64_512": r["drag_err_vs_fp64"], "drag_fz_mean": r["drag"][0]}
                            for st, r in res.items()},
        "drag_vs_oracle": dvo,
    }
    if not args.no_extra:
        log("MRT, bulk factor 100, on the precision workload")
        line["mrt_bulk100"] = run_mrt(pkg, w, ["f32", "f16"], args.warmup, args.steps)
        log("rising sphere 256^3")
        line["rising"] = run_rising(pkg, 2000)
        log("trajectories against the stored FP64 oracle run (64x64x128)")
        line["trajectory_vs_oracle"] = trajectory_vs_oracle(pkg, ["f64", "f32", "f16"])
        log("refined 128x128x512, 3 levels")
        line["refined"] = run_refined(pkg)
        log("adjoint 128^3")
        line["adjoint"] = run_adjoint(pkg)
        line["adjoint_cost"] = round(line["adjoint"]["cost_ratio"], 3)
    if not args.no_cpu:
        log("cpu baseline")
        line["cpu_baseline"] = cpu_baseline(args.n)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
