"""Writes tests/golden/reference_runs.json: FP64 oracle runs of two reduced
instances of the benchmark workloads, against which the library's storage
formats are measured (drag error, trajectory error).  Calls only the
oracle and the seeded input generators.

  drag128   -- the precision-sweep workload reduced to a 128^3 periodic box
               holding one fixed r = 20 sphere (omega 1.6, body force 1e-5
               along z), 1000 steps from rest; the drag is the raw MEM force
               F_z (Eqs. 11-12) and its mean is taken over steps 800-999.
  rising64  -- the rising-sphere workload reduced to 64 x 64 x 128 cells
               (x, y periodic, no-slip walls at z = 0 and 128), a light
               sphere of density ratio 0.5, r = 8, C_v = 0.5, released at
               rest at height 32 with Ga = 150 (Eq. 13), 1000 steps; the
               sphere's height and vertical velocity after every step
               (Sec. 2.2, Sec. 3.3, Algorithm 1).

Run from the repository root: python tests/golden/make_reference_runs.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402


def drag128():
    cfg = synth.base_config((128, 128, 128), omega=1.6, body_force=(0.0, 0.0, 1e-5))
    sph = [synth.sphere((64.3, 63.8, 64.1), 20.0, fixed=True)]
    o = oracle.Uniform(cfg, sph)
    o.init()
    fz = []
    for n in range(1000):
        o.step(1)
        if n >= 800:
            fz.append(float(o.force_torque(0)[0][2]))
    return {"config": cfg, "spheres": sph, "steps": 1000, "window": [800, 1000], "Fz": fz,
            "Fz_mean": sum(fz) / len(fz)}


def rising64():
    w = synth.rising(n=(64, 64, 128), radius=8.0, height=32.0)
    o = oracle.Uniform(w["config"], w["spheres"])
    o.init()
    z, uz = [], []
    for n in range(1000):
        o.step(1)
        x, u, _ = o.particle(0)
        z.append(float(x[2]))
        uz.append(float(u[2]))
    return {"config": w["config"], "spheres": w["spheres"], "steps": 1000, "z": z, "uz": uz}


def main():
    oracle.build()
    out = {"source": "FP64 CPU oracle (oracle/), tests/golden/make_reference_runs.py"}
    for name, fn in (("drag128", drag128), ("rising64", rising64)):
        t = time.time()
        out[name] = fn()
        print(f"{name}: {time.time() - t:.0f} s", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "reference_runs.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
