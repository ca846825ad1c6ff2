"""Writes tests/golden/c5_sphere_dual.json from the oracle alone.

The differentiable-design case on the sphere: icosphere level 3 (1280
panels, 642 vertices), R = 1, V0 = 50 (so |E| > 25 at the surface and the
streamer integral is positive), 128 field lines from area-uniform starts
(seed 6) lifted 1e-6 along the normal, RK4 h = 1e-4, <= 2000 steps,
alpha_eff(E) = 1e-3 max(E - 25, 0)^2, J = sum of the 128 integrals.

Stored: the oracle's forward run (step counts, stop codes, integrals) and
its forward-mode dual derivative of J along 20 single-vertex directions
(workloads.vertex_perturbations, seed 8) and along the body potential.
Only the oracle computes these values; the GPU test compares against them.

    python tests/golden/make_c5_sphere.py      (about 20 minutes on 8 cores)
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from workloads import electrode_line_starts, sphere_problem, vertex_perturbations  # noqa: E402

OUT = os.path.join(HERE, "c5_sphere_dual.json")
LINES, SEED_LINES, SEED_DIRS, N_DIRS = 128, 6, 8, 20
TP = dict(h=1e-4, max_steps=2000, e_min=1e-3, alpha_a=1e-3, alpha_e0=25.0, alpha_p=2.0)


def main():
    p = sphere_problem(3, V0=50.0)
    o = oracle.Oracle(p)
    tp = oracle.trace_params(**TP)
    starts, panel, bary = electrode_line_starts(p, LINES, seed=SEED_LINES)
    A = o.assemble()
    u = np.linalg.solve(A, o.rhs(p.body_V))
    t0 = time.time()
    ns, st, I = o.trace(u[:p.n_tri], starts, tp)
    print(f"forward: J = {I.sum():.15e}, steps {ns.min()}..{ns.max()}, {time.time() - t0:.1f} s", flush=True)
    dirs = []
    gen = vertex_perturbations(p, seed=SEED_DIRS)
    for k in range(N_DIRS):
        v, d = next(gen)
        dv = np.zeros_like(p.vert)
        dv[v] = d
        t0 = time.time()
        Id, dI, _, _, rc = o.dual_streamer(dv, p.body_V, None, panel, bary, tp, ns)
        assert rc == 0
        assert np.max(np.abs(Id - I)) <= 1e-10 * np.max(np.abs(I))
        dirs.append({"vertex": v, "direction": d.tolist(), "dJ": float(dI.sum())})
        print(f"direction {k}: vertex {v} dJ = {dI.sum():.15e} ({time.time() - t0:.1f} s)", flush=True)
    _, dI, _, _, rc = o.dual_streamer(None, p.body_V, np.array([1.0]), panel, bary, tp, ns)
    assert rc == 0
    out = {
        "case": "icosphere level 3, R = 1, V0 = 50, 128 lines (seed 6), RK4 h = 1e-4, <= 2000 steps, "
                "alpha_eff = 1e-3 max(E - 25, 0)^2, J = sum of integrals; directions: vertex_perturbations "
                "(seed 8); values from the oracle's forward-mode dual derivative",
        "trace": TP, "lines": LINES, "seed_lines": SEED_LINES, "seed_dirs": SEED_DIRS,
        "n_steps": ns.tolist(), "stop_code": st.tolist(), "integral": I.tolist(), "J": float(I.sum()),
        "directions": dirs, "dJ_dV0": float(dI.sum()),
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
