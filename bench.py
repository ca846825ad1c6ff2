"""Benchmark of the whole BEM hot path on one MI355X.

One step = the paper's pipeline on the coaxial rod-in-shell device with a
floating ring and a dielectric spacer (19,732 flat panels + 1 floating
potential): FP64 assembly of the collocation matrix, GMRES to 1e-10,
the electric field at every panel centroid (exterior limit, "E surface"),
and 256 field lines (RK4, h = 1e-4, <= 2000 steps) with the streamer
integral, all from inputs already resident in GPU memory.

Prints one JSON line.  value = panel-pair evaluations per second over the
whole step (matrix entries + surface-field pairs + field-line pairs).
The roofline entry is for the dominant kernel, the far-field pass of the
field-line tracer (k_lb_far, one launch per RK4 stage of the live lines of a
line group): algorithmic FP64 flops per launch (regular pairs x 141 flop) / its
average duration over every launch of a repeat of the timed steps, each launch
timed by the kernel itself (profiling mode 2: the earliest block start to the
latest wave end on the device's wall clock; nothing else is timed).  Events
carried in the dispatch would also count the wait for the other line group's
kernel on the second stream (2.2 us a launch more than rocprofv3 measured on
the same box).  The timed steps themselves run with nothing profiled.
phase_ms_per_step (and trace_ms_per_step) come from three more unprofiled steps,
the host clock read after each call (assemble, solve, eval_field,
streamer_integral) has finished; kernel_ms_profiled_step from one more step
with every kernel timed by events (which slow the two-stream tracer, so its
"trace" entry exceeds the unprofiled one).  cpu_baseline times
the plain FP64 CPU oracle, compiled on the host with -march=native, on a
bounded sample of the same workload.  The 64-load-case time-to-solve stops
each path at the loosest tolerance that brings sigma within 1e-5 of the
reference.

After the timed steps, "extras" reports runs outside the step:
- the gradient of 128 lines;
- 64 load cases x 64 lines;
- the 57,230-panel coax in FP64 and mixed precision;
- the bushing with thin sheets;
- the paper's nodal basis: spheres against the constant basis, and the coaxial
  conductors at 67,729 vertices (FP64 and MIXED, with 256 field lines) and at
  233,519 vertices (MIXED).
--extras-only and --nodal-only run those without the timed steps.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# algorithmic work per (point, panel) pair in flops (FMA = 2, rsqrt = 1):
#   classification 9; per node: 3 sub, r^2 5, rsqrt 1, w r^-3 3, F += t d 6  (18 x 7 = 126);
#   sigma_j * F accumulation 6  -> field-only pair 141
#   potential-only pair (assembly of S rows): 9 + 7 x (3 + 5 + 1 + 2) = 86
FLOP_FIELD_PAIR = 141
# HBM traffic of one k_lb_far launch (this workload, FP64, the autotuned 4-wave chunk split, two line
# groups of up to 128 lines): rocprofv3 FETCH_SIZE and WRITE_SIZE per dispatch, averaged over the
# 7616 chunked passes of a step, scaled by the device-copy calibration (FETCH x 2, WRITE x 1); see
# profiles/hbm_counters_coax20k.md.  Re-measure when the kernel changes.
K_LB_FAR_FETCH_KIB = 5058.2
K_LB_FAR_WRITE_KIB = 1862.8
K_LB_FAR_TRAFFIC_BYTES = (2.0 * K_LB_FAR_FETCH_KIB + 1.0 * K_LB_FAR_WRITE_KIB) * 1024.0
# the same for k_lf_pass, the default one-launch-per-stage layout: not yet taken (None)
K_LF_PASS_TRAFFIC_BYTES = None
FLOP_POT_PAIR = 86
FP64_VALU_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--lines", type=int, default=256)
    ap.add_argument("--max-steps", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-rows", type=int, default=19732)
    ap.add_argument("--cpu-sample-lines", type=int, default=48)
    ap.add_argument("--cpu-sample-steps", type=int, default=800)
    ap.add_argument("--no-tts", action="store_true", help="skip the 64-load-case time-to-solve comparison")
    ap.add_argument("--tts-only", action="store_true", help="only the 64-load-case time-to-solve comparison")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the gradient and the 64-load-case x 64-line runs")
    ap.add_argument("--extras-only", action="store_true", help="only the gradient and 4096-line runs")
    ap.add_argument("--nodal-only", action="store_true", help="only the nodal-basis sphere run")
    ap.add_argument("--mixed-step", action="store_true",
                    help="only the benchmark step in MIXED precision (FP32 far field), for kernel profiles")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file (JSON): reuse one tile choice across runs, e.g. for counter runs")
    ap.add_argument("--set-tuning", default=None,
                    help="comma-separated key=value tuning knobs applied after the autotuner (experiments)")
    ap.add_argument("--trace-groups", type=int, default=None,
                    help="line groups of the field-line tracer (1..4; default: the library's)")
    ap.add_argument("--no-far-events", action="store_true",
                    help="skip the repeat of the steps that times the dominant kernel by events (for kernel traces)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run 5 device-to-device copies of 1 GiB (HBM counter calibration)")
    return ap.parse_args()


def calibrate_copy():
    import torch
    a = torch.empty(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
    a.fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "device copy", "bytes_read_per_launch": a.numel() * 8,
                      "bytes_written_per_launch": a.numel() * 8, "launches": 5}))


TTS_TOLS = (1e-4, 3e-5, 1e-5, 3e-6, 1e-6, 3e-7, 1e-7, 3e-8, 1e-8)


def time_to_solve(bem, torch, p, ctx64, nrhs=64, target=1e-5):
    """64 load cases (driven electrode U[0.5, 2], shell at 0) from the assembled state, each path
    stopped at the loosest GMRES tolerance (from TTS_TOLS) whose solution has sigma within
    `target` of the reference in every load case (max_j |s_j - s_ref_j| / max_j |s_ref_j|; the
    reference is the batched FP64 solve to 1e-12, which the parity tests tie to the oracle):
    FP64 one by one, FP64 batched (FP64 matrix cores) and mixed batched (FP32 matrix cores
    inside FP64 refinement).  The tolerance search is untimed; the reported time is the best
    of two runs at the chosen tolerance."""
    from workloads import rod_load_cases
    bv = rod_load_cases(p, nrhs, seed=4)
    N = p.n_tri
    ref, _ = ctx64.solve(bv, tol=1e-12, max_iter=20000)
    refs = ref[:, :N]
    out = {"load_cases": nrhs, "target_sigma_rel_err": target,
           "reference": "batched FP64 solve to 1e-12"}

    def err_of(sol):
        return float(((sol[:, :N] - refs).abs().max(dim=1).values / refs.abs().max(dim=1).values).max().item())

    def run(ctx, key):
        chosen = None
        for tol in TTS_TOLS:
            sol, info = ctx.solve(bv, tol=tol, max_iter=20000, raise_on_noconv=False)
            if info["converged"] and err_of(sol) <= target:
                chosen = tol
                break
        if chosen is None:
            out[key] = {"error": "no tolerance in the list reached the target"}
            return
        best = None
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sol, info = ctx.solve(bv, tol=chosen, max_iter=20000)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        out[key] = {"s": best, "tol": chosen, "iters": info["iters"], "refinements": info["refinements"],
                    "sigma_rel_err": err_of(sol)}

    ctx64.set_tuning("batched_solve", 0)
    run(ctx64, "fp64_one_by_one")
    ctx64.set_tuning("batched_solve", 1)
    run(ctx64, "fp64_batched")
    ctxm = bem.Context.from_problem(p, precision=bem.MIXED, eta=6.0, restart=100)
    ctxm.assemble()
    run(ctxm, "mixed_batched")
    ctxm.close()
    if all("s" in out[k] for k in ("fp64_one_by_one", "fp64_batched", "mixed_batched")):
        out["speedup_mixed_vs_fp64_one_by_one"] = out["fp64_one_by_one"]["s"] / out["mixed_batched"]["s"]
        out["speedup_mixed_vs_fp64_batched"] = out["fp64_batched"]["s"] / out["mixed_batched"]["s"]
    return out


def gradient_run(bem, torch, p, ctx):
    """Gradient of J = sum of the streamer integrals of 128 lines (seed 7) at V0 = 1 with respect to
    all vertex coordinates and body potentials (bem_streamer_grad), after one forward run."""
    from workloads import electrode_line_starts
    starts, panel, bary = electrode_line_starts(p, 128, seed=7)
    st = torch.tensor(starts, device="cuda")
    tp = bem.trace_params(h=1e-4, max_steps=2000, e_min=1e-3)
    sol, _ = ctx.solve(p.body_V, tol=1e-12, max_iter=20000)
    g = torch.ones(128, dtype=torch.float64, device="cuda")
    ctx.streamer_grad(sol, st, g, tp, start_panel=panel, start_bary=bary)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    I, ns, stc, _ = ctx.streamer_integral(sol, st, tp)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dvert, dV, _ = ctx.streamer_grad(sol, st, g, tp, start_panel=panel, start_bary=bary)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    G = dvert.cpu().numpy()
    return {"lines": 128, "J": float(I.sum().item()), "forward_s": t1 - t0, "gradient_s": t2 - t1,
            "gradient_over_forward": (t2 - t1) / (t1 - t0), "dJ_dV_rod": float(dV[0, 1].item()),
            "translation_residual_rel": float(np.linalg.norm(G.sum(axis=0)) / np.abs(G).sum())}


def cases_by_lines_run(bem, torch, p, ctx):
    """64 load cases (rod U[0.5, 2], seed 4) solved together, then 64 lines per case (seed 5):
    4096 field lines with streamer integrals in one call, both line layouts timed."""
    from workloads import electrode_line_starts, rod_load_cases
    bv = rod_load_cases(p, 64, seed=4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol, info = ctx.solve(bv, tol=1e-10, max_iter=20000)
    torch.cuda.synchronize()
    t_solve = time.perf_counter() - t0
    starts, _, _ = electrode_line_starts(p, 4096, seed=5)
    st = torch.tensor(starts, device="cuda")
    lr = np.repeat(np.arange(64, dtype=np.int32), 64)
    tp = bem.trace_params(h=1e-4, max_steps=2000, e_min=1e-3)
    out = {"load_cases": 64, "lines": 4096, "solve_s": t_solve, "solve_iters": info["iters"]}
    for mode, name in ((1, "all_lines_together"), (2, "persistent_per_line")):
        ctx.set_tuning("trace_mode", mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        I, ns, stc, _ = ctx.streamer_integral(sol, st, tp, line_rhs=lr)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ns_h = ns.cpu().numpy()
        passes = int(np.sum(1 + 4 * ns_h + 4 * (stc.cpu().numpy() != 0)))
        out[name] = {"s": dt, "field_evals": passes, "pairs_per_s": passes * p.n_tri / dt,
                     "integral_sum": float(I.sum().item())}
    ctx.set_tuning("trace_mode", 0)
    return out


def mixed_step_run(bem, torch, p, cen, on_panel, starts, tp, args):
    """The benchmark step in MIXED precision (FP32 far field, FP64 near entries, Krylov vectors
    and refinement): assembly, solve to 1e-8, E at the centroids and the 256 field lines, after
    one warm-up step; per-phase kernel times from the library's event timers."""
    ctx = bem.Context.from_problem(p, precision=bem.MIXED, eta=6.0, restart=100)
    ctx.assemble()
    ctx.autotune(args.tune_cache)

    def step():
        ctx.assemble()
        sol, info = ctx.solve(p.body_V, tol=1e-8, max_iter=5000)
        ctx.eval_field(sol, cen, on_panel=on_panel, want_phi=False)
        I, ns, st, _ = ctx.streamer_integral(sol, starts, tp)
        return sol, info, I, ns, st

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sol, info, I, ns, st = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    ctx.set_profiling(1)
    ctx.reset_stats()
    step()
    torch.cuda.synchronize()
    phases = {k: ctx.kernel_stats(k)[1] for k in ("far_assemble", "near_assemble", "gemv", "eval_far", "trace",
                                                    "trace_far", "trace_step", "trace_pass")}
    ctx.set_profiling(0)
    out = {"ms_per_step": ms, "gmres_iters": info["iters"], "refinements": info["refinements"],
           "streamer_integral_sum": float(I.sum().item()), "phase_ms": phases,
           "stop_code_counts": {str(k): int((st.cpu().numpy() == k).sum()) for k in range(6)}}
    ctx.close()
    return out


def c3_run(bem, torch):
    """Coax at ~60k panels: single-right-hand-side solve in FP64 (to 1e-10) and in the mixed mode
    (FP64 refinement to 1e-8) from the assembled state, and the mixed errors on sigma and on |E|
    at 1000 air-gap points (seed 3) against FP64."""
    from workloads import coax_problem_for_size, gap_eval_points
    p = coax_problem_for_size(60000)
    N = p.n_tri
    pts = torch.tensor(gap_eval_points(1000, seed=3), device="cuda")
    out = {"panels": N}
    res = {}
    for name, prec, tol in (("fp64", bem.FP64, 1e-10), ("mixed", bem.MIXED, 1e-8)):
        ctx = bem.Context.from_problem(p, precision=prec, eta=6.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.assemble()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sol, info = ctx.solve(p.body_V, tol=tol, max_iter=20000)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        _, E = ctx.eval_field(sol, pts, want_phi=False)
        res[name] = (sol[0, :N].clone(), torch.linalg.norm(E[0], dim=1))
        out[name] = {"assemble_s": t1 - t0, "solve_s": t2 - t1, "iters": info["iters"],
                     "refinements": info["refinements"], "rel_residual": info["rel_residual"]}
        ctx.close()
        torch.cuda.empty_cache()
    s64, e64 = res["fp64"]
    sm, em = res["mixed"]
    out["mixed_sigma_rel_err"] = float((sm - s64).abs().max() / s64.abs().max())
    out["mixed_E_rel_err"] = float((em - e64).abs().max() / e64.abs().max())
    out["solve_speedup_mixed_vs_fp64"] = out["fp64"]["solve_s"] / out["mixed"]["solve_s"]
    return out


def bushing_run(bem, torch):
    """Bushing-like device with thin floating sheets (element size 8 mm, ~30k panels): FP64
    assembly and solve to 1e-10 (after a warm-up solve), the four floating foils' potentials,
    and 256 field lines from the rod to the first foil."""
    from workloads import bushing_problem, electrode_line_starts
    p = bushing_problem(0.008)
    N = p.n_tri
    ctx = bem.Context.from_problem(p, eta=6.0)
    ctx.assemble()
    ctx.solve(p.body_V, tol=1e-10, max_iter=20000)   # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.assemble()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sol, info = ctx.solve(p.body_V, tol=1e-10, max_iter=20000)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    starts, _, _ = electrode_line_starts(p, 256, seed=3)
    tp = bem.trace_params(h=1e-4, max_steps=2000, e_min=1e-6)
    I, ns, st, _ = ctx.streamer_integral(sol, torch.tensor(starts, device="cuda"), tp)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    V = sol[0, N:N + 4].cpu().numpy()
    out = {"panels": N, "unknowns": int(ctx.n), "assemble_s": t1 - t0, "solve_s": t2 - t1,
           "iters": info["iters"], "rel_residual": info["rel_residual"],
           "floating_foil_potentials_over_V0": [float(v) for v in V],
           "lines": 256, "trace_s": t3 - t2,
           "stop_code_counts": {str(k): int((st.cpu().numpy() == k).sum()) for k in range(6)}}
    ctx.close()
    torch.cuda.empty_cache()
    return out


def nodal_run(bem, torch):
    """The paper's nodal piecewise-linear basis (vertex collocation, Eq. Matrix) beside the
    constant basis on the conductor sphere, whose density is V0/R exactly: FP64 assembly
    (timed after a warm-up) and solve to 1e-10, and the largest density error.  Nodal on
    icospheres of level 5 (10,242 vertices, 20,480 panels) and 6 (40,962 / 81,920);
    constant on level 5 (20,480 unknowns).  Then the nodal system of the coaxial conductors
    (rod, grounded shell, floating ring) at 67,729 vertices, the node count of the paper's
    Table 3 device, with 256 field lines from the rod (RK4, h = 1e-4, <= 2000 steps) and
    their streamer integrals; the same system with FP32 vertex rows (MIXED, as the paper
    stores its matrix); and the conductors at the paper's 232,029-node count in MIXED
    (about 215 GB of FP32 matrix on one GPU)."""
    from workloads import sphere_problem
    out = {}

    def one(level, basis):
        p = sphere_problem(level)
        kw = dict(basis=bem.BASIS_LINEAR, constraint_form=1) if basis else {}
        ctx = bem.Context.from_problem(p, **kw)
        ctx.assemble()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.assemble()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sol, info = ctx.solve(p.body_V, tol=1e-10, max_iter=5000)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        nu = p.n_vert if basis else p.n_tri
        dens = sol[0, :nu].cpu().numpy()
        rows = p.n_vert if basis else p.n_tri
        r = {"unknowns": int(ctx.n), "panels": p.n_tri, "assemble_s": t1 - t0,
             "row_panel_pairs_per_s": rows * p.n_tri / (t1 - t0), "solve_s": t2 - t1, "iters": info["iters"],
             "max_density_error": float(np.max(np.abs(dens - 1.0)))}
        ctx.close()
        torch.cuda.empty_cache()
        return r

    out["linear_L5"] = one(5, True)
    out["linear_L6"] = one(6, True)
    out["constant_L5"] = one(5, False)
    # the coaxial conductors at the node count of the paper's Table 3 device (68,218)
    from workloads import coax_conductors_for_vertices
    p = coax_conductors_for_vertices(68218)
    ctx = bem.Context.from_problem(p, basis=bem.BASIS_LINEAR, constraint_form=1)
    ctx.assemble()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.assemble()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sol, info = ctx.solve(p.body_V, tol=1e-10, max_iter=5000)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    from workloads import electrode_line_starts
    starts, _, _ = electrode_line_starts(p, 256, seed=2)
    tp = bem.trace_params(h=1e-4, max_steps=2000, e_min=1e-3)
    st_d = torch.tensor(starts, device="cuda")
    ctx.streamer_integral(sol, st_d, tp)   # warm-up
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    I, ns, st, _ = ctx.streamer_integral(sol, st_d, tp)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    out["linear_coax_conductors"] = {
        "unknowns": int(ctx.n), "vertices": p.n_vert, "panels": p.n_tri, "assemble_s": t1 - t0,
        "row_panel_pairs_per_s": p.n_vert * p.n_tri / (t1 - t0), "matrix_entries_per_s": ctx.n ** 2 / (t1 - t0),
        "solve_s": t2 - t1, "iters": info["iters"], "ring_potential_over_V0": float(sol[0, p.n_vert].cpu()),
        "lines": 256, "trace_s": t4 - t3, "steps_total": int(ns.sum().cpu()),
        "stop_code_counts": {str(k): int((st.cpu().numpy() == k).sum()) for k in range(6)}}
    x64 = sol[0].cpu().numpy()
    ctx.close()
    torch.cuda.empty_cache()
    # the same system stored as the paper stores its matrix: FP32 vertex rows (MIXED),
    # solved inside FP64 iterative refinement to 1e-8
    ctx = bem.Context.from_problem(p, basis=bem.BASIS_LINEAR, constraint_form=1, precision=bem.MIXED)
    ctx.assemble()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.assemble()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sol, info = ctx.solve(p.body_V, tol=1e-8, max_iter=5000)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    x32 = sol[0].cpu().numpy()
    out["linear_coax_conductors_mixed"] = {
        "unknowns": int(ctx.n), "assemble_s": t1 - t0, "solve_s": t2 - t1, "iters": info["iters"],
        "refinements": info["refinements"],
        "density_error_vs_fp64": float(np.abs(x32 - x64).max() / np.abs(x64).max())}
    ctx.close()
    torch.cuda.empty_cache()
    # the node count of the paper's 232,029-node case, FP32 vertex rows (about 215 GB), one GPU
    p = coax_conductors_for_vertices(232029)
    ctx = bem.Context.from_problem(p, basis=bem.BASIS_LINEAR, constraint_form=1, precision=bem.MIXED)
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.assemble()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sol, info = ctx.solve(p.body_V, tol=1e-8, max_iter=5000)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        out["linear_coax_conductors_232k_mixed"] = {
            "unknowns": int(ctx.n), "vertices": p.n_vert, "panels": p.n_tri,
            "matrix_gb": 4.0 * p.n_vert * ctx.n / 1e9, "assemble_s": t1 - t0,
            "row_panel_pairs_per_s": p.n_vert * p.n_tri / (t1 - t0), "solve_s": t2 - t1, "iters": info["iters"],
            "refinements": info["refinements"], "rel_residual": info["rel_residual"],
            "ring_potential_over_V0": float(sol[0, p.n_vert].cpu())}
    except bem.BemError as e:   # e.g. a GPU with less memory than the 218 GB this needs
        out["linear_coax_conductors_232k_mixed"] = {"error": str(e)}
    finally:
        ctx.close()
        torch.cuda.empty_cache()
    return out


def host_info():
    """CPU model, logical CPUs this process may use, and RAM of the host."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    ram_gb = None
    try:
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                ram_gb = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    return {"cpu_model": model, "cpus_available": len(os.sched_getaffinity(0)), "ram_gib": ram_gb}


def cpu_baseline(p, x, starts, args):
    """The oracle, compiled here with -O3 -march=native, on a bounded sample: a block of matrix
    rows and a few short lines.  cores = the OpenMP threads its parallel loops ran with."""
    import tempfile

    import oracle
    oracle.build_native(os.path.join(tempfile.gettempdir(), "bem_oracle_native"))
    o = oracle.Oracle(p)
    rng = np.random.default_rng(12)
    rows = np.sort(rng.choice(p.n_tri, size=min(args.cpu_sample_rows, p.n_tri), replace=False))
    t0 = time.perf_counter()
    o.assemble_rows(rows)
    t_rows = time.perf_counter() - t0
    tp = oracle.trace_params(h=1e-4, max_steps=args.cpu_sample_steps)
    t0 = time.perf_counter()
    ns, st, _ = o.trace(x, starts[:args.cpu_sample_lines], tp)
    t_lines = time.perf_counter() - t0
    passes = int(np.sum(1 + 4 * ns + 4 * (st != 0)))
    pairs = len(rows) * p.n_tri + passes * p.n_tri
    out = {"value": pairs / (t_rows + t_lines), "unit": "pairs/s", "cores": oracle.num_threads(), "kind": "oracle",
           "sample": f"{len(rows)} matrix rows x {p.n_tri} panels + {args.cpu_sample_lines} field lines x "
                     f"{args.cpu_sample_steps} RK4 steps on the same mesh ({t_rows + t_lines:.1f} s)",
           "build": "gcc -O3 -march=native -ffp-contract=off -fopenmp"}
    out.update(host_info())
    return out


def main():
    args = parse()
    if args.calibrate_copy:
        calibrate_copy()
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import paper_2003_12663_amd as bem
    from workloads import coax_problem_for_size, electrode_line_starts

    torch.cuda.set_device(0)
    p = coax_problem_for_size(20000)
    N = p.n_tri
    starts_h, _, _ = electrode_line_starts(p, args.lines, seed=2)
    cen_h = p.vert[p.tri].mean(axis=1)
    dev = torch.device("cuda", 0)
    starts = torch.tensor(starts_h, device=dev)
    cen = torch.tensor(cen_h, device=dev)
    on_panel = torch.arange(N, dtype=torch.int32, device=dev)
    tp = bem.trace_params(h=1e-4, max_steps=args.max_steps, e_min=1e-3)
    ctx = bem.Context.from_problem(p, precision=bem.FP64, eta=6.0, restart=100)
    print(f"[bench] coax N={N} lines={args.lines}", file=sys.stderr, flush=True)
    if args.nodal_only:
        ctx.close()
        print(json.dumps({"nodal_basis": nodal_run(bem, torch)}))
        return
    if args.mixed_step:
        ctx.close()
        print(json.dumps({"mixed_step": mixed_step_run(bem, torch, p, cen, on_panel, starts, tp, args)}))
        return
    if args.tts_only:
        ctx.assemble()
        print(json.dumps({"time_to_solve_64_load_cases": time_to_solve(bem, torch, p, ctx)}))
        ctx.close()
        return
    if args.extras_only:
        ctx.assemble()
        ctx.autotune(None)
        print(json.dumps({"gradient_coax_128_lines": gradient_run(bem, torch, p, ctx),
                          "cases_64_x_lines_64": cases_by_lines_run(bem, torch, p, ctx),
                          "coax_60k_mixed_vs_fp64": c3_run(bem, torch),
                          "bushing_thin_sheets": bushing_run(bem, torch),
                          "nodal_basis": nodal_run(bem, torch)}))
        ctx.close()
        return
    # tile shapes for this problem, timed before the timed region (tuning re-assembles)
    ctx.assemble()
    ctx.autotune(args.tune_cache)
    if args.trace_groups is not None:
        ctx.set_tuning("trace_groups", args.trace_groups)
    if args.set_tuning:
        for kv in args.set_tuning.split(","):
            key, val = kv.split("=")
            ctx.set_tuning(key.strip(), int(val))
    tuning = {k: ctx.get_tuning(k) for k in ("far_rows", "gemv_rows", "gemm_blocks", "eval_blocks", "trace_mode",
                                              "trace_lpb", "trace_rnd", "trace_tile", "trace_splitk", "trace_split",
                                              "trace_few", "trace_groups")}
    if tuning["trace_groups"] == 0:   # the library's default: two line groups from 128 lines
        tuning["trace_groups"] = 2 if args.lines >= 128 else 1

    def step():
        ctx.assemble()
        sol, info = ctx.solve(p.body_V, tol=1e-10, max_iter=5000)
        _, E = ctx.eval_field(sol, cen, on_panel=on_panel, want_phi=False)
        I, ns, st, ex = ctx.streamer_integral(sol, starts, tp)
        return sol, info, I, ns, st

    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        print(f"[bench] warmup {w} done", file=sys.stderr, flush=True)
    # timed region: nothing profiled
    ctx.set_profiling(0)
    ctx.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        sol, info, I, ns, st = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    print(f"[bench] timed {args.steps} steps: {ms_step:.1f} ms/step", file=sys.stderr, flush=True)
    # regular pairs and launches of the two-kernel far passes (k_lb_far) and of the one-launch stages
    # (k_lf_pass: the last few lines by default, every stage with trace_mode 3)
    far_launches = ctx.counter("trace_far_launches") / args.steps
    far_pairs = ctx.counter("trace_far_pairs") / args.steps
    pass_launches = ctx.counter("trace_pass_launches") / args.steps
    pass_pairs = ctx.counter("trace_pass_pairs") / args.steps
    near_line_pairs = (ctx.counter("trace_near_pairs") + ctx.counter("trace_pass_near_pairs")) / args.steps
    # the same steps again with the dominant kernel timed by events carried in its own dispatches
    # (profiling mode 2): its launch durations for the roofline (the events slow the step, so these
    # steps are not the timed ones)
    ms_step_prof = None
    if not args.no_far_events:
        ctx.set_profiling(2)
        ctx.reset_stats()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for k in range(args.steps):
            step()
        torch.cuda.synchronize()
        ms_step_prof = (time.perf_counter() - t2) * 1e3 / args.steps
    fused = far_launches == 0   # one launch per stage throughout (trace_mode 3)
    tf_n, tf_ms = ctx.kernel_stats("trace_pass" if fused else "trace_far")
    if fused:
        far_launches, far_pairs = pass_launches, pass_pairs
    # one more step, untimed, with every kernel timed: the per-phase breakdown
    ctx.set_profiling(1)
    ctx.reset_stats()
    step()
    torch.cuda.synchronize()
    ctx.set_profiling(0)

    ns_h = ns.cpu().numpy()
    st_h = st.cpu().numpy()
    passes = int(np.sum(1 + 4 * ns_h + 4 * (st_h != 0)))    # field evaluations per step on the lines
    n_unk = ctx.n
    n_float_rows = int(np.sum(p.body_kind[p.tri_body] == bem.FLOATING))
    pairs_matrix = N * N + n_float_rows * N
    pairs_surface = N * N
    pairs_lines = passes * N
    pairs = pairs_matrix + pairs_surface + pairs_lines
    stats = {k: ctx.kernel_stats(k) for k in ("geometry", "far_assemble", "near_mask_csr", "near_assemble",
                                                "finalize", "gemv", "gmres_ortho", "gmres_iter", "eval_mask",
                                                "eval_near_csr", "eval_far", "eval_near", "trace", "trace_far",
                                                "trace_step", "trace_pass")}
    # dominant kernel: the far-field pass of the field-line tracer (k_lb_far), one launch per RK4 stage,
    # every launch of a repeat of the timed steps timed by its own clock stamps (profiling mode 2)
    far_flop_per_launch = far_pairs * FLOP_FIELD_PAIR / far_launches
    far_avg_ms = tf_ms / tf_n if tf_n > 0 else None
    achieved = far_flop_per_launch / (far_avg_ms * 1e-3) / 1e12 if far_avg_ms else None
    gv_n, gv_ms = stats["gemv"]
    gemv_ms = gv_ms / max(gv_n, 1)
    gemv_gbs = (8.0 * n_unk * n_unk) / (gemv_ms * 1e-3) / 1e9
    fa_n, fa_ms = stats["far_assemble"]
    kernel_ms = {k: v[1] for k, v in stats.items()}   # one profiled step after the timed ones

    # wall time of each phase, unprofiled: a few more steps with the host clock read after each
    # call has finished (each call depends on the one before, so the synchronisations add little
    # more than the launch latency of the next call's first kernel)
    wall = {"assemble": 0.0, "solve": 0.0, "eval_field": 0.0, "trace": 0.0}
    n_wall = 3
    for _ in range(n_wall):
        torch.cuda.synchronize()
        ta = time.perf_counter()
        ctx.assemble()
        torch.cuda.synchronize()
        tb = time.perf_counter()
        sol, info = ctx.solve(p.body_V, tol=1e-10, max_iter=5000)
        torch.cuda.synchronize()
        tc = time.perf_counter()
        ctx.eval_field(sol, cen, on_panel=on_panel, want_phi=False)
        torch.cuda.synchronize()
        td = time.perf_counter()
        ctx.streamer_integral(sol, starts, tp)
        torch.cuda.synchronize()
        te = time.perf_counter()
        for k, dt in zip(wall, (tb - ta, tc - tb, td - tc, te - td)):
            wall[k] += dt * 1e3 / n_wall
    trace_ms = wall["trace"]

    extras = {}
    if not args.no_extras:
        print("[bench] gradient and 64 x 64 lines", file=sys.stderr, flush=True)
        extras["gradient_coax_128_lines"] = gradient_run(bem, torch, p, ctx)
        extras["cases_64_x_lines_64"] = cases_by_lines_run(bem, torch, p, ctx)
        extras["coax_60k_mixed_vs_fp64"] = c3_run(bem, torch)
        extras["bushing_thin_sheets"] = bushing_run(bem, torch)
        extras["nodal_basis"] = nodal_run(bem, torch)

    tts = None
    if not args.no_tts:
        print("[bench] time-to-solve, 64 load cases", file=sys.stderr, flush=True)
        tts = time_to_solve(bem, torch, p, ctx)

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle sample)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(p, sol[0].cpu().numpy(), starts_h, args)

    out = {
        "metric": "panel-pair evals/s",
        "value": pairs / (ms_step * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "coax rod-in-shell, floating torus, eps_r=4 spacer; FP64 assembly + GMRES(1e-10) + "
                        "surface E at all centroids + 256 field lines (RK4 h=1e-4, <=2000 steps) with streamer "
                        "integral",
            "panels": N, "unknowns": n_unk, "lines": args.lines, "max_steps": args.max_steps, "eta": 6.0,
            "gmres_restart": 100,
        },
        "field_evals_per_s": passes / (trace_ms * 1e-3),
        "field_line_passes": passes,
        "gmres_iters": info["iters"],
        "gmres_rel_residual": info["rel_residual"],
        "assembly_pairs_per_s": pairs_matrix / (fa_ms / max(fa_n, 1) * 1e-3),
        "gemv_GBps": gemv_gbs,
        "gemv_frac_hbm": gemv_gbs / HBM_PEAK_GBS,
        "phase_ms_per_step": wall,
        "kernel_ms_profiled_step": kernel_ms,
        "streamer_integral_sum": float(I.sum().item()),
        "stop_code_counts": {str(k): int(np.sum(st_h == k)) for k in range(6)},
        "roofline": {"kernel": ("k_lf_pass (one launch per RK4 stage of the field lines: the previous stage's "
                                "step, then the regular and near pairs of all live lines, FP64)") if fused else
                               "k_lb_far (far-field pass of the field-line tracer, FP64)", "bound": "alu",
                     "achieved": achieved, "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VALU_PEAK_TFLOPS if achieved else None,
                     "traffic": K_LF_PASS_TRAFFIC_BYTES if fused else K_LB_FAR_TRAFFIC_BYTES,
                     "traffic_unit": "bytes per launch (HBM, counters)",
                     "flop_per_pair": FLOP_FIELD_PAIR, "pairs_per_launch": far_pairs / far_launches,
                     "launches_per_step": far_launches, "avg_launch_ms": far_avg_ms,
                     "timed_launches": tf_n, "ms_per_step_with_far_events": ms_step_prof},
        "trace_ms_per_step": trace_ms,
        "trace_near_pairs": near_line_pairs,
        "cpu_baseline": cpu,
        "time_to_solve_64_load_cases": tts,
        "tuning": tuning,
    }
    out.update(extras)
    print(json.dumps(out))
    ctx.close()


if __name__ == "__main__":
    main()
