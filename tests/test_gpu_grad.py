"""GPU gradient of the streamer integrals (bem_streamer_grad) against the oracle.

The oracle's forward-mode dual-number derivative (pinned to finite differences
of the plain oracle in test_oracle_grad.py) gives dJ along a direction
(dvert, dV); the GPU's reverse-mode gradient dotted with the same direction
must agree to 1e-8 relative.  The weights dJ/dI_l are seeded.  Also checked:
rigid-motion invariance and the autograd wrapper.
"""

import numpy as np
import pytest

from workloads import (bushing_problem, coated_sphere_problem, coax_problem_for_size, electrode_line_starts,
                       floating_shell_problem, sphere_problem, sphere_sheet_problem, union_problem)

pytestmark = pytest.mark.gpu

REL = 1e-8


@pytest.fixture(scope="module")
def bem():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_12663_amd as bem
    return bem


def _case(bem, oracle_mod, p, L, steps, h, cf=0, seed=6, nrhs=1, batch=None):
    import torch
    dev = torch.device("cuda", 0)
    starts, panel, bary = electrode_line_starts(p, L, seed=seed)
    ctx = bem.Context.from_problem(p, precision=bem.FP64, eta=6.0, constraint_form=cf)
    if batch is not None:
        ctx.set_tuning("grad_batch", batch)
    ctx.assemble()
    bv = np.stack([p.body_V * (1.0 + 0.25 * r) for r in range(nrhs)])
    sol, info = ctx.solve(bv, tol=1e-13, max_iter=20000)
    tp = bem.trace_params(h=h, max_steps=steps, e_min=1e-3)
    lr = (np.arange(L) % nrhs).astype(np.int32) if nrhs > 1 else None
    I, ns, st, _ = ctx.streamer_integral(sol, torch.tensor(starts, device=dev), tp, line_rhs=lr)
    g = np.random.default_rng(11).uniform(0.5, 1.5, L)
    dvert, dV, dstart = ctx.streamer_grad(sol, torch.tensor(starts, device=dev), torch.tensor(g, device=dev), tp,
                                          line_rhs=lr, start_panel=panel, start_bary=bary, want_dstart=True)
    return dict(ctx=ctx, starts=starts, panel=panel, bary=bary, bv=bv, sol=sol, I=I.cpu().numpy(),
                ns=ns.cpu().numpy(), st=st.cpu().numpy(), g=g, lr=lr, dvert=dvert.cpu().numpy(),
                dV=dV.cpu().numpy(), dstart=dstart.cpu().numpy(), tp=tp)


def _oracle_dir(oracle_mod, p, c, dvert, dV, cf=0):
    """Oracle dJ along (dvert, dV) for every load case's lines."""
    o = oracle_mod.Oracle(p, constraint_form=cf)
    tp = oracle_mod.trace_params(h=c["tp"].h, max_steps=c["tp"].max_steps, e_min=c["tp"].e_min)
    nrhs = c["bv"].shape[0]
    J = dJ = 0.0
    for r in range(nrhs):
        sel = np.arange(len(c["g"])) if c["lr"] is None else np.nonzero(c["lr"] == r)[0]
        I, dI, u, du, rc = o.dual_streamer(dvert, c["bv"][r], dV[r] if dV is not None else None, c["panel"][sel],
                                           c["bary"][sel], tp, c["ns"][sel])
        assert rc == 0
        assert np.max(np.abs(I - c["I"][sel])) <= 1e-10 * max(np.max(np.abs(I)), 1e-300)
        J += float(np.dot(c["g"][sel], I))
        dJ += float(np.dot(c["g"][sel], dI))
    return J, dJ


def _sheet_and_shell():
    return union_problem(sphere_sheet_problem(1, V0=100.0, eps_in=4.0), floating_shell_problem(1, V0=50.0),
                         (6.0, 0.0, 0.0))


CASES = [
    ("sphere", lambda: sphere_problem(1, V0=50.0), 4, 60, 1e-2, 0, 1),
    ("floating_shell_hits", lambda: floating_shell_problem(1, V0=50.0), 6, 200, 5e-3, 0, 1),
    ("floating_shell_reduced", lambda: floating_shell_problem(1, V0=50.0), 4, 30, 5e-3, 1, 1),
    ("coated_sphere", lambda: coated_sphere_problem(1, V0=200.0), 4, 30, 5e-3, 0, 1),
    ("sphere_two_load_cases", lambda: sphere_problem(2, V0=50.0), 6, 40, 1e-2, 0, 2),
    # thin floating sheets (Eq. sheets): a sheet between two dielectrics, a sheet next to a closed
    # floating shell (per-body constraint rows, both forms), a coarse bushing (four sheets and an
    # insulator interface; lines end on the first foil)
    ("sphere_sheet", lambda: sphere_sheet_problem(1, V0=100.0, eps_in=4.0), 4, 30, 5e-3, 0, 1),
    ("sheet_and_shell", lambda: _sheet_and_shell(), 6, 30, 5e-3, 0, 1),
    ("sheet_and_shell_reduced", lambda: _sheet_and_shell(), 6, 30, 5e-3, 1, 1),
    ("bushing", lambda: bushing_problem(0.08, V0=5.0), 6, 40, 2e-3, 0, 2),
]


@pytest.mark.parametrize("name,make,L,steps,h,cf,nrhs", CASES, ids=[c[0] for c in CASES])
def test_gradient_matches_oracle_dual(bem, oracle_mod, name, make, L, steps, h, cf, nrhs):
    p = make()
    print(f"[grad] {name} N={p.n_tri} L={L} steps={steps}", flush=True)
    c = _case(bem, oracle_mod, p, L, steps, h, cf, nrhs=nrhs)
    assert np.all(c["I"] > 0.0)
    rng = np.random.default_rng(8)
    for trial in range(2):
        dv = rng.standard_normal(p.vert.shape)
        dV = rng.standard_normal((nrhs, p.n_body))
        _, dJ = _oracle_dir(oracle_mod, p, c, dv, dV, cf)
        gpu = float(np.sum(c["dvert"] * dv) + np.sum(c["dV"] * dV))
        scale = np.linalg.norm(c["dvert"]) * np.linalg.norm(dv) + np.linalg.norm(c["dV"]) * np.linalg.norm(dV)
        assert abs(gpu - dJ) <= REL * scale, (gpu, dJ, scale)
    c["ctx"].close()


def _check_dirs(oracle_mod, p, c, cf=0, trials=2):
    rng = np.random.default_rng(8)
    nrhs = c["bv"].shape[0]
    for trial in range(trials):
        dv = rng.standard_normal(p.vert.shape)
        dV = rng.standard_normal((nrhs, p.n_body))
        _, dJ = _oracle_dir(oracle_mod, p, c, dv, dV, cf)
        gpu = float(np.sum(c["dvert"] * dv) + np.sum(c["dV"] * dV))
        scale = np.linalg.norm(c["dvert"]) * np.linalg.norm(dv) + np.linalg.norm(c["dV"]) * np.linalg.norm(dV)
        assert abs(gpu - dJ) <= REL * scale, (trial, gpu, dJ, scale)


def test_gradient_small_batches(bem, oracle_mod):
    """Point batches smaller than the panel count (stage points and collocation points)."""
    p = sphere_problem(2, V0=50.0)
    c = _case(bem, oracle_mod, p, 6, 40, 1e-2, nrhs=2, batch=100)
    _check_dirs(oracle_mod, p, c)
    c["ctx"].close()


@pytest.mark.parametrize("L,steps", [(4, 2000), (80, 150)], ids=["4_full_lines", "80_short_lines"])
def test_gradient_coarse_coax(bem, oracle_mod, L, steps):
    """Coax with all body kinds (grounded shell, driven rod, floating torus, eps_r = 4 spacer),
    coarse mesh; lines hit the shell (first case) or run out of steps (second)."""
    from workloads import coax_problem
    p = coax_problem(0.012)
    print(f"[grad] coarse coax N={p.n_tri} L={L} steps={steps}", flush=True)
    c = _case(bem, oracle_mod, p, L, steps, 1e-4, seed=7)
    assert np.all(c["I"] >= 0.0) and c["I"].sum() > 0.0
    _check_dirs(oracle_mod, p, c, trials=1)
    G = c["dvert"]
    assert np.linalg.norm(G.sum(axis=0)) <= 1e-9 * np.abs(G).sum()
    c["ctx"].close()


def test_gradient_body_potential_only(bem, oracle_mod):
    """dJ/dV alone (vertex direction zero) on a floating-shell case."""
    p = floating_shell_problem(1, V0=50.0)
    c = _case(bem, oracle_mod, p, 4, 30, 5e-3)
    dV = np.zeros((1, p.n_body))
    dV[0, 0] = 1.0
    _, dJ = _oracle_dir(oracle_mod, p, c, None, dV)
    assert abs(c["dV"][0, 0] - dJ) <= REL * abs(dJ)
    assert c["dV"][0, 1] == 0.0          # floating body: no prescribed potential
    c["ctx"].close()


def test_gradient_line_starts(bem, oracle_mod):
    """dJ/dstarts (mesh fixed) against central differences of the oracle trace (step 1e-8: the
    starts sit 1e-6 above their panels, a larger step could move one through the surface)."""
    p = sphere_problem(1, V0=50.0)
    c = _case(bem, oracle_mod, p, 4, 60, 1e-2)
    o = oracle_mod.Oracle(p)
    u = c["sol"][0].cpu().numpy()
    tp = oracle_mod.trace_params(h=1e-2, max_steps=60, e_min=1e-3)
    ds = np.random.default_rng(9).standard_normal(c["starts"].shape)
    hfd = 1e-8
    nsp, _, Ip = o.trace(u[:p.n_tri], c["starts"] + hfd * ds, tp)
    nsm, _, Im = o.trace(u[:p.n_tri], c["starts"] - hfd * ds, tp)
    assert np.array_equal(nsp, c["ns"]) and np.array_equal(nsm, c["ns"])
    fd = float(np.dot(c["g"], (Ip - Im) / (2 * hfd)))
    gpu = float(np.sum(c["dstart"] * ds))
    assert abs(gpu - fd) <= 1e-6 * np.linalg.norm(c["dstart"]) * np.linalg.norm(ds)
    c["ctx"].close()


@pytest.mark.parametrize("motion", ["translation", "rotation"])
def test_gradient_rigid_motion(bem, oracle_mod, motion):
    """Moving mesh and starts together changes nothing: sum_v dJ/dv = 0, sum_v v x dJ/dv = 0."""
    p = floating_shell_problem(2, V0=50.0)
    c = _case(bem, oracle_mod, p, 8, 60, 5e-3)
    G = c["dvert"]
    if motion == "translation":
        res = np.linalg.norm(G.sum(axis=0))
    else:
        res = np.linalg.norm(np.cross(p.vert, G).sum(axis=0))
        G = G * np.linalg.norm(p.vert, axis=1, keepdims=True)
    assert res <= 1e-9 * np.abs(G).sum()
    c["ctx"].close()


def test_autograd_function(bem, oracle_mod):
    import torch
    p = sphere_problem(1, V0=50.0)
    starts, panel, bary = electrode_line_starts(p, 4, seed=6)
    dev = torch.device("cuda", 0)
    vert = torch.tensor(p.vert, device=dev, requires_grad=True)
    bV = torch.tensor(p.body_V, device=dev, requires_grad=True)
    tp = bem.trace_params(h=1e-2, max_steps=60, e_min=1e-3)
    I = bem.streamer_integral(vert, bV, p, panel, bary, tp)
    w = torch.tensor(np.random.default_rng(11).uniform(0.5, 1.5, 4), device=dev)
    J = (w * I).sum()
    gv, gV = torch.autograd.grad(J, (vert, bV))
    o = oracle_mod.Oracle(p)
    otp = oracle_mod.trace_params(h=1e-2, max_steps=60, e_min=1e-3)
    A = o.assemble()
    u = np.linalg.solve(A, o.rhs(p.body_V))
    ns, st, I0 = o.trace(u[:p.n_tri], starts, otp)
    assert np.max(np.abs(I.detach().cpu().numpy() - I0)) <= 1e-10 * np.max(np.abs(I0))
    dv = np.random.default_rng(3).standard_normal(p.vert.shape)
    _, dI, _, _, _ = o.dual_streamer(dv, p.body_V, np.array([0.7]), panel, bary, otp, ns)
    ref = float(np.dot(w.cpu().numpy(), dI))
    got = float((gv.cpu().numpy() * dv).sum() + gV.cpu().numpy()[0] * 0.7)
    assert abs(got - ref) <= REL * (np.linalg.norm(gv.cpu().numpy()) * np.linalg.norm(dv) + abs(gV.cpu().numpy()[0]))


def test_gradient_coax_full_size_invariants(bem):
    """Coax (~20k panels, rod at V0 = 1), 128 lines: translation invariance of the vertex
    gradient and Euler homogeneity in the potentials, sum_k V_k dJ/dV_k = dJ/dlambda of
    J(lambda V), the latter by central differences of the GPU forward (a self-consistency
    check: paths do not depend on lambda when only the rod is driven)."""
    import torch
    p = coax_problem_for_size(20000)
    dev = torch.device("cuda", 0)
    starts, panel, bary = electrode_line_starts(p, 128, seed=7)
    print(f"[grad] coax N={p.n_tri} L=128", flush=True)
    ctx = bem.Context.from_problem(p, precision=bem.FP64, eta=6.0)
    ctx.assemble()
    tp = bem.trace_params(h=1e-4, max_steps=2000, e_min=1e-3)
    st_t = torch.tensor(starts, device=dev)

    def J_of(scale):
        sol, _ = ctx.solve(p.body_V * scale, tol=1e-13, max_iter=20000)
        I, ns, st, _ = ctx.streamer_integral(sol, st_t, tp)
        return sol, I.cpu().numpy(), ns.cpu().numpy()

    sol, I, ns = J_of(1.0)
    assert I.sum() > 0.0
    g = np.ones(128)
    dvert, dV, _ = ctx.streamer_grad(sol, st_t, torch.tensor(g, device=dev), tp, start_panel=panel,
                                     start_bary=bary)
    G = dvert.cpu().numpy()
    assert np.linalg.norm(G.sum(axis=0)) <= 1e-8 * np.abs(G).sum()
    hfd = 1e-6
    _, Ip, nsp = J_of(1.0 + hfd)
    _, Im, nsm = J_of(1.0 - hfd)
    assert np.array_equal(nsp, ns) and np.array_equal(nsm, ns)
    euler = float(np.dot(dV.cpu().numpy()[0], p.body_V))
    fd = float((Ip.sum() - Im.sum()) / (2 * hfd))
    assert abs(euler - fd) <= 1e-6 * abs(fd)
    ctx.close()


def test_gradient_c5_sphere_against_stored_dual():
    """The differentiable-design case on the sphere at its stated size: icosphere level 3 (1280
    panels), V0 = 50, 128 lines (seed 6), RK4 h = 1e-4, <= 2000 steps, J = sum of the integrals.
    The GPU forward reproduces the oracle's step counts and stop codes exactly and J to 1e-10;
    the GPU gradient along 20 single-vertex directions (seed 8) and along the potential matches
    the oracle's dual derivative, stored by tests/golden/make_c5_sphere.py, to 1e-8 relative to
    |grad| |direction|; and it matches central differences (h = 1e-6) of the GPU forward to
    1e-5 of the same scale (the forward's solve error, divided by 2h)."""
    import json
    import os

    import torch
    import paper_2003_12663_amd as bem
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "c5_sphere_dual.json")))
    p = sphere_problem(3, V0=50.0)
    starts, panel, bary = electrode_line_starts(p, gold["lines"], seed=gold["seed_lines"])
    tp = bem.trace_params(**gold["trace"])
    print(f"[grad] C5 sphere N={p.n_tri} L={gold['lines']}", flush=True)

    def forward(vert, bv):
        c = bem.Context(vert, p.tri, p.tri_body, p.body_kind, p.eps_plus, p.eps_minus)
        c.assemble()
        sol, _ = c.solve(bv, tol=1e-13, max_iter=20000)
        st_d = c.panel_points(panel, bary, tp.start_offset)
        I, ns, st, _ = c.streamer_integral(sol, st_d, tp)
        return c, sol, st_d, I.cpu().numpy(), ns.cpu().numpy(), st.cpu().numpy()

    c, sol, st_d, I, ns, st = forward(p.vert, p.body_V)
    assert np.array_equal(ns, gold["n_steps"]) and np.array_equal(st, gold["stop_code"])
    assert abs(I.sum() - gold["J"]) <= 1e-10 * abs(gold["J"])
    g = torch.ones(gold["lines"], dtype=torch.float64, device="cuda")
    dvert, dV, _ = c.streamer_grad(sol, st_d, g, tp, start_panel=panel, start_bary=bary)
    G = dvert.cpu().numpy()
    dV0 = float(dV[0, 0].item())
    scale = np.linalg.norm(G)
    c.close()
    assert abs(dV0 - gold["dJ_dV0"]) <= REL * abs(gold["dJ_dV0"])
    worst_dual = worst_fd = 0.0
    hfd = 1e-6
    for d in gold["directions"]:
        v, u = d["vertex"], np.array(d["direction"])
        got = float(G[v] @ u)
        worst_dual = max(worst_dual, abs(got - d["dJ"]) / scale)
        Js = []
        for sgn in (1.0, -1.0):
            vert = p.vert.copy()
            vert[v] += sgn * hfd * u
            cc, _, _, Ih, nsh, _ = forward(vert, p.body_V)
            cc.close()
            assert np.array_equal(nsh, ns)
            Js.append(Ih.sum())
        fd = (Js[0] - Js[1]) / (2 * hfd)
        worst_fd = max(worst_fd, abs(got - fd) / scale)
    print(f"[grad] C5 sphere: |grad| {scale:.3e}, dual error {worst_dual:.2e}, FD error {worst_fd:.2e} "
          f"(relative to |grad|)", flush=True)
    assert worst_dual <= REL and worst_fd <= 1e-5


def test_gradient_c5_coax_against_central_differences():
    """The differentiable-design case on the ~20k-panel coax at V0 = 1, 128 lines (seed 7), RK4
    h = 1e-4, <= 2000 steps: the GPU gradient along 20 single-vertex directions (seed 8) against
    central differences (h = 1e-6) of the parity-tested GPU forward, the line starts moving
    with their panels.  A draw whose perturbed runs change a line's step count is skipped for
    the next (the derivative is that of the piece containing the state).  Bar: 1e-5 of
    |grad| |direction| (the forward's solve error, about 1e-11 of J, divided by 2h)."""
    import torch
    import paper_2003_12663_amd as bem
    from workloads import vertex_perturbations
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    p = coax_problem_for_size(20000)
    starts, panel, bary = electrode_line_starts(p, 128, seed=7)
    tp = bem.trace_params(h=1e-4, max_steps=2000, e_min=1e-3)
    print(f"[grad] C5 coax N={p.n_tri} L=128", flush=True)

    def forward(vert):
        c = bem.Context(vert, p.tri, p.tri_body, p.body_kind, p.eps_plus, p.eps_minus)
        c.assemble()
        sol, _ = c.solve(p.body_V, tol=1e-13, max_iter=20000)
        st_d = c.panel_points(panel, bary, tp.start_offset)
        I, ns, st, _ = c.streamer_integral(sol, st_d, tp)
        return c, sol, st_d, I.cpu().numpy(), ns.cpu().numpy()

    c, sol, st_d, I, ns = forward(p.vert)
    g = torch.ones(128, dtype=torch.float64, device="cuda")
    dvert, dV, _ = c.streamer_grad(sol, st_d, g, tp, start_panel=panel, start_bary=bary)
    G = dvert.cpu().numpy()
    c.close()
    scale = np.linalg.norm(G)
    hfd = 1e-6
    gen = vertex_perturbations(p, seed=8)
    worst, skipped, done = 0.0, 0, 0
    while done < 20:
        v, u = next(gen)
        Js = []
        ok = True
        for sgn in (1.0, -1.0):
            vert = p.vert.copy()
            vert[v] += sgn * hfd * u
            cc, _, _, Ih, nsh = forward(vert)
            cc.close()
            ok = ok and np.array_equal(nsh, ns)
            Js.append(Ih.sum())
        if not ok:
            skipped += 1
            assert skipped <= 5
            continue
        fd = (Js[0] - Js[1]) / (2 * hfd)
        got = float(G[v] @ u)
        worst = max(worst, abs(got - fd) / scale)
        done += 1
    print(f"[grad] C5 coax: |grad| {scale:.3e}, FD error {worst:.2e} (relative to |grad|), "
          f"{skipped} draws skipped", flush=True)
    assert worst <= 1e-5
