"""Nodal piecewise-linear basis (Sec. 3, Eq. Matrix) on the GPU against the FP64 oracle.

Vertex hats collocated at the vertices, conductor and floating-conductor
bodies, a floating body's row its net charge.  Bars as for the constant basis:
matrix entries 1e-12 of the row's largest, right-hand sides exact, solutions,
potentials and fields 1e-10.  Cases: spheres and a floating shell (vertex counts that
leave ragged row tiles and column groups), two devices in one problem, the
coaxial conductors with a floating ring (flat caps: coplanar near pairs), and
on sampled oracle rows a level-5 sphere (10,242 vertices) and the coaxial
conductors at 67,729 vertices.  Field lines and streamer integrals of the nodal
density against the oracle's: step counts and stop codes exact, integrals 1e-10.
"""

import numpy as np
import pytest

import oracle
from workloads import (coax_conductors_for_vertices, coax_conductors_problem, floating_shell_problem, sphere_problem,
                       union_problem)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def bem():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_12663_amd as bem
    return bem


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _ctx(bem, p):
    c = bem.Context.from_problem(p, basis=bem.BASIS_LINEAR, constraint_form=1)
    c.assemble()
    return c


CASES = [
    ("sphere_L1", lambda: sphere_problem(1, V0=2.0)),
    ("sphere_L3", lambda: sphere_problem(3)),
    ("floating_shell_L2", lambda: floating_shell_problem(2, V0=3.0)),
    ("sphere_and_shell", lambda: union_problem(sphere_problem(2, V0=1.5), floating_shell_problem(1, V0=-1.0),
                                               (4.0, 0.5, 0.0))),
    # rod, grounded shell and floating ring; flat caps give coplanar near pairs
    ("coax_conductors", lambda: coax_conductors_problem(0.012)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_nodal_matrix_rhs_solution(bem, name, make):
    p = make()
    o = oracle.Oracle(p, constraint_form=1)
    A = o.p1_assemble()
    b_ref = o.p1_rhs(p.body_V)
    x_ref = np.linalg.solve(A, b_ref)
    c = _ctx(bem, p)
    print(f"[nodal] {name}: n_vert {p.n_vert}, n {c.n}", flush=True)
    assert c.n == A.shape[0] == p.n_vert + int(np.sum(p.body_kind == 1))
    G = c.copy_rows(0, c.n).cpu().numpy()
    assert (np.abs(G - A) / np.abs(A).max(axis=1, keepdims=True)).max() <= 1e-12
    b = c.rhs(p.body_V)[0].cpu().numpy()
    assert np.array_equal(b, b_ref)
    sol, info = c.solve(p.body_V, tol=1e-13, max_iter=5000)
    assert info["converged"]
    assert rel(sol[0].cpu().numpy(), x_ref) <= 1e-10
    # potential at points inside, outside and near the surface
    rng = np.random.default_rng(4)
    pts = np.concatenate([rng.uniform(-3, 3, (40, 3)), p.vert[rng.integers(0, p.n_vert, 8)] * 1.02])
    phi = c.potential(sol, pts)[0].cpu().numpy()
    phi_ref, E_ref = o.p1_field(sol[0].cpu().numpy(), pts)
    assert rel(phi, phi_ref) <= 1e-10
    phi2, E = c.eval_field(sol, pts)
    assert np.array_equal(phi2[0].cpu().numpy(), phi)
    assert rel(E[0].cpu().numpy(), E_ref) <= 1e-10
    c.close()


def test_nodal_matches_closed_form_sphere(bem):
    """Conductor sphere at V0: u = V0/R at every vertex to the discretisation error
    (second order: level 4 below 2e-3), potential V0 R/|x| and field V0 R x/|x|^3
    outside, V0 and 0 inside."""
    p = sphere_problem(4, V0=1.0)
    c = _ctx(bem, p)
    sol, info = c.solve(p.body_V, tol=1e-12, max_iter=5000)
    u = sol[0].cpu().numpy()
    assert np.max(np.abs(u - 1.0)) < 2e-3
    pts = np.array([[0.0, 0.0, 3.0], [2.0, -1.0, 0.5], [0.1, 0.2, -0.3], [0.0, 1.3, 0.2]])
    phi, E = c.eval_field(sol, pts)
    phi, E = phi[0].cpu().numpy(), E[0].cpu().numpy()
    r = np.linalg.norm(pts, axis=1)
    assert np.max(np.abs(phi - np.where(r > 1, 1 / r, 1.0))) < 2e-3
    assert np.max(np.abs(E - np.where((r > 1)[:, None], pts / r[:, None] ** 3, 0.0))) < 2e-3
    c.close()


def test_nodal_large_sampled_rows(bem):
    """Level-5 sphere (10,242 vertices, 20,480 triangles): sampled rows of the
    GPU matrix against the oracle's rows, and the GPU solution's residual on
    those rows."""
    p = sphere_problem(5)
    c = _ctx(bem, p)
    rows = np.unique(np.concatenate([[0, 1, 63, 64, p.n_vert - 1], np.random.default_rng(2).integers(0, p.n_vert, 11)]))
    R = oracle.Oracle(p, constraint_form=1).p1_assemble_rows(rows)
    for k, r in enumerate(rows):
        g = c.copy_rows(int(r), 1)[0].cpu().numpy()
        assert np.abs(g - R[k]).max() <= 1e-12 * np.abs(R[k]).max(), r
    sol, info = c.solve(p.body_V, tol=1e-12, max_iter=5000)
    x = sol[0].cpu().numpy()
    b = oracle.Oracle(p, constraint_form=1).p1_rhs(p.body_V)[rows]
    assert np.abs(R @ x - b).max() <= 1e-10
    c.close()


def test_nodal_paper_size_sampled_rows(bem):
    """The coaxial conductors at 67,729 vertices (135,450 panels; the paper's Table 3
    device has 68,218 nodes): sampled rows against the oracle, the GPU solution's
    residual on them, and the floating ring between its neighbours' potentials."""
    p = coax_conductors_for_vertices(68218)
    print(f"[nodal] coax conductors: {p.n_vert} vertices, {p.n_tri} panels", flush=True)
    c = _ctx(bem, p)
    nv = p.n_vert
    rows = np.unique(np.concatenate([[0, 255, 256, nv - 1, nv], np.random.default_rng(5).integers(0, nv, 7)]))
    o = oracle.Oracle(p, constraint_form=1)
    R = o.p1_assemble_rows(rows)
    for k, r in enumerate(rows):
        g = c.copy_rows(int(r), 1)[0].cpu().numpy()
        assert np.abs(g - R[k]).max() <= 1e-12 * np.abs(R[k]).max(), r
    sol, info = c.solve(p.body_V, tol=1e-10, max_iter=5000)
    assert info["converged"]
    x = sol[0].cpu().numpy()
    assert np.abs(R @ x - o.p1_rhs(p.body_V)[rows]).max() <= 1e-8
    assert 0.0 < x[nv] < 1.0
    c.close()
    torch.cuda.empty_cache()


def _lines_vs_oracle(bem, p, starts, tp_kw):
    o = oracle.Oracle(p, constraint_form=1)
    u_ref = np.linalg.solve(o.p1_assemble(), o.p1_rhs(p.body_V))
    c = _ctx(bem, p)
    sol, info = c.solve(p.body_V, tol=1e-13, max_iter=5000)
    assert rel(sol[0].cpu().numpy(), u_ref) <= 1e-10
    ns_o, st_o, I_o = o.p1_trace(sol[0].cpu().numpy(), starts, oracle.trace_params(**tp_kw))
    I, ns, st, _ = c.streamer_integral(sol, torch.tensor(starts, device="cuda"), bem.trace_params(**tp_kw))
    ns, st, I = ns.cpu().numpy(), st.cpu().numpy(), I.cpu().numpy()
    assert np.array_equal(ns, ns_o) and np.array_equal(st, st_o)
    assert np.max(np.abs(I - I_o)) <= 1e-10 * max(np.max(np.abs(I_o)), 1e-300)
    c.close()
    return ns, st, I


def test_nodal_field_lines_sphere(bem):
    """Radial lines of the nodal solution on the conductor sphere at V0 = 100:
    step counts and stop codes exact, integrals 1e-10 against the oracle, and
    the integral within the discretisation error of the closed form."""
    p = sphere_problem(3, V0=100.0)
    dirs = np.random.default_rng(9).standard_normal((12, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    kw = dict(h=5e-3, max_steps=100, e_min=1e-3, alpha_a=1e-3, alpha_e0=25.0, alpha_p=2.0)
    ns, st, I = _lines_vs_oracle(bem, p, 1.1 * dirs, kw)
    F = lambda r: 1e-3 * (-1e4 / (3 * r ** 3) + 2 * 100.0 * 25.0 / r + 625.0 * r)
    assert np.all(ns == 100) and np.max(np.abs(I / (F(1.6) - F(1.1)) - 1.0)) < 1e-2


def test_nodal_field_lines_coax(bem):
    """40 lines from the rod of the coaxial conductors (nodal basis): lines end
    on the shell (code 1) or the floating ring (code 2) or run out of steps; the
    far passes go from the split to the few-line kernel as lines stop."""
    from workloads import electrode_line_starts
    p = coax_conductors_problem(0.012, V0=40.0)
    starts, _, _ = electrode_line_starts(p, 40, seed=4)
    kw = dict(h=2e-3, max_steps=300, e_min=1e-3, alpha_a=1e-3, alpha_e0=25.0, alpha_p=2.0)
    ns, st, I = _lines_vs_oracle(bem, p, starts, kw)
    print(f"[nodal] coax lines: stop codes {np.bincount(st, minlength=6)}", flush=True)
    assert np.any(st == 1) and np.any(ns > 20) and np.any(I > 0)


def test_nodal_field_lines_two_load_cases(bem):
    """Lines of two load cases in one call (nodal basis: traced case by case inside)
    equal the single-case calls bit for bit and the oracle's lines per case to
    1e-10; paths keep the slots after each line's last point untouched."""
    p = union_problem(sphere_problem(2, V0=100.0), sphere_problem(2, V0=0.0), (3.0, 0.0, 0.0))
    c = _ctx(bem, p)
    bv = np.array([[100.0, 0.0], [0.0, 80.0]])
    sol, _ = c.solve(bv, tol=1e-13, max_iter=5000)
    dirs = np.random.default_rng(12).standard_normal((10, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    starts = 1.15 * dirs + np.where((np.arange(10) % 2 == 1)[:, None], np.array([3.0, 0.0, 0.0]), 0.0)
    lr = (np.arange(10) % 2).astype(np.int32)
    kw = dict(h=5e-3, max_steps=60, e_min=1e-3, alpha_a=1e-3, alpha_e0=25.0, alpha_p=2.0)
    tp = bem.trace_params(**kw)
    I, ns, st, _ = c.streamer_integral(sol, torch.tensor(starts, device="cuda"), tp, line_rhs=lr)
    ns_p, st_p, path = c.trace_lines(sol, torch.tensor(starts, device="cuda"), tp, line_rhs=lr, want_path=True)
    I, ns, st = I.cpu().numpy(), ns.cpu().numpy(), st.cpu().numpy()
    assert np.array_equal(ns, ns_p.cpu().numpy()) and np.array_equal(st, st_p.cpu().numpy())
    o = oracle.Oracle(p, constraint_form=1)
    for r in range(2):
        sel = np.nonzero(lr == r)[0]
        I1, ns1, st1, _ = c.streamer_integral(sol[r:r + 1], torch.tensor(starts[sel], device="cuda"), tp)
        assert np.array_equal(I[sel], I1.cpu().numpy()) and np.array_equal(ns[sel], ns1.cpu().numpy())
        ns_o, st_o, I_o = o.p1_trace(sol[r].cpu().numpy(), starts[sel], oracle.trace_params(**kw))
        assert np.array_equal(ns[sel], ns_o) and np.array_equal(st[sel], st_o)
        assert np.max(np.abs(I[sel] - I_o)) <= 1e-10 * np.max(np.abs(I_o))
    P = path.cpu().numpy()   # NaN-filled before the call
    for l in range(10):
        assert np.all(np.isfinite(P[l, :ns[l] + 1])) and np.all(np.isnan(P[l, ns[l] + 1:]))
        assert np.allclose(P[l, 0], starts[l], rtol=0, atol=0)
    c.close()


@pytest.mark.parametrize("name,make", [CASES[2], CASES[4]], ids=[CASES[2][0], CASES[4][0]])
def test_nodal_mixed_precision(bem, name, make):
    """MIXED storage of the nodal system: vertex rows in FP32 (each entry formed in
    FP64, then rounded; a near contribution adds a second rounding, and all
    entries are positive, so within 2.4e-7 of the FP64 entry), constraint rows in
    FP64 and equal to the FP64 matrix's; the solution with iterative refinement and
    its field within 1e-5 of FP64."""
    p = make()
    c64 = _ctx(bem, p)
    c32 = bem.Context.from_problem(p, basis=bem.BASIS_LINEAR, constraint_form=1, precision=bem.MIXED)
    c32.assemble()
    nv = p.n_vert
    G64 = c64.copy_rows(0, c64.n).cpu().numpy()
    G32 = c32.copy_rows(0, c32.n).cpu().numpy()
    assert np.all(np.abs(G32[:nv] - G64[:nv]) <= 2.4e-7 * np.abs(G64[:nv]))
    assert np.array_equal(G32[nv:], G64[nv:])
    s64, _ = c64.solve(p.body_V, tol=1e-12, max_iter=5000)
    s32, info = c32.solve(p.body_V, tol=1e-8, max_iter=5000)
    assert info["converged"] and info["refinements"] >= 1
    assert rel(s32[0].cpu().numpy(), s64[0].cpu().numpy()) <= 1e-5
    pts = np.random.default_rng(7).uniform(-0.3, 0.3, (32, 3)) + np.array([0.0, 0.0, 1.8 if name != "coax_conductors" else 0.2])
    _, E64 = c64.eval_field(s64, pts)
    _, E32 = c32.eval_field(s32, pts)
    assert rel(E32[0].cpu().numpy(), E64[0].cpu().numpy()) <= 1e-5
    print(f"[nodal] mixed {name}: sigma {rel(s32[0].cpu().numpy(), s64[0].cpu().numpy()):.2e} "
          f"iters {info['iters']} refinements {info['refinements']}", flush=True)
    c64.close()
    c32.close()


def test_nodal_mixed_field_lines(bem):
    """Field lines of the nodal density in a MIXED context.  The nodal far-field records
    exist in FP64 only, so the line passes are the FP64 ones in either precision: driven
    by the same vertex values, a MIXED context's lines equal an FP64 context's bit for
    bit, one load case and the few-line tail included.  Driven by the MIXED solution
    (within 1e-5 of FP64), stop codes and step counts match the FP64 run's and the
    integrals agree to 1e-4 (the density error, amplified by alpha's slope)."""
    from workloads import electrode_line_starts
    p = coax_conductors_problem(0.012, V0=40.0)
    c64 = _ctx(bem, p)
    c32 = bem.Context.from_problem(p, basis=bem.BASIS_LINEAR, constraint_form=1, precision=bem.MIXED)
    c32.assemble()
    starts, _, _ = electrode_line_starts(p, 24, seed=4)
    kw = dict(h=2e-3, max_steps=300, e_min=1e-3, alpha_a=1e-3, alpha_e0=25.0, alpha_p=2.0)
    tp = bem.trace_params(**kw)
    s64, _ = c64.solve(p.body_V, tol=1e-12, max_iter=5000)
    s32, _ = c32.solve(p.body_V, tol=1e-8, max_iter=5000)
    I64, ns64, st64, _ = c64.streamer_integral(s64, starts, tp)
    I32, ns32, st32, _ = c32.streamer_integral(s64, starts, tp)
    assert np.array_equal(I32.cpu().numpy(), I64.cpu().numpy())
    assert np.array_equal(ns32.cpu().numpy(), ns64.cpu().numpy())
    assert np.array_equal(st32.cpu().numpy(), st64.cpu().numpy())
    Im, nsm, stm, _ = c32.streamer_integral(s32, starts, tp)
    assert np.array_equal(stm.cpu().numpy(), st64.cpu().numpy())
    nsm, ns64h = nsm.cpu().numpy(), ns64.cpu().numpy()
    assert np.abs(nsm - ns64h).max() <= 1
    same = nsm == ns64h           # a hit can move by one step; compare integrals where it did not
    assert same.sum() >= len(same) - 2
    e = rel(Im.cpu().numpy()[same], I64.cpu().numpy()[same])
    print(f"[nodal] mixed lines: integral error vs FP64 {e:.2e}", flush=True)
    assert e <= 1e-4
    # the same lines against the oracle's nodal trace of the FP64 vertex values
    o = oracle.Oracle(p, constraint_form=1)
    ns_o, st_o, I_o = o.p1_trace(s64[0].cpu().numpy(), starts, oracle.trace_params(**kw))
    assert np.array_equal(ns32.cpu().numpy(), ns_o) and np.array_equal(st32.cpu().numpy(), st_o)
    assert np.abs(I32.cpu().numpy() - I_o).max() <= 1e-10 * np.abs(I_o).max()
    c64.close()
    c32.close()


def test_nodal_mixed_232k_sampled_rows(bem):
    """The coaxial conductors at 233,519 vertices (the paper's 232,029-node case) in
    MIXED storage, 218 GB of FP32 rows on one GPU.  Checked: sampled rows within 2.4e-7
    of the oracle's FP64 rows, the FP64 constraint row to its summation order, the solution's residual
    against those FP64 rows, and the ring's potential against the 67,729-vertex FP64
    solution's (0.41826 V0)."""
    p = coax_conductors_for_vertices(232029)
    print(f"[nodal] coax conductors: {p.n_vert} vertices, {p.n_tri} panels, MIXED", flush=True)
    c = bem.Context.from_problem(p, basis=bem.BASIS_LINEAR, constraint_form=1, precision=bem.MIXED)
    c.assemble()
    nv = p.n_vert
    rows = np.unique(np.concatenate([[0, nv - 1, nv], np.random.default_rng(6).integers(0, nv, 5)]))
    o = oracle.Oracle(p, constraint_form=1)
    R = o.p1_assemble_rows(rows)
    for k, r in enumerate(rows):
        g = c.copy_rows(int(r), 1)[0].cpu().numpy()
        if r < nv:
            assert np.all(np.abs(g - R[k]) <= 2.4e-7 * np.abs(R[k]) + 1e-300), r
        else:   # FP64 constraint row: the body's area is a sum over 233,519 vertices on the GPU and
            # over triangles in the oracle, so the two differ in summation order (bound ~ n eps)
            assert np.abs(g - R[k]).max() <= 1e-11 * np.abs(R[k]).max(), r
    sol, info = c.solve(p.body_V, tol=1e-8, max_iter=5000)
    assert info["converged"]
    x = sol[0].cpu().numpy()
    b = o.p1_rhs(p.body_V)[rows]
    assert np.abs(R @ x - b).max() <= 1e-5 * np.abs(b).max() + 1e-5
    assert abs(x[nv] - 0.41826) < 1e-3
    c.close()
    torch.cuda.empty_cache()


def test_nodal_empty_inputs(bem):
    """No points and no lines are no-ops."""
    p = sphere_problem(1)
    c = _ctx(bem, p)
    sol, _ = c.solve(p.body_V, tol=1e-12)
    phi, E = c.eval_field(sol, np.zeros((0, 3)))
    assert phi.shape == (1, 0) and E.shape == (1, 0, 3)
    I, ns, st, _ = c.streamer_integral(sol, torch.zeros((0, 3), dtype=torch.float64, device="cuda"),
                                       bem.trace_params(h=1e-3))
    assert I.numel() == 0 and ns.numel() == 0
    c.close()


def test_nodal_batched_load_cases(bem):
    """Several load cases in one call agree with one-by-one solves."""
    p = union_problem(sphere_problem(2, V0=1.0), sphere_problem(2, V0=0.0), (3.0, 0.0, 0.0))
    c = _ctx(bem, p)
    bv = np.array([[1.0, 0.0], [0.0, 1.0], [1.0, -1.0]])
    sol, info = c.solve(bv, tol=1e-12, max_iter=5000)
    for r in range(3):
        s1, _ = c.solve(bv[r], tol=1e-12, max_iter=5000)
        assert rel(sol[r].cpu().numpy(), s1[0].cpu().numpy()) <= 1e-9
    # linearity: case 2 = case 0 - case 1
    s = sol.cpu().numpy()
    assert rel(s[2], s[0] - s[1]) <= 1e-9
    c.close()


def test_nodal_refusals(bem):
    p = sphere_problem(1)
    c = _ctx(bem, p)
    sol, _ = c.solve(p.body_V, tol=1e-10)
    with pytest.raises(bem.BemError):   # volume points only
        c.eval_field(sol, p.vert[p.tri[:1]].mean(axis=1), on_panel=np.zeros(1, dtype=np.int32))
    c.set_tuning("trace_mode", 2)
    with pytest.raises(bem.BemError):   # field lines in the batched layout only
        c.streamer_integral(sol, torch.tensor([[0.0, 0.0, 1.2]], device="cuda"), bem.trace_params(h=1e-3))
    c.set_tuning("trace_mode", 0)
    with pytest.raises(bem.BemError):   # no gradient
        c.streamer_grad(sol, torch.tensor([[0.0, 0.0, 1.2]], device="cuda"),
                        torch.ones(1, dtype=torch.float64, device="cuda"), bem.trace_params(h=1e-3, max_steps=5))
    c.close()
