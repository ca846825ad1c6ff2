"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars (FP64 mode): matrix entries within 1e-12 of the row's largest entry;
sigma and |E| within 1e-10 in the max-norm relative metric
max_j |a_j - b_j| / max_j |b_j|; field-line step counts and stop codes
bit-exact; streamer integrals within 1e-10 relative.
"""

import sys

import numpy as np
import pytest

import oracle
from workloads import (coated_sphere_problem, coax_problem, electrode_line_starts, floating_shell_problem,
                       gap_eval_points, sphere_eval_points, sphere_problem)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(msg):
    print(f"[gpu-parity] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bem():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_12663_amd as bem
    return bem


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _ctx(bem, p, **kw):
    c = bem.Context.from_problem(p, **kw)
    c.assemble()
    return c


def _matrix_check(bem, p, rows=None, **kw):
    o = oracle.Oracle(p, eta=kw.get("eta", 6.0), constraint_form=kw.get("constraint_form", 0))
    c = _ctx(bem, p, **kw)
    if rows is None:
        A = o.assemble()
        G = c.copy_rows(0, c.n).cpu().numpy()
    else:
        A = o.assemble_rows(rows)
        G = np.stack([c.copy_rows(int(r), 1).cpu().numpy()[0] for r in rows])
    scale = np.abs(A).max(axis=1, keepdims=True)
    err = (np.abs(G - A) / scale).max()
    return c, o, err


@pytest.mark.parametrize("name,maker", [
    ("sphere_L3", lambda: sphere_problem(3)),
    ("coated_sphere_L2", lambda: coated_sphere_problem(2)),
    ("floating_shell_L2", lambda: floating_shell_problem(2)),
    ("coax_h012", lambda: coax_problem(0.012)),
])
def test_matrix_parity(bem, name, maker):
    p = maker()
    _say(f"matrix {name} N={p.n_tri}")
    c, o, err = _matrix_check(bem, p)
    assert err <= 1e-12, err
    # near-pair count equals the oracle's classification of centroid/panel pairs
    cen = p.vert[p.tri].mean(axis=1)
    assert c.near_pairs == int((o.classify(cen) == 0).sum())
    c.close()


def test_matrix_parity_reduced_constraint(bem):
    p = floating_shell_problem(2)
    _say("matrix floating shell reduced constraint")
    c, o, err = _matrix_check(bem, p, constraint_form=1)
    assert err <= 1e-12
    c.close()


def test_matrix_parity_ragged_small(bem):
    # N not a multiple of 64 or 256, one body, tiny mesh
    p = sphere_problem(1)          # 80 panels
    _say("matrix sphere L1")
    c, o, err = _matrix_check(bem, p)
    assert err <= 1e-12
    c.close()
    one = sphere_problem(0)        # 20 panels
    q = one.__class__(**{**one.__dict__, "tri": one.tri[:1], "tri_body": one.tri_body[:1]})
    _say("matrix single triangle")
    c, o, err = _matrix_check(bem, q)
    assert err <= 1e-12
    c.close()


def _sigma_case(bem, p, tol_gpu=1e-13):
    o = oracle.Oracle(p)
    A = o.assemble()
    b = o.rhs(p.body_V)
    x_ref = np.linalg.solve(A, b)
    c = _ctx(bem, p)
    sol, info = c.solve(p.body_V, tol=tol_gpu, max_iter=20000)
    assert info["converged"] and info["rel_residual"] <= tol_gpu
    x = sol[0].cpu().numpy()
    return c, o, x, x_ref


def test_sphere_solution_and_field(bem):
    p = sphere_problem(3)
    _say("sphere solve + eval")
    c, o, x, x_ref = _sigma_case(bem, p)
    assert rel(x, x_ref) <= 1e-10
    pts = sphere_eval_points()
    phi_o, E_o = o.eval(x_ref, pts)
    phi, E = c.eval_field(torch.tensor(x, device="cuda"), pts)
    E = E[0].cpu().numpy()
    assert rel(np.linalg.norm(E, axis=1), np.linalg.norm(E_o, axis=1)) <= 1e-10
    assert rel(E, E_o) <= 1e-10
    assert rel(phi[0].cpu().numpy(), phi_o) <= 1e-10
    # closed form (discretisation error of the L3 sphere)
    r = np.linalg.norm(pts, axis=1)
    Eex = pts / r[:, None] ** 3
    assert (np.linalg.norm(E - Eex, axis=1) / np.linalg.norm(Eex, axis=1)).max() < 5e-3
    # on-surface (exterior limit) at every 7th centroid
    idx = np.arange(0, p.n_tri, 7).astype(np.int32)
    cen = p.vert[p.tri[idx]].mean(axis=1)
    phs, Es = c.eval_field(torch.tensor(x, device="cuda"), cen, on_panel=idx)
    phso, Eso = o.eval(x, cen, on_panel=idx)
    assert rel(Es[0].cpu().numpy(), Eso) <= 1e-10
    assert rel(phs[0].cpu().numpy(), phso) <= 1e-10
    c.close()


@pytest.mark.parametrize("maker", [lambda: coated_sphere_problem(2), lambda: floating_shell_problem(2),
                                   lambda: coax_problem(0.012)])
def test_solution_parity_bodies(bem, maker):
    p = maker()
    _say(f"solve {p.name}")
    c, o, x, x_ref = _sigma_case(bem, p)
    assert rel(x, x_ref) <= 1e-10
    c.close()


def test_matvec_and_transpose(bem):
    p = coax_problem(0.012)
    _say("matvec coax")
    o = oracle.Oracle(p)
    A = o.assemble()
    c = _ctx(bem, p)
    rng = np.random.default_rng(0)
    X = rng.standard_normal((3, c.n))
    Xt = torch.tensor(X, device="cuda")
    Y = c.matvec(Xt).cpu().numpy()
    assert rel(Y, X @ A.T) <= 1e-12
    YT = c.matvec(Xt, transpose=True).cpu().numpy()
    assert rel(YT, X @ A) <= 1e-12
    c.close()


def test_coax_field_parity(bem):
    p = coax_problem(0.012)
    _say("coax eval")
    c, o, x, x_ref = _sigma_case(bem, p)
    pts = gap_eval_points(300, seed=3)
    phi_o, E_o = o.eval(x, pts)
    phi, E = c.eval_field(torch.tensor(x, device="cuda"), pts)
    assert rel(np.linalg.norm(E[0].cpu().numpy(), axis=1), np.linalg.norm(E_o, axis=1)) <= 1e-10
    assert rel(E[0].cpu().numpy(), E_o) <= 1e-10          # the vector, component by component
    assert rel(phi[0].cpu().numpy(), phi_o) <= 1e-10
    c.close()


def _trace_compare(bem, c, o, x, starts, params_kw, L_check=None):
    tp_o = oracle.trace_params(**params_kw)
    tp_g = bem.trace_params(**params_kw)
    sol = torch.tensor(x, device="cuda")
    I, ns, st, ex = c.streamer_integral(sol, starts, tp_g)
    ns2, st2, path = c.trace_lines(sol, starts, tp_g, want_path=True)
    I, ns, st = I.cpu().numpy(), ns.cpu().numpy(), st.cpu().numpy()
    assert np.array_equal(ns, ns2.cpu().numpy()) and np.array_equal(st, st2.cpu().numpy())
    sel = np.arange(len(starts)) if L_check is None else np.asarray(L_check)
    nso, sto, Io, patho = o.trace(x, starts[sel], tp_o, want_path=True)
    assert np.array_equal(ns[sel], nso), (ns[sel], nso)
    assert np.array_equal(st[sel], sto), (st[sel], sto)
    assert np.abs(I[sel] - Io).max() <= 1e-10 * max(np.abs(Io).max(), 1e-300)
    path = path.cpu().numpy()
    for k, l in enumerate(sel):
        m = ns[l] + 1
        assert np.abs(path[l, :m] - patho[k, :m]).max() <= 1e-9 * np.abs(patho[k, :m]).max()
    return I, ns, st


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_sphere_trace(bem, mode):
    p = sphere_problem(3, V0=50.0)
    _say(f"sphere trace mode {mode}")
    c, o, x, x_ref = _sigma_case(bem, p)
    c.set_tuning("trace_mode", mode)
    starts, _, _ = electrode_line_starts(p, 8, seed=6)
    I, ns, st = _trace_compare(bem, c, o, x, starts, dict(h=1e-4, max_steps=300))
    assert np.all(ns == 300) and np.all(st == 0) and np.all(I > 0)
    c.close()


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_coax_trace_stop_codes(bem, mode):
    p = coax_problem(0.012)
    _say(f"coax trace mode {mode}")
    c, o, x, x_ref = _sigma_case(bem, p)
    c.set_tuning("trace_mode", mode)
    starts, _, _ = electrode_line_starts(p, 12, seed=2)
    # h = 1e-3 keeps the oracle fast; lines reach the shell, ring or disc
    I, ns, st = _trace_compare(bem, c, o, x, starts, dict(h=1e-3, max_steps=200))
    assert set(st.tolist()) - {0, 1, 2, 3} == set()
    assert (st != 0).any()
    c.close()


@pytest.mark.parametrize("loop", [0, 64])
def test_tail_starts_on_a_hit_step(bem, loop):
    """The one-launch tail takes over after pass 31 (live counts are read every 32 passes), so
    its first launch evaluates the end point of step 8 (pass 32).  With h = 0.0105 from the coax
    rod, 26 of 32 lines cross the shell during step 8: the step's segment must be tested against
    the near panels in that first launch, and the lines must stop there (7 steps, Dirichlet
    hit) as in the oracle.  Both forms of the tail: one launch per stage (trace_loop 0) and one
    persistent launch."""
    p = coax_problem(0.012)
    _say(f"tail from a hit step, trace_loop {loop}")
    c, o, x, x_ref = _sigma_case(bem, p)
    c.set_tuning("trace_mode", 0)
    c.set_tuning("trace_tail", 4096)
    c.set_tuning("trace_loop", loop)
    starts, _, _ = electrode_line_starts(p, 32, seed=3)
    I, ns, st = _trace_compare(bem, c, o, x, starts, dict(h=0.0105, max_steps=12))
    assert ((ns == 7) & (st == 1)).sum() >= 20
    c.close()


def test_persistent_tail_wait_bound(bem):
    """A bound of zero polls on the persistent launch's waits between blocks (forced from the
    host): the call either reports that a wait reached its bound or, had no wait needed a poll,
    returns the oracle's results; the context traces correctly afterwards either way."""
    p = coax_problem(0.012)
    c, o, x, x_ref = _sigma_case(bem, p)
    c.set_tuning("trace_mode", 3)
    c.set_tuning("trace_loop", 64)   # the 16 lines in one persistent launch from the start
    starts, _, _ = electrode_line_starts(p, 16, seed=21)
    kw = dict(h=1e-3, max_steps=100)
    sol = torch.tensor(x, device="cuda")
    c.set_tuning("trace_spin", 0)
    try:
        ns, st, _ = c.trace_lines(sol, starts, bem.trace_params(**kw))
        raised = False
    except bem.BemError as e:
        assert "bound" in str(e)
        raised = True
    _say(f"zero-poll bound raised: {raised}")
    c.set_tuning("trace_spin", 1 << 22)
    _trace_compare(bem, c, o, x, starts, kw)
    c.close()


_LAYOUT_REF = {}


@pytest.mark.parametrize("layout", [
    # far pass + step kernel (trace_mode 1): split over 2, 4 or 8 waves, unsplit 64/128/256-line
    # tiles, split then the few-line tail
    dict(trace_mode=1, trace_splitk=2, trace_split=4096, trace_few=0),
    dict(trace_mode=1, trace_splitk=4, trace_split=4096, trace_few=0),
    dict(trace_mode=1, trace_splitk=8, trace_split=4096, trace_few=0),
    dict(trace_mode=1, trace_tile=64, trace_split=0, trace_few=0),
    dict(trace_mode=1, trace_tile=128, trace_split=0, trace_few=0),
    dict(trace_mode=1, trace_tile=256, trace_split=0, trace_few=0),
    dict(trace_mode=1, trace_splitk=4, trace_split=256, trace_tile=128, trace_few=8),
    # one launch per stage (trace_mode 3): 1, 2, 4, 8 line slots and 1, 2, 4 panel rounds per
    # block, fixed, and the shape chosen by the live count (with the fold of live slots)
    dict(trace_mode=3, trace_lpb=1, trace_rnd=1),
    dict(trace_mode=3, trace_lpb=2, trace_rnd=4),
    dict(trace_mode=3, trace_lpb=4, trace_rnd=2),
    dict(trace_mode=3, trace_lpb=8, trace_rnd=4),
    dict(trace_mode=3, trace_lpb=8, trace_rnd=1),
    dict(trace_mode=3),
    # all 16 lines in one persistent launch from the first stage
    dict(trace_mode=3, trace_loop=64),
    dict(trace_mode=3, trace_loop=64, trace_lpb=2, trace_rnd=2),
    # the same, one launch per stage to the end (no persistent launch)
    dict(trace_mode=3, trace_loop=0, trace_lpb=1, trace_rnd=1),
    dict(trace_mode=3, trace_loop=0, trace_lpb=4, trace_rnd=2),
    dict(trace_mode=3, trace_loop=0),
    # the default: two kernels, then one launch per stage once at most trace_tail lines are live
    dict(trace_mode=0, trace_tail=8),
    dict(trace_mode=0, trace_tail=16),
    dict(trace_mode=0, trace_tail=16, trace_loop=0),
], ids=["split2", "split4", "split8", "tile64", "tile128", "tile256", "split4_few8",
        "fused_l1r1", "fused_l2r4", "fused_l4r2", "fused_l8r4", "fused_l8r1", "fused_auto", "loop_auto", "loop_l2r2",
    "stage_l1r1", "stage_l4r2",
    "stage_auto", "tail8", "tail16", "tail16_stage"])
def test_trace_layouts(bem, layout):
    """Every tile shape of the two-kernel layout (the split far passes at 2, 4 and 8 waves per
    chunk, the unsplit ones at 64, 128 and 256 lines per block, the few-line tail) and of the
    one-launch layout (line slots and panel rounds per block) against the oracle on 16 coax lines (seed 21) that end on the shell or the ring or run out of
    steps: step counts and stop codes exact, integrals and paths 1e-10 / 1e-9."""
    p = coax_problem(0.012)
    _say(f"trace layout {layout}")
    c, o, x, x_ref = _sigma_case(bem, p)
    for k, v in layout.items():
        c.set_tuning(k, v)
    starts, _, _ = electrode_line_starts(p, 16, seed=21)
    kw = dict(h=1e-3, max_steps=200)
    sol = torch.tensor(x, device="cuda")
    I, ns, st, _ = c.streamer_integral(sol, starts, bem.trace_params(**kw))
    ns2, st2, path = c.trace_lines(sol, starts, bem.trace_params(**kw), want_path=True)
    I, ns, st, path = I.cpu().numpy(), ns.cpu().numpy(), st.cpu().numpy(), path.cpu().numpy()
    assert np.array_equal(ns, ns2.cpu().numpy()) and np.array_equal(st, st2.cpu().numpy())
    key = x.tobytes()
    if key not in _LAYOUT_REF:
        _LAYOUT_REF.clear()
        _LAYOUT_REF[key] = o.trace(x, starts, oracle.trace_params(**kw), want_path=True)
    nso, sto, Io, patho = _LAYOUT_REF[key]
    assert np.array_equal(ns, nso) and np.array_equal(st, sto)
    assert len(set(sto.tolist()) - {0}) >= 2
    assert np.abs(I - Io).max() <= 1e-10 * np.abs(Io).max()
    for l in range(len(starts)):
        m = ns[l] + 1
        assert np.abs(path[l, :m] - patho[l, :m]).max() <= 1e-9 * np.abs(patho[l, :m]).max()
    c.close()


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_trace_edge_cases(bem, mode):
    p = sphere_problem(2)
    _say(f"trace edge cases mode {mode}")
    c, o, x, x_ref = _sigma_case(bem, p)
    c.set_tuning("trace_mode", mode)
    sol = torch.tensor(x, device="cuda")
    starts, _, _ = electrode_line_starts(p, 3, seed=1)
    # one step
    ns, st, _ = c.trace_lines(sol, starts, bem.trace_params(h=1e-3, max_steps=1))
    assert np.all(ns.cpu().numpy() == 1) and np.all(st.cpu().numpy() == 0)
    # inward lines hit the sphere at once (stop 1, no step)
    ns, st, _ = c.trace_lines(sol, starts, bem.trace_params(h=1e-3, max_steps=5, direction=-1))
    assert np.all(ns.cpu().numpy() == 0) and np.all(st.cpu().numpy() == 1)
    # weak field: e_min above |E| everywhere -> stop 4 before the first step
    ns, st, _ = c.trace_lines(sol, starts, bem.trace_params(h=1e-3, max_steps=5, e_min=1e6))
    assert np.all(ns.cpu().numpy() == 0) and np.all(st.cpu().numpy() == 4)
    # no lines, no points
    ns, st, _ = c.trace_lines(sol, np.zeros((0, 3)), bem.trace_params(h=1e-3, max_steps=5))
    assert ns.numel() == 0
    phi, E = c.eval_field(sol, np.zeros((0, 3)))
    assert E.numel() == 0
    # step too long for the near radius is rejected before any launch
    with pytest.raises(bem.BemError):
        c.trace_lines(sol, starts, bem.trace_params(h=1.0, max_steps=5))
    c.close()


def test_error_paths(bem):
    _say("error paths")
    p = sphere_problem(1)
    # solve before assemble
    c = bem.Context.from_problem(p)
    with pytest.raises(bem.BemError) as e:
        c.solve(p.body_V)
    assert e.value.code == 6
    c.assemble()
    # max_iter = 1 does not converge: NOCONV with the iterate written
    sol, info = c.solve(p.body_V, tol=1e-14, max_iter=1, raise_on_noconv=False)
    assert not info["converged"] and info["iters"] == 1
    with pytest.raises(bem.BemError) as e:
        c.solve(p.body_V, tol=1e-14, max_iter=1)
    assert e.value.code == 5
    c.close()
    bad = p.tri.copy()
    bad[0, 1] = bad[0, 0]
    with pytest.raises(bem.BemError) as e:
        bem.Context(p.vert, bad, p.tri_body, p.body_kind, p.eps_plus, p.eps_minus)
    assert e.value.code in (1, 2)
    bad = p.tri.copy()
    bad[3, 2] = len(p.vert)
    with pytest.raises(bem.BemError) as e:
        bem.Context(p.vert, bad, p.tri_body, p.body_kind, p.eps_plus, p.eps_minus)
    assert e.value.code == 1
    v = p.vert.copy()
    v[5, 0] = np.nan
    with pytest.raises(bem.BemError) as e:
        bem.Context(v, p.tri, p.tri_body, p.body_kind, p.eps_plus, p.eps_minus)
    assert e.value.code == 1
    # collinear triangle
    v = p.vert.copy()
    t0 = p.tri[0]
    v[t0[2]] = 0.5 * (v[t0[0]] + v[t0[1]])
    with pytest.raises(bem.BemError) as e:
        bem.Context(v, p.tri, p.tri_body, p.body_kind, p.eps_plus, p.eps_minus)
    assert e.value.code == 2


def test_mixed_precision_sphere_and_coax(bem):
    for p in (sphere_problem(3), coax_problem(0.012)):
        _say(f"mixed {p.name}")
        o = oracle.Oracle(p)
        A = o.assemble()
        x_ref = np.linalg.solve(A, o.rhs(p.body_V))
        c = _ctx(bem, p, precision=bem.MIXED)
        sol, info = c.solve(p.body_V, tol=1e-8)
        assert info["converged"] and info["refinements"] >= 1
        x = sol[0].cpu().numpy()
        assert rel(x[:p.n_tri], x_ref[:p.n_tri]) <= 1e-5
        pts = sphere_eval_points(200) if p.name.startswith("sphere") else gap_eval_points(200)
        _, E_o = o.eval(x_ref, pts)
        _, E = c.eval_field(sol, pts)
        assert rel(np.linalg.norm(E[0].cpu().numpy(), axis=1), np.linalg.norm(E_o, axis=1)) <= 1e-5
        c.close()


def test_multi_rhs_linearity(bem):
    p = coax_problem(0.012)
    _say("multi rhs")
    c = _ctx(bem, p)
    bv = np.tile(p.body_V, (3, 1))
    bv[:, 1] = [0.5, 1.0, 2.0]
    sol, info = c.solve(bv, tol=1e-12)
    s = sol.cpu().numpy()
    assert rel(s[0], 0.5 * s[1]) <= 1e-10 and rel(s[2], 2.0 * s[1]) <= 1e-10
    c.close()


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_trace_multi_rhs_lines(bem, mode):
    # lines driven by different load cases (line_rhs), both trace layouts
    p = coax_problem(0.012)
    _say(f"multi-rhs lines mode {mode}")
    c = _ctx(bem, p)
    c.set_tuning("trace_mode", mode)
    bv = np.tile(p.body_V, (3, 1))
    bv[:, 1] = [0.7, 1.0, 1.6]
    sol, info = c.solve(bv, tol=1e-13, max_iter=20000)
    starts, _, _ = electrode_line_starts(p, 9, seed=11)
    line_rhs = np.array([0, 1, 2] * 3, dtype=np.int32)
    tp = bem.trace_params(h=1e-3, max_steps=60)
    I, ns, st, _ = c.streamer_integral(sol, starts, tp, line_rhs=line_rhs)
    o = oracle.Oracle(p)
    s_h = sol.cpu().numpy()
    for r in range(3):
        sel = np.nonzero(line_rhs == r)[0]
        nso, sto, Io = o.trace(s_h[r], starts[sel], oracle.trace_params(h=1e-3, max_steps=60))
        assert np.array_equal(ns.cpu().numpy()[sel], nso) and np.array_equal(st.cpu().numpy()[sel], sto)
        assert np.abs(I.cpu().numpy()[sel] - Io).max() <= 1e-10 * max(np.abs(Io).max(), 1e-300)
    c.close()


def test_trace_line_groups(bem):
    """Lines cut into two groups on two streams, folded into one when few lines remain.  With
    the pass layout fixed (chunked, or split, at every live count) a line's arithmetic does not
    depend on the grouping, so step counts, stop codes, integrals and paths are bitwise equal to
    the one-group run.  With the layout switching by live count, each group switches by its own
    count, which moves only the summation order: those runs are checked against the oracle."""
    p = coax_problem(0.012)
    _say("line groups")
    c, o, x, x_ref = _sigma_case(bem, p)
    c.set_tuning("trace_mode", 1)   # line groups belong to the two-kernel layout
    sol = torch.tensor(x, device="cuda")
    starts, _, _ = electrode_line_starts(p, 37, seed=4)
    params = dict(h=1e-3, max_steps=120)
    tp = bem.trace_params(**params)
    nso, sto, Io, patho = o.trace(x, starts, oracle.trace_params(**params), want_path=True)
    assert len(set(sto.tolist())) >= 2, "the case must stop lines in more than one way"

    def run(groups, few, split):
        c.set_tuning("trace_groups", groups)
        c.set_tuning("trace_few", few)
        c.set_tuning("trace_split", split)
        assert c.get_tuning("trace_groups") == groups
        I, ns, st, _ = c.streamer_integral(sol, starts, tp)
        ns2, st2, path = c.trace_lines(sol, starts, tp, want_path=True)
        got = [t.cpu().numpy() for t in (I, ns, st, ns2, st2, path)]
        assert np.array_equal(got[1], nso) and np.array_equal(got[2], sto), (groups, few, split)
        assert np.array_equal(got[3], nso) and np.array_equal(got[4], sto), (groups, few, split)
        assert np.abs(got[0] - Io).max() <= 1e-10 * np.abs(Io).max(), (groups, few, split)
        for l in range(len(starts)):
            m = nso[l] + 1
            assert np.abs(got[5][l, :m] - patho[l, :m]).max() <= 1e-9 * np.abs(patho[l, :m]).max()
        return got

    for split in (0, 4096):   # always chunked, always split
        ref = run(1, 0, split)
        got = run(2, 0, split)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b, equal_nan=True), split   # paths are NaN past a line's end
    for groups, few, split in [(2, 8, 16), (2, 16, 64), (2, 0, 64), (1, 8, 16)]:
        run(groups, few, split)
    c.close()


def test_batched_matvec_mfma(bem):
    # the multi-vector product on the matrix cores against the oracle matrix
    for prec in (bem.FP64, bem.MIXED):
        p = coax_problem(0.012)
        _say(f"batched matvec precision {prec}")
        o = oracle.Oracle(p)
        A = o.assemble()
        c = _ctx(bem, p, precision=prec)
        rng = np.random.default_rng(5)
        X = rng.standard_normal((37, c.n))
        Y = c.matvec(torch.tensor(X, device="cuda")).cpu().numpy()
        if prec == bem.FP64:
            assert rel(Y, X @ A.T) <= 1e-12
        else:
            G = c.copy_rows(0, c.n).cpu().numpy()       # the mixed operator itself
            assert rel(Y, X @ G.T) <= 1e-12
            assert rel(Y, X @ A.T) <= 1e-6
        c.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_solve_many_rhs(bem, prec):
    p = coax_problem(0.012)
    _say(f"batched solve {prec}")
    o = oracle.Oracle(p)
    A = o.assemble()
    rng = np.random.default_rng(4)
    nr = 70                                     # two groups: 64 + 6
    bv = np.tile(p.body_V, (nr, 1))
    bv[:, 1] = rng.uniform(0.5, 2.0, nr)        # rod potential
    bv[::3, 0] = rng.uniform(-0.5, 0.5, len(bv[::3]))   # some load cases also drive the shell (rank 2)
    X_ref = np.linalg.solve(A, np.stack([o.rhs(v) for v in bv]).T).T
    kw = dict(precision=bem.FP64) if prec == "fp64" else dict(precision=bem.MIXED)
    c = _ctx(bem, p, **kw)
    tol = 1e-13 if prec == "fp64" else 1e-8
    sol, info = c.solve(bv, tol=tol, max_iter=20000)
    assert info["converged"] and info["rel_residual"] <= tol
    S = sol.cpu().numpy()
    N = p.n_tri
    for r in range(nr):
        e = rel(S[r, :N], X_ref[r, :N])
        assert e <= (1e-10 if prec == "fp64" else 1e-5), (r, e)
    if prec == "mixed":
        assert info["refinements"] >= 1
    # the batched and one-by-one solvers agree
    c.set_tuning("batched_solve", 0)
    sol1, _ = c.solve(bv[:3], tol=tol, max_iter=20000)
    assert rel(sol1.cpu().numpy()[:, :N], S[:3, :N]) <= (1e-10 if prec == "fp64" else 1e-5)
    c.close()
