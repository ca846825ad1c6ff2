"""Nodal rows that need the normal field n . E on the GPU against the FP64 oracle:
interface vertices (Eq. nonconductors / Final3), the literal floating-body row
(Eq. Final4, constraint_form 0) and thin sheets (Eq. sheets).  A vertex of flat
panels has no normal, so these rows are the hat-weighted mean of the condition
over the centroids of the triangles around the vertex (or of the body), each
with its triangle's normal; the oracle pins this reading against closed forms.
Bars as for the rest of the nodal basis: matrix entries 1e-12 of the row's
largest, right-hand sides exact, solutions and fields 1e-10.  Cases: the coated
sphere, the floating shell with the literal row, the sphere with a thin sheet,
and the coax with its spacer disc (rim vertices coincide with vertices of the
rod and the shell) in both constraint forms; MIXED storage of the coax with
disc against FP64; field lines of the coax with disc against the oracle's."""

import numpy as np
import pytest

import oracle
from workloads import coated_sphere_problem, coax_problem, floating_shell_problem
from workloads.meshes import sphere_sheet_problem

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


CASES = [
    ("coated_sphere_L2", lambda: coated_sphere_problem(2), 0),
    ("floating_shell_L2_literal", lambda: floating_shell_problem(2, V0=3.0), 0),
    ("sphere_sheet_L2", lambda: sphere_sheet_problem(2), 0),
    ("coax_disc_literal", lambda: coax_problem(0.03), 0),
    ("coax_disc_net_charge", lambda: coax_problem(0.02), 1),
]


@pytest.mark.parametrize("name,make,form", CASES, ids=[c[0] for c in CASES])
def test_nodal_normal_field_rows(bem, name, make, form):
    p = make()
    o = oracle.Oracle(p, constraint_form=form)
    A = o.p1_assemble()
    b_ref = o.p1_rhs(p.body_V)
    x_ref = np.linalg.solve(A, b_ref)
    c = bem.Context.from_problem(p, basis=bem.BASIS_LINEAR, constraint_form=form)
    c.assemble()
    print(f"[nodal-iface] {name}: n_vert {p.n_vert}, n {c.n}", flush=True)
    assert c.n == A.shape[0]
    G = c.copy_rows(0, c.n).cpu().numpy()
    err = (np.abs(G - A) / np.abs(A).max(axis=1, keepdims=True)).max()
    print(f"[nodal-iface] {name}: matrix {err:.2e}", flush=True)
    assert err <= 1e-12
    b = c.rhs(p.body_V)[0].cpu().numpy()
    assert np.array_equal(b, b_ref)
    sol, info = c.solve(p.body_V, tol=1e-13, max_iter=5000)
    assert info["converged"]
    assert rel(sol[0].cpu().numpy(), x_ref) <= 1e-10
    rng = np.random.default_rng(7)
    lo, hi = p.vert.min(axis=0), p.vert.max(axis=0)
    pts = rng.uniform(lo - 0.3 * (hi - lo), hi + 0.3 * (hi - lo), (40, 3))
    _, E = c.eval_field(sol, pts)
    _, E_ref = o.p1_field(sol[0].cpu().numpy(), pts)
    assert rel(E[0].cpu().numpy(), E_ref) <= 1e-10
    c.close()


def test_nodal_coax_disc_mixed(bem):
    """MIXED storage (FP32 vertex rows, interface rows included; FP64 constraint rows)
    solved inside FP64 refinement: solution within 1e-5 of FP64."""
    p = coax_problem(0.012)
    c64 = bem.Context.from_problem(p, basis=bem.BASIS_LINEAR, constraint_form=0)
    c64.assemble()
    s64, _ = c64.solve(p.body_V, tol=1e-12, max_iter=5000)
    c32 = bem.Context.from_problem(p, basis=bem.BASIS_LINEAR, constraint_form=0, precision=bem.MIXED)
    c32.assemble()
    s32, info = c32.solve(p.body_V, tol=1e-10, max_iter=5000)
    e = rel(s32[0].cpu().numpy(), s64[0].cpu().numpy())
    print(f"[nodal-iface] coax disc MIXED vs FP64: {e:.2e} ({info['refinements']} refinements)", flush=True)
    assert info["converged"] and e <= 1e-5
    c64.close()
    c32.close()


def test_nodal_coax_disc_field_lines(bem):
    """Lines from the rod of the coax with disc (nodal basis): step counts and stop codes
    exact against the oracle's lines (some end on the disc, code 3), integrals 1e-10."""
    from workloads import electrode_line_starts
    p = coax_problem(0.02, V0=40.0)
    o = oracle.Oracle(p, constraint_form=0)
    u_ref = np.linalg.solve(o.p1_assemble(), o.p1_rhs(p.body_V))
    c = bem.Context.from_problem(p, basis=bem.BASIS_LINEAR, constraint_form=0)
    c.assemble()
    sol, _ = c.solve(p.body_V, tol=1e-13, max_iter=5000)
    assert rel(sol[0].cpu().numpy(), u_ref) <= 1e-10
    starts, _, _ = electrode_line_starts(p, 24, seed=4)
    kw = dict(h=2e-3, max_steps=200, e_min=1e-3, alpha_a=1e-3, alpha_e0=25.0, alpha_p=2.0)
    ns_o, st_o, I_o = o.p1_trace(sol[0].cpu().numpy(), starts, oracle.trace_params(**kw))
    I, ns, st, _ = c.streamer_integral(sol, torch.tensor(starts, device="cuda"), bem.trace_params(**kw))
    ns, st, I = ns.cpu().numpy(), st.cpu().numpy(), I.cpu().numpy()
    print(f"[nodal-iface] coax disc lines: stop codes {np.bincount(st, minlength=6)}", flush=True)
    assert np.array_equal(ns, ns_o) and np.array_equal(st, st_o)
    assert np.max(np.abs(I - I_o)) <= 1e-10 * max(np.max(np.abs(I_o)), 1e-300)
    c.close()
