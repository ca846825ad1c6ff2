"""Thin floating sheets (Eq. sheets) on the GPU against the FP64 oracle.

A sheet is one open surface with an unknown potential; its constraint row is the
net charge over both sides.  Cases: a conductor sphere inside a floating
spherical sheet between two dielectrics (closed form in the oracle pins) and a
bushing-like device (a rod in an insulator, five graded coaxial foils, the
outermost grounded).  Bars as in test_gpu_parity: matrix entries 1e-12 of the
row's largest, sigma and potentials 1e-10, field-line step counts and stop codes
exact, integrals 1e-10; mixed precision 1e-5 against FP64.
"""

import numpy as np
import pytest

import oracle
from workloads import bushing_problem, electrode_line_starts, sphere_sheet_problem

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


@pytest.mark.parametrize("eps_in", [4.0, 1.0])
@pytest.mark.parametrize("form", [0, 1])
def test_sphere_sheet_matrix_and_solution(bem, eps_in, form):
    p = sphere_sheet_problem(2, eps_in=eps_in)
    o = oracle.Oracle(p, constraint_form=form)
    A = o.assemble()
    x_ref = np.linalg.solve(A, o.rhs(p.body_V))
    c = bem.Context.from_problem(p, constraint_form=form)
    c.assemble()
    G = c.copy_rows(0, c.n).cpu().numpy()
    assert G.shape == A.shape
    assert (np.abs(G - A) / np.abs(A).max(axis=1, keepdims=True)).max() <= 1e-12
    sol, info = c.solve(p.body_V, tol=1e-13, max_iter=5000)
    x = sol[0].cpu().numpy()
    assert rel(x, x_ref) <= 1e-10
    N = p.n_tri
    print(f"[sheets] eps_in {eps_in} form {form}: V_sheet {x[N]:.6f} (oracle {x_ref[N]:.6f})", flush=True)
    c.close()


def _bushing(bem, h=0.02, precision=None):
    p = bushing_problem(h)
    kw = {} if precision is None else {"precision": precision}
    c = bem.Context.from_problem(p, **kw)
    c.assemble()
    return p, c


def test_bushing_against_oracle(bem):
    p, c = _bushing(bem)
    o = oracle.Oracle(p)
    A = o.assemble()
    x_ref = np.linalg.solve(A, o.rhs(p.body_V))
    G = c.copy_rows(0, c.n).cpu().numpy()
    assert (np.abs(G - A) / np.abs(A).max(axis=1, keepdims=True)).max() <= 1e-12
    sol, info = c.solve(p.body_V, tol=1e-13, max_iter=20000)
    x = sol[0].cpu().numpy()
    assert rel(x, x_ref) <= 1e-10
    N = p.n_tri
    V = x[N:N + 4]
    print(f"[sheets] bushing N={N}: floating foil potentials {np.round(V, 5).tolist()} (GMRES {info['iters']})",
          flush=True)
    # field grading: the floating foils lie between the rod (1) and the grounded foil (0), outermost lowest
    assert np.all(np.diff(V) < 0) and V[0] < 1.0 and V[-1] > 0.0
    # field lines from the rod: stop codes and integrals against the oracle (lines end on foils)
    starts, _, _ = electrode_line_starts(p, 12, seed=3)
    params = dict(h=1e-3, max_steps=150, e_min=1e-6)
    I, ns, st, _ = c.streamer_integral(sol, starts, bem.trace_params(**params))
    nso, sto, Io = o.trace(x_ref, starts, oracle.trace_params(**params))
    assert np.array_equal(ns.cpu().numpy(), nso) and np.array_equal(st.cpu().numpy(), sto)
    assert np.abs(I.cpu().numpy() - Io).max() <= 1e-10 * max(np.abs(Io).max(), 1e-300)
    assert (sto == 2).any(), "some line must end on a floating foil"
    c.close()


def test_bushing_mixed_precision(bem):
    p, c64 = _bushing(bem)
    s64, _ = c64.solve(p.body_V, tol=1e-12, max_iter=20000)
    p, c32 = _bushing(bem, precision=bem.MIXED)
    s32, info = c32.solve(p.body_V, tol=1e-8, max_iter=20000)
    assert rel(s32.cpu().numpy(), s64.cpu().numpy()) <= 1e-5
    c64.close()
    c32.close()
