"""Failure paths of the C ABI on the GPU: out-of-memory detected before any
allocation, non-finite densities (stop code 5, non-finite fields), and
nrhs = 0 refused by every call that takes load cases.  Every case is forced
from the host; no kernel is made to fault."""

import ctypes
import sys

import numpy as np
import pytest

from workloads import electrode_line_starts, sphere_problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(f"[gpu-failures] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bem():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_12663_amd as bem
    return bem


def test_oom_before_any_allocation(bem):
    """A level-7 icosphere (327,680 panels) needs an 858 GB FP64 matrix (429 GB in FP32):
    bem_assemble returns OOM from its size check, device memory is unchanged, and the
    context stays unassembled (a solve is a STATE error)."""
    p = sphere_problem(7)
    _say(f"oom: sphere L7 N={p.n_tri}")
    for prec in (bem.FP64, bem.MIXED):
        c = bem.Context.from_problem(p, precision=prec)
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        with pytest.raises(bem.BemError) as e:
            c.assemble()
        assert e.value.code == 3, e.value
        assert "MiB" in str(e.value)
        free1, _ = torch.cuda.mem_get_info()
        assert abs(free1 - free0) <= (64 << 20), (free0, free1)
        with pytest.raises(bem.BemError) as e:
            c.solve(p.body_V)
        assert e.value.code == 6
        c.close()


def test_nonfinite_density(bem):
    """A NaN in sigma: the field at every point is non-finite (each sums over all panels) and
    every field line stops before its first step with code 5, in both line layouts and in
    the few-line pass."""
    p = sphere_problem(2, V0=50.0)
    _say("nonfinite density")
    c = bem.Context.from_problem(p)
    c.assemble()
    sol, _ = c.solve(p.body_V, tol=1e-12)
    bad = sol.clone()
    bad[0, 7] = float("nan")
    pts = np.array([[2.0, 0.1, 0.3], [0.0, -1.7, 0.4], [0.5, 0.5, 2.5]])
    phi, E = c.eval_field(bad, pts)
    assert not torch.isfinite(phi).any() and not torch.isfinite(E).any()
    starts, _, _ = electrode_line_starts(p, 12, seed=6)
    tp = bem.trace_params(h=1e-3, max_steps=20)
    for mode in (1, 2, 3):
        c.set_tuning("trace_mode", mode)
        for few in ((0, 16) if mode == 1 else (0,)):
            c.set_tuning("trace_few", few)
            I, ns, st, _ = c.streamer_integral(bad, starts, tp)
            assert np.all(st.cpu().numpy() == 5), (mode, few, st)
            assert np.all(ns.cpu().numpy() == 0)
    # the same lines with the finite solution run their 20 steps
    c.set_tuning("trace_mode", 0)
    I, ns, st, _ = c.streamer_integral(sol, starts, tp)
    assert np.all(st.cpu().numpy() == 0) and np.all(ns.cpu().numpy() == 20)
    c.close()


def test_zero_load_cases_refused(bem):
    """nrhs = 0 is INVALID for every call that takes load cases, checked on the host."""
    from paper_2003_12663_amd import _lib
    p = sphere_problem(1)
    _say("nrhs = 0")
    c = bem.Context.from_problem(p)
    c.assemble()
    lib, h = c.lib, c._ctx
    sol, _ = c.solve(p.body_V)
    x = torch.zeros((1, c.n), dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    pts = torch.tensor([[2.0, 0.0, 0.0]], dtype=torch.float64, device="cuda")
    E = torch.zeros((1, 3), dtype=torch.float64, device="cuda")
    phi = torch.zeros(1, dtype=torch.float64, device="cuda")
    ns = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    I = torch.zeros(1, dtype=torch.float64, device="cuda")
    bv = np.ascontiguousarray(p.body_V, dtype=np.float64)
    info = _lib.SolveInfo()
    tp = bem.trace_params(h=1e-3, max_steps=5)
    P = lambda t: ctypes.c_void_p(t.data_ptr())
    calls = {
        "bem_rhs": lambda: lib.bem_rhs(h, 0, bv.ctypes.data, P(y)),
        "bem_matvec": lambda: lib.bem_matvec(h, 0, P(x), P(y), 0),
        "bem_solve_gmres": lambda: lib.bem_solve_gmres(h, 0, bv.ctypes.data, 1e-8, 100, P(y), ctypes.byref(info)),
        "bem_eval_field": lambda: lib.bem_eval_field(h, 0, P(sol), 1, P(pts), None, P(phi), P(E)),
        "bem_trace_lines": lambda: lib.bem_trace_lines(h, 0, P(sol), 1, None, P(pts), ctypes.byref(tp), P(ns),
                                                        P(st), None),
        "bem_streamer_integral": lambda: lib.bem_streamer_integral(h, 0, P(sol), 1, None, P(pts), ctypes.byref(tp),
                                                                    P(I), P(ns), P(st), None),
    }
    for name, call in calls.items():
        assert call() == _lib.BEM_ERR_INVALID, name
        assert b"nrhs" in lib.bem_last_error(), name
    c.close()
