"""bem_matvec_noalloc (the product without device allocation) against bem_matvec,
both called through the C ABI on the same inputs: two calls in a row, the second
on a smaller problem (the work array keeps the first call's contents), for A x and
A^T x in FP64 and A x in MIXED precision.  The one-vector calls run the same
kernels in the same order, so they agree bit for bit; several vectors against the
batched matrix-core product of bem_matvec agree to FP64 rounding (1e-12 of the
largest entry, the FP64 bar is 1e-10).  Also checked: the size limit and the
transposed product in MIXED precision are refused before any work."""

import ctypes
import sys

import numpy as np
import pytest

from workloads import coax_problem, sphere_problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(f"[no-alloc] {msg}", flush=True)
    sys.stdout.flush()


def _call(c, fn, x, transpose):
    y = torch.full_like(x, float("nan"))
    rc = fn(c._ctx, x.shape[0], ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), int(transpose))
    assert rc == 0, c.lib.bem_last_error().decode()
    torch.cuda.synchronize()
    return y.cpu().numpy()


def _compare(c, nrhs, transpose, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    x = torch.randn((nrhs, c.n), generator=g, dtype=torch.float64).to(c.device)
    ref = _call(c, c.lib.bem_matvec, x, transpose)
    out = _call(c, c.lib.bem_matvec_noalloc, x, transpose)
    assert np.isfinite(out).all()
    if nrhs == 1:
        assert np.array_equal(out, ref), np.abs(out - ref).max()
    else:
        scale = np.abs(ref).max(axis=1, keepdims=True)
        assert (np.abs(out - ref) / scale).max() <= 1e-12


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_matches_matvec_two_calls(precision):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_12663_amd as bem
    prec = bem.FP64 if precision == "fp64" else bem.MIXED
    big = coax_problem(0.012)          # rod, shell, floating ring, spacer disc: n = N + 1
    small = sphere_problem(2)          # 320 panels
    for p, nrhs, seed in ((big, 3, 11), (small, 1, 12)):
        _say(f"{precision} N={p.n_tri} nrhs={nrhs}")
        with bem.Context.from_problem(p, precision=prec) as c:
            c.assemble()
            c.set_tuning("batched_solve", 1)
            _compare(c, 1, False, seed)
            _compare(c, nrhs, False, seed + 100)
            if prec == bem.FP64:
                _compare(c, 1, True, seed + 200)
                _compare(c, nrhs, True, seed + 300)
            else:
                x = torch.zeros((1, c.n), dtype=torch.float64, device=c.device)
                y = torch.zeros_like(x)
                rc = c.lib.bem_matvec_noalloc(c._ctx, 1, ctypes.c_void_p(x.data_ptr()),
                                              ctypes.c_void_p(y.data_ptr()), 1)
                assert rc == 1   # INVALID: no FP64 copy of the far entries to transpose


def test_noalloc_refuses_above_its_limit():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_12663_amd as bem
    p = sphere_problem(6)              # 81,920 panels: above the 65,536 unknowns of the work array
    _say(f"limit N={p.n_tri}")
    with bem.Context.from_problem(p) as c:
        x = torch.zeros((1, c.n), dtype=torch.float64, device=c.device)
        y = torch.zeros_like(x)
        rc = c.lib.bem_matvec_noalloc(c._ctx, 1, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), 0)
        assert rc == 1 and b"65536" in c.lib.bem_last_error()
