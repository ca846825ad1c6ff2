"""The compressed operator (bem_compress: hierarchical matrix with adaptive cross
approximation, the outlook of Sec. 6) against the oracle's dense matrix, through
the C ABI:
- with no admissible pair (eta_adm tiny) every block is a dense leaf block, so the
  product equals the dense matrix's to rounding (1e-12 of the largest entry of y):
  this checks the cluster order, the block tree, the floating columns and the
  constraint rows;
- at eps = 1e-8 and 1e-5 the product's error against the oracle matrix on random
  vectors (relative 2-norm) stays below 10 eps, and falls with eps; the coax's flat
  spacer faces hold whole blocks of interface rows that vanish against panels in
  their own plane, the case where cross approximation with plain partial pivoting
  stops early (it left 1.3e-4 at eps = 1e-5);
- GMRES on the compressed operator reaches the oracle LU solution to 100 eps;
- on the 19,732-panel coax against the dense GPU operator (itself parity-tested
  against sampled oracle rows): product and solution within 100 eps, with fewer
  than half the dense matrix's entries stored."""

import sys

import numpy as np
import pytest

import oracle
from workloads import coax_problem, coax_problem_for_size, sphere_problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(msg):
    print(f"[gpu-hmatrix] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bem():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_12663_amd as bem
    return bem


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("case", ["sphere", "coax"])
def test_all_dense_blocks_equal_the_dense_matrix(bem, case):
    p = sphere_problem(3) if case == "sphere" else coax_problem(0.012)
    A = oracle.Oracle(p).assemble()
    with bem.Context.from_problem(p) as c:
        info = c.compress(eps=1e-8, eta_adm=1e-9, leaf=32)
        assert info["lowrank_blocks"] == 0 and info["dense_entries"] == p.n_tri * p.n_tri
        X = np.random.default_rng(3).standard_normal((2, c.n))
        Y = c.matvec(torch.tensor(X, device="cuda")).cpu().numpy()
    Yr = X @ A.T
    err = np.abs(Y - Yr).max() / np.abs(Yr).max()
    _say(f"{case} N={p.n_tri}: all-dense compressed product vs oracle {err:.2e}")
    assert err <= 1e-12, err


@pytest.mark.parametrize("case", ["sphere", "coax"])
def test_compressed_product_and_solution(bem, case):
    p = sphere_problem(4) if case == "sphere" else coax_problem(0.008)
    o = oracle.Oracle(p)
    A = o.assemble()
    b = o.rhs(p.body_V)
    x_ref = np.linalg.solve(A, b)
    X = np.random.default_rng(4).standard_normal((2, A.shape[0]))
    errs = {}
    for eps in (1e-5, 1e-8):
        with bem.Context.from_problem(p) as c:
            info = c.compress(eps=eps, eta_adm=1.0, leaf=32)
            Y = c.matvec(torch.tensor(X, device="cuda")).cpu().numpy()
            e_prod = max(_rel(Y[k], A @ X[k]) for k in range(2))
            sol, sinfo = c.solve(p.body_V, tol=1e-12, max_iter=5000)
            e_sol = _rel(sol[0].cpu().numpy(), x_ref)
        stored = info["dense_entries"] + info["factor_entries"]
        _say(f"{case} N={p.n_tri} eps={eps:g}: product {e_prod:.2e}, solution {e_sol:.2e}, "
             f"stored {stored / p.n_tri ** 2:.3f} of dense, {info['lowrank_blocks']} low-rank blocks, "
             f"max rank {info['max_rank']}, {sinfo['iters']} iterations")
        assert sinfo["converged"]
        assert e_prod <= 10 * eps and e_sol <= 100 * eps, (eps, e_prod, e_sol)
        assert info["lowrank_blocks"] > 0
        errs[eps] = e_prod
    assert errs[1e-8] < errs[1e-5]


def test_compressed_at_full_size(bem):
    p = coax_problem_for_size(20000)
    X = torch.tensor(np.random.default_rng(5).standard_normal((1, p.n_tri + 1)), device="cuda")
    with bem.Context.from_problem(p) as c:
        c.assemble()
        Yd = c.matvec(X).cpu().numpy()
        sd, _ = c.solve(p.body_V, tol=1e-12, max_iter=5000)
        sd = sd[0].cpu().numpy()
        info = c.compress(eps=1e-8, eta_adm=1.0, leaf=64)
        Yc = c.matvec(X).cpu().numpy()
        sc, sinfo = c.solve(p.body_V, tol=1e-12, max_iter=5000)
        sc = sc[0].cpu().numpy()
    stored = info["dense_entries"] + info["factor_entries"]
    e_prod, e_sol = _rel(Yc[0], Yd[0]), _rel(sc, sd)
    _say(f"coax N={p.n_tri}: product {e_prod:.2e}, solution {e_sol:.2e}, stored {stored / p.n_tri ** 2:.3f} "
         f"of dense, max rank {info['max_rank']}")
    assert e_prod <= 1e-6 and e_sol <= 1e-6
    assert stored < 0.5 * p.n_tri ** 2


def test_compressed_refusals(bem):
    p = sphere_problem(2)
    with bem.Context.from_problem(p, precision=bem.MIXED) as c:
        with pytest.raises(bem.BemError):
            c.compress()
    with bem.Context.from_problem(p) as c:
        for kw in (dict(eps=0.0), dict(eps=1.0), dict(eta_adm=-1.0), dict(leaf=4), dict(leaf=512)):
            with pytest.raises(bem.BemError):
                c.compress(**kw)
        c.compress()
        x = torch.zeros((1, c.n), dtype=torch.float64, device="cuda")
        with pytest.raises(bem.BemError):
            c.matvec(x, transpose=True)
        with pytest.raises(bem.BemError):
            c.copy_rows(0, 1)
        c.assemble()                       # back to the dense operator
        assert c.copy_rows(0, 1).shape == (1, c.n)
