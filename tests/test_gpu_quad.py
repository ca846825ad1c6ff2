"""GPU parity of the near-singular rule on curved quadratic panels (bem_quad_pair_integrals,
Sec. 3 curved panels, Sec. 4 closest point + subdivision + Duffy) against the oracle's
implementation of the same rule (orc_quad_duffy, pinned in test_oracle_quad.py): curved
patches at distances from 1e-6 to 2 panel sizes and on the panel, flat panels against the
flat rule and the closed forms, a sphere of quadratic panels, and the refusals."""

import math

import numpy as np
import pytest

import oracle
from quad_cases import curved_patch, flat_nodes, near_points, qmap, quad_sphere
from workloads import sphere_problem

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def bem():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_12663_amd as bem
    return bem


@pytest.fixture(scope="module")
def ctx(bem):
    p = sphere_problem(1)
    c = bem.Context.from_problem(p)
    yield c
    c.close()


def _say(msg):
    print(f"[quad] {msg}", flush=True)


@pytest.mark.parametrize("dmin,dmax,bar", [(1e-3, 2.0, 1e-12), (1e-6, 1e-3, 1e-12)])
def test_quad_rule_against_oracle(ctx, dmin, dmax, bar):
    """Both sides take the same steps and differ only in rounding (the GPU contracts
    multiply-adds)."""
    rng = np.random.default_rng(31 + int(-math.log10(dmin)))
    pts, nodes = [], []
    for seed in range(16):
        P, L, n = curved_patch(300 + seed, bulge=0.1 + 0.02 * (seed % 5))
        for x in near_points(P, L, n, rng, 8, dmin, dmax):
            pts.append(x)
            nodes.append(P)
    pts, nodes = np.array(pts), np.array(nodes)
    _say(f"{len(pts)} curved pairs at {dmin:g}..{dmax:g} panel sizes")
    S, F = ctx.quad_pair_integrals(pts, nodes)
    worst = 0.0
    for k in range(len(pts)):
        So, Fo = oracle.quad_duffy(pts[k], nodes[k])
        worst = max(worst, abs(S[k] - So) / abs(So), np.abs(F[k] - Fo).max() / np.abs(Fo).max())
    _say(f"worst {worst:.2e}")
    assert worst <= bar, worst


def test_quad_rule_on_the_panel(ctx):
    """Points on curved panels (the singular pair): S against the oracle, F not formed (NaN)."""
    rng = np.random.default_rng(32)
    pts, nodes = [], []
    for seed in range(10):
        P, L, n = curved_patch(400 + seed)
        for _ in range(4):
            st = rng.dirichlet(np.ones(3))[:2]
            pts.append(qmap(P, st[0], st[1]))
            nodes.append(P)
    pts, nodes = np.array(pts), np.array(nodes)
    S, F = ctx.quad_pair_integrals(pts, nodes)
    for k in range(len(pts)):
        So, _ = oracle.quad_duffy(pts[k], nodes[k])
        assert abs(S[k] - So) <= 1e-12 * abs(So), (k, S[k], So)
    assert np.all(np.isnan(F))


def test_quad_flat_panels_against_flat_rule(ctx, bem):
    """Flat panels with mid-edge nodes (affine map): the curved kernel against the flat
    closed forms of the flat triangle (and the flat rule's pin, 1e-10)."""
    rng = np.random.default_rng(33)
    pts, nodes, tris = [], [], []
    for seed in range(12):
        v = rng.standard_normal((3, 3))
        L = max(np.linalg.norm(v[1] - v[0]), np.linalg.norm(v[2] - v[1]), np.linalg.norm(v[0] - v[2]))
        n = np.cross(v[1] - v[0], v[2] - v[0])
        n /= np.linalg.norm(n)
        for x in near_points(flat_nodes(v), L, n, rng, 6, 1e-5, 2.0):
            pts.append(x)
            nodes.append(flat_nodes(v))
            tris.append(v)
    S, F = ctx.quad_pair_integrals(np.array(pts), np.array(nodes))
    for k in range(len(pts)):
        Sa, Fa = oracle.tri_analytic(pts[k], *tris[k])
        assert abs(S[k] - Sa) <= 1e-10 * abs(Sa)
        assert np.abs(F[k] - Fa).max() <= 1e-10 * np.abs(Fa).max()


def test_quad_sphere(ctx):
    """Unit sphere of 320 quadratic panels, unit density: the GPU's sums against the oracle's
    (1e-12) and the closed forms (S = 1, F = 0 inside; 1/r, x/r^3 outside) to the panels'
    geometric error (5e-5 at this level)."""
    Q = quad_sphere(2)
    for x in (np.array([0.2, -0.1, 0.35]), np.array([0.8, 1.1, -0.4]), np.array([0.0, 0.0, 0.97])):
        S, F = ctx.quad_pair_integrals(np.tile(x, (len(Q), 1)), Q)
        So = Fo = 0.0
        for P in Q:
            s, f = oracle.quad_duffy(x, P)
            So = So + s
            Fo = Fo + f
        assert abs(S.sum() - So) <= 1e-12 * abs(So)
        assert np.abs(F.sum(axis=0) - Fo).max() <= 1e-12 * max(np.abs(Fo).max(), 1.0)
        r = np.linalg.norm(x)
        Se, Fe = (1.0, np.zeros(3)) if r < 1 else (1.0 / r, x / r ** 3)
        if r < 0.95:
            assert abs(S.sum() - Se) <= 5e-5 * Se


def test_quad_refusals(ctx, bem):
    P, L, n = curved_patch(500)
    x = np.array([[0.0, 0.0, 3.0]])
    S, F = ctx.quad_pair_integrals(np.zeros((0, 3)), np.zeros((0, 6, 3)))
    assert S.shape == (0,)
    bad = P.copy()[None]
    bad[0, 4, 1] = float("nan")
    with pytest.raises(bem.BemError):
        ctx.quad_pair_integrals(x, bad)
    flat = np.repeat(P[:1], 6, axis=0)[None]   # all nodes at one point: no area
    with pytest.raises(bem.BemError):
        ctx.quad_pair_integrals(x, flat)
    with pytest.raises(bem.BemError):
        ctx.quad_pair_integrals(np.array([[np.inf, 0.0, 0.0]]), P[None])
    S, F = ctx.quad_pair_integrals(x, P[None], want_F=False)
    assert F is None and np.isfinite(S).all()
