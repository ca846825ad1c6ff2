"""Pins of the oracle's near-singular rule on curved quadratic panels (Sec. 3: piecewise
quadratic parametrization of curved triangles; Sec. 4: closest point, subdivision so that
it is a corner, Duffy transformation), which the GPU kernel for curved panels is checked
against.  Pinned to things other than itself:
- the closest point against a dense sampling of the curved patch;
- a flat panel with its edge nodes at the edge midpoints (an affine map) against the flat
  rule and the flat closed forms;
- a flat triangle with its edge nodes moved along the edges (the same flat triangle under a
  non-affine quadratic map) against the flat closed forms: the Jacobian and the closest-point
  search in a non-affine map;
- curved patches against an independent brute force (adaptive subdivision of the parameter
  triangle with a tensor Gauss-Legendre rule on well-separated pieces, in numpy);
- F = -grad S by central differences;
- the unit sphere built from quadratic panels: the potential and field of a unit surface
  density inside (1, 0) and outside (1/r, x/r^3), converging as the panels refine."""

import math

import numpy as np
import pytest

from quad_cases import curved_patch as _curved_patch, flat_nodes as _flat_nodes, near_points as _near_points
from quad_cases import qmap as _qmap, quad_sphere as _quad_sphere


def _qjac(P, s, t):
    """|y_s x y_t| of the quadratic map, from the derivatives of its shape functions."""
    l1 = 1.0 - s - t
    z = np.zeros_like(s)
    Ns = np.stack([-(4 * l1 - 1), 4 * s - 1, z, 4 * (l1 - s), 4 * t, -4 * t], -1)
    Nt = np.stack([-(4 * l1 - 1), z, 4 * t - 1, -4 * s, 4 * s, 4 * (l1 - t)], -1)
    return np.linalg.norm(np.cross(Ns @ P, Nt @ P), axis=-1)


def _gl(n):
    z, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (z + 1.0), 0.5 * w


def _brute(x, P, ratio=0.15, nq=10):
    """S, F of unit density on the quadratic panel at x (x off the panel) by adaptive midpoint
    subdivision of the reference triangle: a piece is integrated once its mapped size is at most
    `ratio` times its distance to x, with nq x nq Gauss-Legendre nodes on the square collapsed
    onto it (its own corner 0 as apex)."""
    t_, w_ = _gl(nq)
    U, V = np.meshgrid(t_, t_, indexing="ij")
    W = np.outer(w_, w_)
    todo = np.array([[[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]]])
    S = 0.0
    F = np.zeros(3)
    while len(todo):
        a, b, c = todo[:, 0], todo[:, 1], todo[:, 2]
        pts = np.stack([a, b, c, 0.5 * (a + b), 0.5 * (b + c), 0.5 * (c + a)], 1)   # (m, 6, 2)
        Y = _qmap(P, pts[..., 0], pts[..., 1])                                      # (m, 6, 3)
        diam = np.max(np.linalg.norm(Y[:, :, None] - Y[:, None, :], axis=-1), axis=(1, 2))
        dist = np.min(np.linalg.norm(Y - x, axis=-1), axis=1) - 0.5 * diam
        ok = diam <= ratio * np.maximum(dist, 0.0)
        for k in np.nonzero(ok)[0]:
            ca, cb, cc = todo[k]
            # collapsed square: corner 0 + u ((1 - v)(b - a) + v (c - a)), Jacobian u |det|
            det = abs((cb[0] - ca[0]) * (cc[1] - ca[1]) - (cb[1] - ca[1]) * (cc[0] - ca[0]))
            s = ca[0] + U * ((1 - V) * (cb[0] - ca[0]) + V * (cc[0] - ca[0]))
            t = ca[1] + U * ((1 - V) * (cb[1] - ca[1]) + V * (cc[1] - ca[1]))
            y = _qmap(P, s, t)
            r = x - y
            R = np.linalg.norm(r, axis=-1)
            jw = U * det * _qjac(P, s, t) * W
            S += np.sum(jw / R)
            F += np.einsum("ij,ijk->k", jw / R ** 3, r)
        split = todo[~ok]
        if len(split) == 0:
            break
        a, b, c = split[:, 0], split[:, 1], split[:, 2]
        ab, bc, ca = 0.5 * (a + b), 0.5 * (b + c), 0.5 * (c + a)
        todo = np.concatenate([np.stack(q, 1) for q in ([a, ab, ca], [ab, b, bc], [ca, bc, c], [bc, ca, ab])])
    return S / (4 * math.pi), F / (4 * math.pi)


def test_quad_closest_against_sampling(oracle_mod):
    rng = np.random.default_rng(2)
    g = np.linspace(0.0, 1.0, 161)
    S, T = np.meshgrid(g, g, indexing="ij")
    m = S + T <= 1.0 + 1e-12
    S, T = S[m], np.clip(T[m], 0.0, 1.0 - S[m])
    for seed in range(12):
        P, L, n = _curved_patch(seed, bulge=0.25)
        Y = _qmap(P, S, T)
        for x in _near_points(P, L, n, rng, 8, 1e-3, 1.5):
            c = oracle_mod.quad_closest(x, P)
            assert c.min() >= 0.0 and c.sum() <= 1.0 + 1e-14
            dc = np.linalg.norm(x - _qmap(P, c[0], c[1]))
            dmin = np.linalg.norm(Y - x, axis=1).min()
            # no sample is closer, and the sampling's own resolution bounds the gap
            assert dc <= dmin + 1e-12 and dmin - dc <= 2.0 * L / 160.0


def test_quad_flat_affine_is_the_flat_rule(oracle_mod):
    """Edge nodes at the edge midpoints: the map is affine and the curved rule is the flat one,
    up to where each puts the closest point (the flat rule by the foot point in closed form, the
    curved one by Newton's method in the parameter plane), which moves the graded cells by
    rounding and the result within the rule's own accuracy."""
    rng = np.random.default_rng(5)
    worst_rule = worst_cf = 0.0
    for seed in range(20):
        v = rng.standard_normal((3, 3))
        P = _flat_nodes(v)
        L = max(np.linalg.norm(v[1] - v[0]), np.linalg.norm(v[2] - v[1]), np.linalg.norm(v[0] - v[2]))
        n = np.cross(v[1] - v[0], v[2] - v[0])
        n /= np.linalg.norm(n)
        for x in _near_points(P, L, n, rng, 10, 1e-6, 2.0):
            S, F = oracle_mod.quad_duffy(x, P)
            Sf, Ff = oracle_mod.tri_duffy(x, *v)
            Sa, Fa = oracle_mod.tri_analytic(x, *v)
            worst_rule = max(worst_rule, abs(S - Sf) / abs(Sf), np.abs(F - Ff).max() / np.abs(Ff).max())
            worst_cf = max(worst_cf, abs(S - Sa) / abs(Sa), np.abs(F - Fa).max() / np.abs(Fa).max())
    assert worst_rule <= 1e-11, worst_rule
    assert worst_cf <= 1e-10, worst_cf


@pytest.mark.parametrize("w", [(0.4, 0.55, 0.6), (0.35, 0.65, 0.5)])
def test_quad_reparametrized_flat_triangle(oracle_mod, w):
    """Edge nodes moved along straight edges: a non-affine quadratic map onto the same flat
    triangle, so S and F are the flat closed forms."""
    rng = np.random.default_rng(int(100 * w[0]))
    worst = 0.0
    for seed in range(15):
        v = rng.standard_normal((3, 3))
        a = 0.5 * np.linalg.norm(np.cross(v[1] - v[0], v[2] - v[0]))
        L = max(np.linalg.norm(v[1] - v[0]), np.linalg.norm(v[2] - v[1]), np.linalg.norm(v[0] - v[2]))
        if a / L ** 2 < 0.15:
            continue
        P = _flat_nodes(v, w)
        n = np.cross(v[1] - v[0], v[2] - v[0])
        n /= np.linalg.norm(n)
        for x in _near_points(_flat_nodes(v), L, n, rng, 10, 1e-5, 2.0):
            S, F = oracle_mod.quad_duffy(x, P)
            Sa, Fa = oracle_mod.tri_analytic(x, *v)
            worst = max(worst, abs(S - Sa) / abs(Sa), np.abs(F - Fa).max() / np.abs(Fa).max())
    assert worst <= 1e-10, worst


def test_quad_curved_against_brute_force(oracle_mod):
    rng = np.random.default_rng(9)
    worst = 0.0
    for seed in range(6):
        P, L, n = _curved_patch(40 + seed)
        for x in _near_points(P, L, n, rng, 4, 1e-3, 1.0):
            S, F = oracle_mod.quad_duffy(x, P)
            Sb, Fb = _brute(x, P)
            worst = max(worst, abs(S - Sb) / abs(Sb), np.abs(F - Fb).max() / np.abs(Fb).max())
    assert worst <= 1e-12, worst


def test_quad_field_is_minus_grad_potential(oracle_mod):
    rng = np.random.default_rng(13)
    for seed in range(5):
        P, L, n = _curved_patch(60 + seed)
        for x in _near_points(P, L, n, rng, 3, 1e-2, 1.0):
            _, F = oracle_mod.quad_duffy(x, P)
            h = 1e-5 * L
            g = np.array([(oracle_mod.quad_duffy(x + h * e, P)[0] - oracle_mod.quad_duffy(x - h * e, P)[0]) / (2 * h)
                          for e in np.eye(3)])
            assert np.abs(F + g).max() <= 1e-7 * np.abs(F).max()


def test_quad_sphere_converges(oracle_mod):
    """Unit sphere, unit density: S = 1 and F = 0 inside, S = 1/r and F = x/r^3 outside.
    Quadratic panels reproduce the sphere to O(h^3); the errors must fall at least 6x per
    level (h halves) and stay small at level 3."""
    pts = [np.array([0.1, -0.2, 0.3]), np.array([0.0, 0.5, -0.4]), np.array([1.3, 0.4, -0.2]),
           np.array([-0.9, -1.6, 0.7])]
    errs = []
    for level in (1, 2, 3):
        Q = _quad_sphere(level)
        e = 0.0
        for x in pts:
            S = 0.0
            F = np.zeros(3)
            for P in Q:
                s, f = oracle_mod.quad_duffy(x, P)
                S += s
                F += f
            r = np.linalg.norm(x)
            Se, Fe = (1.0, np.zeros(3)) if r < 1 else (1.0 / r, x / r ** 3)
            e = max(e, abs(S - Se) / abs(Se), np.abs(F - Fe).max() / max(np.abs(Fe).max(), 1.0))
        errs.append(e)
    assert errs[0] / errs[1] >= 6.0 and errs[1] / errs[2] >= 6.0, errs
    assert errs[2] <= 2e-4, errs


def test_quad_singular_potential(oracle_mod):
    """A point on the panel: the Duffy integrand of S is smooth there; on a flat panel (any
    edge-node placement along the edges) S is the principal-value closed form; F is NaN."""
    rng = np.random.default_rng(17)
    for seed in range(10):
        v = rng.standard_normal((3, 3))
        for w in ((0.5, 0.5, 0.5), (0.42, 0.58, 0.47)):
            P = _flat_nodes(v, w)
            b = rng.dirichlet(np.ones(3))
            x = b @ v
            S, F = oracle_mod.quad_duffy(x, P)
            Sa, _ = oracle_mod.tri_analytic(x, *v, on_plane=True)
            assert abs(S - Sa) <= 1e-11 * abs(Sa), (S, Sa)
            assert np.all(np.isnan(F))
