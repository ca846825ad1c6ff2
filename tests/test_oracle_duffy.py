"""Pins of the oracle's near-singular rule (Sec. 4: closest point, subdivision so
that it is a corner, Duffy transformation), which the GPU's Duffy near pass is
checked against.  Pinned to things other than itself: the closest point against
a dense sampling of the triangle; S and F against the closed forms of a flat
triangle (themselves pinned against an independent brute force and closed-form
values in test_oracle_pins.py), over distances from 1e-7 to 3 triangle sizes,
above the interior, near edges and vertices and in the plane outside; the
singular (on-triangle) potential against the principal-value closed form and the
equilateral-centroid value sqrt(3) a ln(2 + sqrt(3)); and the area of the
pieces (S of a far point times the distance tends to area / 4pi)."""

import math

import numpy as np
import pytest


def _tri(seed):
    rng = np.random.default_rng(seed)
    while True:
        v = rng.standard_normal((3, 3))
        a = 0.5 * np.linalg.norm(np.cross(v[1] - v[0], v[2] - v[0]))
        L = max(np.linalg.norm(v[1] - v[0]), np.linalg.norm(v[2] - v[1]), np.linalg.norm(v[0] - v[2]))
        if a / L ** 2 > 0.15:
            return v, L


def _points(v, L, rng, n, dmin, dmax):
    """Points around the triangle at distances ~ [dmin, dmax] L from a random point of (an
    enlargement of) it: above, in the plane outside, and skew."""
    nrm = np.cross(v[1] - v[0], v[2] - v[0])
    nrm /= np.linalg.norm(nrm)
    out = []
    for _ in range(n):
        b = rng.uniform(-0.3, 1.3, 3)
        b /= b.sum()
        h = L * 10 ** rng.uniform(math.log10(dmin), math.log10(dmax)) * rng.choice([-1.0, 1.0])
        kind = rng.integers(3)
        if kind == 0:
            x = b @ v + h * nrm
        elif kind == 1:
            t = rng.standard_normal(3)
            t -= (t @ nrm) * nrm
            x = b @ v + abs(h) * t / np.linalg.norm(t)
        else:
            x = b @ v + h * nrm + 0.3 * abs(h) * rng.standard_normal(3)
        out.append(x)
    return out


def test_closest_point_against_sampling(oracle_mod):
    rng = np.random.default_rng(1)
    g = np.linspace(0.0, 1.0, 201)
    B = np.array([(a, b, 1.0 - a - b) for a in g for b in g if a + b <= 1.0 + 1e-12])
    for s in range(20):
        v, L = _tri(s)
        samples = np.clip(B, 0.0, 1.0) @ v
        for x in _points(v, L, rng, 10, 1e-3, 2.0):
            c = oracle_mod.closest_point(x, *v)
            dmin = np.linalg.norm(samples - x, axis=1).min()
            dc = np.linalg.norm(x - c)
            assert dc <= dmin + 1e-12 and dmin - dc <= (1.0 / 200.0) * L * 1.5   # c is no farther than any sample
            # c lies in the closed triangle: non-negative barycentric coordinates
            T = np.stack([v[1] - v[0], v[2] - v[0]], axis=1)
            uv, *_ = np.linalg.lstsq(T, c - v[0], rcond=None)
            assert uv.min() >= -1e-12 and uv.sum() <= 1.0 + 1e-12


@pytest.mark.parametrize("dmin,dmax,bar", [(1e-3, 3.0, 1e-11), (1e-7, 1e-3, 1e-10)])
def test_duffy_against_closed_forms(oracle_mod, dmin, dmax, bar):
    rng = np.random.default_rng(int(-math.log10(dmin)))
    worst = 0.0
    for s in range(30):
        v, L = _tri(100 + s)
        for x in _points(v, L, rng, 20, dmin, dmax):
            if np.linalg.norm(x - oracle_mod.closest_point(x, *v)) < 0.1 * dmin * L:
                continue      # an in-plane point that fell on the triangle: the singular case below
            S, F = oracle_mod.tri_duffy(x, *v)
            Sa, Fa = oracle_mod.tri_analytic(x, *v)
            e = max(abs(S - Sa) / abs(Sa), np.abs(F - Fa).max() / np.abs(Fa).max())
            worst = max(worst, e)
    assert worst <= bar, worst


def test_closed_forms_above_an_edge(oracle_mod):
    """Points a short height above an edge of slender triangles (foot on the edge): the
    closed form's log term (R- + s-) loses digits to R - |s| there unless it is taken as
    R0^2 / (R- - s-); against the near-singular rule, which has no such cancellation.
    Both forms of the log term are the same number; the bar, 3e-10, is set by the height
    itself, known to about eps |x - v1| / |w| (1e-9 relative at 1e-7 of the edge), while the
    cancelling form was off by 7e-8 on such points."""
    rng = np.random.default_rng(11)
    worst = 0.0
    for s in range(30):
        # a slender triangle: base along x, apex displaced, height 0.1..0.3 of the base
        L = 1.0
        v = np.array([[0.0, 0.0, 0.0], [L, 0.0, 0.0], [rng.uniform(0.1, 0.9), rng.uniform(0.1, 0.3), 0.0]])
        R = np.linalg.qr(rng.standard_normal((3, 3)))[0]
        v = v @ R.T + rng.standard_normal(3)
        nrm = np.cross(v[1] - v[0], v[2] - v[0])
        nrm /= np.linalg.norm(nrm)
        for _ in range(6):
            a = rng.uniform(0.05, 0.95)
            foot = v[0] + a * (v[1] - v[0])
            h = 10 ** rng.uniform(-7, -4) * rng.choice([-1.0, 1.0])
            x = foot + h * nrm
            S, F = oracle_mod.tri_duffy(x, *v)
            Sa, Fa = oracle_mod.tri_analytic(x, *v)
            worst = max(worst, abs(S - Sa) / abs(Sa), np.abs(F - Fa).max() / np.abs(Fa).max())
    assert worst <= 3e-10, worst


def test_duffy_singular_potential(oracle_mod):
    # x on the triangle (the self pair at the centroid, and other interior points): the
    # potential against the principal-value closed form; F is not produced (NaN)
    rng = np.random.default_rng(3)
    for s in range(20):
        v, L = _tri(200 + s)
        for b in [np.full(3, 1.0 / 3.0)] + [rng.dirichlet(np.ones(3)) for _ in range(3)]:
            x = b @ v
            S, F = oracle_mod.tri_duffy(x, *v)
            Sa, _ = oracle_mod.tri_analytic(x, *v, on_plane=True)
            assert abs(S - Sa) <= 1e-12 * abs(Sa)
            assert np.all(np.isnan(F))
    for side in (1.0, 0.2):
        v = np.array([[0.0, 0.0, 0.0], [side, 0.0, 0.0], [0.5 * side, 0.5 * math.sqrt(3) * side, 0.0]])
        S, _ = oracle_mod.tri_duffy(v.mean(axis=0), *v)
        assert abs(4 * math.pi * S - math.sqrt(3) * side * math.log(2 + math.sqrt(3))) <= 1e-13 * side


def test_duffy_far_limit(oracle_mod):
    # far away the potential of a unit-density triangle is area / (4 pi r) to O(r^-3)
    v, L = _tri(7)
    area = 0.5 * np.linalg.norm(np.cross(v[1] - v[0], v[2] - v[0]))
    c = v.mean(axis=0)
    for r in (1e2, 1e3):
        x = c + r * np.array([0.6, -0.48, 0.64])
        S, _ = oracle_mod.tri_duffy(x, *v)
        assert abs(S * 4 * math.pi * np.linalg.norm(x - c) / area - 1.0) <= 10 * (L / r) ** 2
