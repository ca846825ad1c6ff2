"""Seeded curved quadratic panels and points for the tests of the near-singular rule on
curved panels (oracle pins and GPU parity share them; none of the rule's arithmetic: the map
qmap only places the points)."""

import math

import numpy as np

from workloads import sphere_problem


def flat_nodes(v, w=(0.5, 0.5, 0.5)):
    """Six nodes of a flat triangle v with the edge nodes of edges 1-2, 2-3, 3-1 at fractions w."""
    return np.array([v[0], v[1], v[2], v[0] + w[0] * (v[1] - v[0]), v[1] + w[1] * (v[2] - v[1]),
                     v[2] + w[2] * (v[0] - v[2])])


def qmap(P, s, t):
    """The quadratic map (numpy, written from the shape functions) at arrays s, t."""
    l1 = 1.0 - s - t
    N = np.stack([l1 * (2 * l1 - 1), s * (2 * s - 1), t * (2 * t - 1), 4 * l1 * s, 4 * s * t, 4 * t * l1], -1)
    return N @ P


def curved_patch(seed, bulge=0.15):
    """A curved patch: a random well-shaped triangle with its edge nodes lifted off the plane
    by up to `bulge` of its size (and moved a little along their edges)."""
    rng = np.random.default_rng(seed)
    while True:
        v = rng.standard_normal((3, 3))
        a = 0.5 * np.linalg.norm(np.cross(v[1] - v[0], v[2] - v[0]))
        L = max(np.linalg.norm(v[1] - v[0]), np.linalg.norm(v[2] - v[1]), np.linalg.norm(v[0] - v[2]))
        if a / L ** 2 > 0.2:
            break
    n = np.cross(v[1] - v[0], v[2] - v[0])
    n /= np.linalg.norm(n)
    P = flat_nodes(v, rng.uniform(0.45, 0.55, 3))
    P[3:] += (bulge * L * rng.uniform(0.3, 1.0, 3))[:, None] * n + 0.03 * L * rng.standard_normal((3, 3))
    return P, L, n


def near_points(P, L, n, rng, k, dmin, dmax):
    out = []
    for _ in range(k):
        st = rng.dirichlet(np.ones(3))[:2] * rng.uniform(0.0, 1.2)
        y = qmap(P, st[0], st[1])
        h = L * 10 ** rng.uniform(math.log10(dmin), math.log10(dmax))
        d = rng.standard_normal(3) * 0.3 + rng.choice([-1.0, 1.0]) * n
        out.append(y + h * d / np.linalg.norm(d))
    return out


def quad_sphere(level):
    """The icosphere of the given level with each flat triangle replaced by the quadratic panel
    through its corners and its edge midpoints pushed out to the unit sphere."""
    p = sphere_problem(level)
    V = p.vert[p.tri]                                   # (N, 3, 3)
    mids = np.stack([V[:, 0] + V[:, 1], V[:, 1] + V[:, 2], V[:, 2] + V[:, 0]], 1)
    mids /= np.linalg.norm(mids, axis=-1, keepdims=True)
    return np.concatenate([V, mids], 1)                # (N, 6, 3)
