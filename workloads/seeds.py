"""Seeded point sets, field-line starts and load cases (numpy PCG64).

Draw orders are fixed so that every consumer (oracle tests, GPU tests, bench)
sees the same values for the same seed.
"""

from __future__ import annotations

import numpy as np

from .meshes import COAX, Problem


def sphere_eval_points(n: int = 1000, seed: int = 1, rmin: float = 1.5, rmax: float = 3.0):
    """Points around the unit sphere: directions = normalised N(0, I3) (n x 3 drawn
    first), then radius ~ U[rmin, rmax] (n draws).  Uniform in radius, not volume."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = rng.uniform(rmin, rmax, n)
    return np.ascontiguousarray(d * r[:, None])


def gap_eval_points(n: int = 1000, seed: int = 3, margin: float = 0.004):
    """Points in the air gap of the coax: rho ~ U[rod_r+m, shell_r-m],
    phi ~ U[0, 2pi), z ~ U[-0.14, 0.14]; points inside the disc slab or within
    `margin` of the torus surface are redrawn (in draw order)."""
    g = COAX
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        rho = rng.uniform(g["rod_r"] + margin, g["shell_r"] - margin)
        ph = rng.uniform(0.0, 2 * np.pi)
        z = rng.uniform(-0.14, 0.14)
        if abs(z) <= g["disc_z"] + margin:
            continue
        dt = np.hypot(rho - g["ring_R"], z - g["ring_z"])
        if dt <= g["ring_r"] + margin:
            continue
        out.append((rho * np.cos(ph), rho * np.sin(ph), z))
    return np.ascontiguousarray(np.array(out, dtype=np.float64))


def electrode_line_starts(p: Problem, n: int, seed: int, offset: float = 1e-6):
    """Area-uniform random points on the start panels of `p`, lifted by `offset`
    along the panel's eps+ normal.

    Draw order: panel indices (rng.choice with p proportional to area), then
    (n x 2) uniforms for the barycentric coordinates (square-root map).
    Returns (starts [n,3], panel [n] int32, bary [n,3]).
    """
    rng = np.random.default_rng(seed)
    mask = p.start_mask if p.start_mask is not None else np.ones(p.n_tri, bool)
    cand = np.nonzero(mask)[0]
    a, b, c = (p.vert[p.tri[cand, k]] for k in range(3))
    cr = np.cross(b - a, c - a)
    area = 0.5 * np.linalg.norm(cr, axis=1)
    pick = rng.choice(len(cand), size=n, p=area / area.sum())
    u = rng.uniform(0.0, 1.0, (n, 2))
    s = np.sqrt(u[:, 0])
    bary = np.stack([1.0 - s, s * (1.0 - u[:, 1]), s * u[:, 1]], axis=1)
    A, B, C = a[pick], b[pick], c[pick]
    y = bary[:, :1] * A + bary[:, 1:2] * B + bary[:, 2:3] * C
    nrm = cr[pick] / np.linalg.norm(cr[pick], axis=1, keepdims=True)
    starts = y + offset * nrm
    return (np.ascontiguousarray(starts), cand[pick].astype(np.int32),
            np.ascontiguousarray(bary))


def rod_load_cases(p: Problem, n: int = 64, seed: int = 4, lo: float = 0.5, hi: float = 2.0,
                   driven_body: int = 1):
    """n load cases: the driven body's potential ~ U[lo, hi], all others as in p
    (the shell stays at 0).  Returns body_V [n, n_body]."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(lo, hi, n)
    out = np.tile(p.body_V, (n, 1)).astype(np.float64)
    out[:, driven_body] = v
    return np.ascontiguousarray(out)


def vertex_perturbations(p: Problem, n: int = 20, seed: int = 8):
    """n single-vertex perturbation directions of the mesh: draw k = 0, 1, ...: a vertex index
    ~ U{0..n_vert-1}, then a direction N(0, I_3) normalised, one after the other.  Yields
    (vertex, unit direction) pairs without end; a consumer that must skip a draw (its
    classification or step counts change under the perturbation) takes the next one, so the
    sequence stays deterministic.  Returned as a generator."""
    rng = np.random.default_rng(seed)
    while True:
        v = int(rng.integers(0, p.n_vert))
        d = rng.standard_normal(3)
        yield v, d / np.linalg.norm(d)
