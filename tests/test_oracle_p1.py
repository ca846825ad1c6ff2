"""Pins of the oracle's nodal piecewise-linear discretisation (Sec. 3, Eq. Matrix).

sigma_h = sum_k u_k psi_k with vertex hats psi_k, collocated at the vertices.
The oracle's pieces are pinned by things that do not come from it:
  * the closed form of int lambda_k / (4 pi R) over a flat triangle against an
    independent brute-force integration (split at the projection of x, Duffy
    transformation, graded Gauss-Legendre, written here in numpy), for far,
    near, coplanar-outside and on-vertex points, to 1e-12;
  * linear precision: sum_k lambda_k = 1 and sum_k lambda_k v_k = y make the
    three integrals add up to the unit-density potential and their
    vertex-weighted sum the first moment, both computed by the brute force;
  * a conductor sphere (u = V0/R, phi = V0 R/|x| outside and V0 inside) with
    second-order convergence of the nodal solution on icospheres;
  * a floating shell (its potential V_f = 0.6 V0, net charge zero);
  * the matrix of Eq. Matrix against a 7-point-free brute-force row (every
    triangle integrated by the brute force) on a coarse sphere;
  * the field of the hats against a brute force (1e-10), against central
    differences of the hat potentials and, summed, against the unit-density
    field; the sphere's field V0 R x/|x|^3 outside and 0 inside with
    second-order convergence;
  * field lines of the nodal density on the sphere against the closed-form
    streamer integral of a radial line, second order;
  * rigid motions of the mesh leave the matrix and solution unchanged and
    rotate the field;
  * refusal of vertices shared by two bodies.
"""

import json
import math
import os

import numpy as np
import pytest

from workloads import floating_shell_problem, sphere_problem
from workloads.meshes import Problem

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def _gl(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def brute_hats(x, v1, v2, v3, nv=160, nu=24):
    """Brute-force int lambda_k / (4 pi |x - y|) dS (k = 1..3), the unit-density
    integral and the first moment int y / (4 pi |x - y|) dS.

    The triangle is split at the projection rho of x into three signed
    sub-triangles with a corner at rho; each maps to the unit square by the
    Duffy transformation (the Jacobian cancels 1/r at rho) and is integrated
    with composite Gauss-Legendre, graded geometrically towards rho on the
    scale |w|.  lambda_k(y) from signed sub-areas.
    """
    x, v1, v2, v3 = (np.asarray(a, dtype=np.float64) for a in (x, v1, v2, v3))
    cr0 = np.cross(v2 - v1, v3 - v1)
    twoA = np.linalg.norm(cr0)
    n = cr0 / twoA
    w = float(np.dot(x - v1, n))
    rho = x - w * n
    size = max(np.linalg.norm(v2 - v1), np.linalg.norm(v3 - v2), np.linalg.norm(v1 - v3))
    base = max(abs(w) / (4 * size), 1e-7)
    bps = [0.0]
    b = base / 64
    while b < 1.0:
        bps.append(b)
        b *= 2.0
    bps.append(1.0)
    ug, uw = _gl(nu)
    vg, vw = _gl(nv)
    hats = np.zeros(3)
    S = 0.0
    M = np.zeros(3)
    V = (v1, v2, v3)
    for a, bb in ((v1, v2), (v2, v3), (v3, v1)):
        pa, pb = a - rho, bb - rho
        cr = np.cross(pa, pb)
        sgn = np.sign(np.dot(cr, n))
        J = np.linalg.norm(cr)
        if J < 1e-300:
            continue
        for lo, hi in zip(bps[:-1], bps[1:]):
            u = lo + (hi - lo) * ug
            wu = (hi - lo) * uw
            U, Vv = np.meshgrid(u, vg, indexing="ij")
            W = np.outer(wu, vw)
            d = (1 - Vv)[..., None] * pa + Vv[..., None] * pb
            y = rho + U[..., None] * d
            R = np.linalg.norm(x - y, axis=-1)
            jac = U * J * W * sgn / R
            S += np.sum(jac)
            M += np.einsum("ij,ijk->k", jac, y)
            for k in range(3):
                p1, p2 = V[(k + 1) % 3], V[(k + 2) % 3]
                lam = np.einsum("ijk,k->ij", np.cross(p1 - y, p2 - y), n) / twoA
                hats[k] += np.sum(jac * lam)
    return hats / (4 * math.pi), S / (4 * math.pi), M / (4 * math.pi)


def _tri(seed):
    rng = np.random.default_rng(seed)
    while True:
        v = rng.standard_normal((3, 3))
        a = 0.5 * np.linalg.norm(np.cross(v[1] - v[0], v[2] - v[0]))
        L = max(np.linalg.norm(v[1] - v[0]), np.linalg.norm(v[2] - v[1]), np.linalg.norm(v[0] - v[2]))
        if a / L ** 2 > 0.15:
            return v


def _points(v, rng):
    """far, near above the interior, near above an edge, coplanar outside, above a vertex."""
    n = np.cross(v[1] - v[0], v[2] - v[0])
    n /= np.linalg.norm(n)
    c = v.mean(axis=0)
    size = max(np.linalg.norm(v[1] - v[0]), np.linalg.norm(v[2] - v[1]), np.linalg.norm(v[0] - v[2]))
    b = rng.dirichlet([2, 2, 2])
    inner = b @ v
    edge = 0.5 * (v[0] + v[1])
    out = v[2] + 0.7 * (v[2] - c)           # in the plane, beyond vertex 3
    return [
        ("far", c + 5.0 * size * n + 2.0 * size * (v[0] - c)),
        ("near_interior", inner + 0.03 * size * n),
        ("near_edge", edge - 0.02 * size * n),
        ("coplanar_outside", out),
        ("above_vertex", v[1] + 0.01 * size * n),
    ]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_hat_integrals_brute_force(oracle_mod, seed):
    v = _tri(seed)
    rng = np.random.default_rng(100 + seed)
    for name, x in _points(v, rng):
        got = oracle_mod.tri_linear_analytic(x, *v)
        ref, S, M = brute_hats(x, *v)
        # the closed form cancels at distances of several sizes (the method uses the
        # 7-point rule there): 1e-11 on the far point, 1e-12 elsewhere
        tol = 1e-11 if name == "far" else 1e-12
        assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref)), (name, got, ref)
        # linear precision of the hats: they add to the unit-density integral and
        # their vertex-weighted sum is the first moment
        assert abs(got.sum() - S) <= tol * abs(S), name
        assert np.max(np.abs(got @ v - M)) <= tol * np.max(np.abs(M)), name


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_hat_integrals_at_a_vertex(oracle_mod, seed):
    """Singular pairs of Eq. Matrix: the collocation point is a vertex of the triangle."""
    v = _tri(seed)
    for k in range(3):
        got = oracle_mod.tri_linear_analytic(v[k], *v, on_plane=True)
        assert np.all(np.isfinite(got))
        ref, S, _ = brute_hats(v[k], *v)
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref)), (k, got, ref)
        # the vertex's own hat carries more than the others at its vertex
        assert got[k] > max(got[(k + 1) % 3], got[(k + 2) % 3])


def brute_hat_fields(x, v1, v2, v3, nv=200, nu=32):
    """Brute-force int lambda_k (x - y) / (4 pi |x - y|^3) dS, [k][3], by the
    splitting and graded Duffy rule of brute_hats."""
    x, v1, v2, v3 = (np.asarray(a, dtype=np.float64) for a in (x, v1, v2, v3))
    cr0 = np.cross(v2 - v1, v3 - v1)
    twoA = np.linalg.norm(cr0)
    n = cr0 / twoA
    w = float(np.dot(x - v1, n))
    rho = x - w * n
    size = max(np.linalg.norm(v2 - v1), np.linalg.norm(v3 - v2), np.linalg.norm(v1 - v3))
    base = max(abs(w) / (4 * size), 1e-7)
    bps = [0.0]
    b = base / 64
    while b < 1.0:
        bps.append(b)
        b *= 2.0
    bps.append(1.0)
    ug, uw = _gl(nu)
    vg, vw = _gl(nv)
    out = np.zeros((3, 3))
    V = (v1, v2, v3)
    for a, bb in ((v1, v2), (v2, v3), (v3, v1)):
        pa, pb = a - rho, bb - rho
        cr = np.cross(pa, pb)
        sgn = np.sign(np.dot(cr, n))
        J = np.linalg.norm(cr)
        if J < 1e-300:
            continue
        for lo, hi in zip(bps[:-1], bps[1:]):
            u = lo + (hi - lo) * ug
            wu = (hi - lo) * uw
            U, Vv = np.meshgrid(u, vg, indexing="ij")
            W = np.outer(wu, vw)
            d = (1 - Vv)[..., None] * pa + Vv[..., None] * pb
            y = rho + U[..., None] * d
            r = x - y
            R = np.linalg.norm(r, axis=-1)
            jac = U * J * W * sgn / R ** 3
            for k in range(3):
                p1, p2 = V[(k + 1) % 3], V[(k + 2) % 3]
                lam = np.einsum("ijk,k->ij", np.cross(p1 - y, p2 - y), n) / twoA
                out[k] += np.einsum("ij,ijk->k", jac * lam, r)
    return out / (4 * math.pi)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_hat_fields(oracle_mod, seed):
    """Field of the hats: against the brute force (1e-10; the 1/R^3 kernel is
    harder for it), against central differences of the hat potentials (whose
    closed form the brute force pins to 1e-12), and their sum against the
    unit-density field of the plain closed form."""
    v = _tri(seed)
    rng = np.random.default_rng(200 + seed)
    for name, x in _points(v, rng):
        if name == "coplanar_outside":
            x = x + 1e-3 * np.cross(v[1] - v[0], v[2] - v[0])   # a volume point just off the plane
        got = oracle_mod.tri_linear_field(x, *v)
        ref = brute_hat_fields(x, *v)
        tol = 1e-9 if name == "far" else 1e-10
        assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref)), (name, got, ref)
        # E = -grad phi, hat by hat (not on the far point: the closed-form potential's
        # cancellation there, ~1e-15, over the step would swamp the bar)
        if name == "far":
            continue
        h = 1e-5 * max(np.linalg.norm(v[1] - v[0]), 1.0)
        fd = np.zeros((3, 3))
        for d in range(3):
            e = np.zeros(3)
            e[d] = h
            fd[:, d] = -(oracle_mod.tri_linear_analytic(x + e, *v) - oracle_mod.tri_linear_analytic(x - e, *v)) / (2 * h)
        assert np.max(np.abs(got - fd)) <= 1e-7 * np.max(np.abs(got)), name
    for name, x in _points(v, rng):
        if name == "coplanar_outside":
            x = x + 1e-3 * np.cross(v[1] - v[0], v[2] - v[0])
        got = oracle_mod.tri_linear_field(x, *v)
        _, F = oracle_mod.tri_analytic(x, *v)
        assert np.max(np.abs(got.sum(axis=0) - F)) <= 1e-11 * np.max(np.abs(F)), name


def test_sphere_nodal_field(oracle_mod):
    """E of the nodal solution on the conductor sphere: V0 R x/|x|^3 outside and
    0 inside, second order in h."""
    pts = np.array([[0.0, 0.0, 1.5], [1.2, -0.9, 0.4], [0.2, 0.1, -0.3], [-0.4, 0.3, 0.2]])
    r = np.linalg.norm(pts, axis=1)
    exact = np.where((r > 1.0)[:, None], pts / r[:, None] ** 3, 0.0)
    errs = []
    for level in (2, 3, 4):
        p = sphere_problem(level)
        o = oracle_mod.Oracle(p)
        u = np.linalg.solve(o.p1_assemble(), o.p1_rhs(p.body_V))
        phi, E = o.p1_field(u, pts)
        assert np.allclose(phi, o.p1_potential(u, pts), rtol=0, atol=1e-13)
        errs.append(np.max(np.abs(E - exact)))
    assert errs[-1] < 2e-3 and errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


def test_sphere_nodal_streamer_integral(oracle_mod):
    """Field lines of the nodal solution on the conductor sphere at V0 run
    radially; the streamer integral from r0 to r1 is then
    a [-V0^2/(3 r^3) + 2 V0 e0 / r + e0^2 r] between them (alpha = a (E - e0)^2,
    E = V0/r^2 > e0).  The nodal lines converge to it at second order, and the
    path stays radial."""
    V0, a, e0 = 100.0, 1e-3, 25.0
    dirs = np.array([[0.3, -0.5, 0.81], [-0.7, 0.2, 0.1], [0.05, 0.9, -0.4]])
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    r0, h, steps = 1.1, 5e-3, 100   # away from the flat panels, where the error is asymptotic
    r1 = r0 + h * steps
    F = lambda r: a * (-V0 ** 2 / (3 * r ** 3) + 2 * V0 * e0 / r + e0 ** 2 * r)
    exact = F(r1) - F(r0)
    tp = oracle_mod.trace_params(h=h, max_steps=steps, e_min=1e-3, alpha_a=a, alpha_e0=e0, alpha_p=2.0)
    errs = []
    for level in (2, 3, 4):
        p = sphere_problem(level, V0=V0)
        o = oracle_mod.Oracle(p)
        u = np.linalg.solve(o.p1_assemble(), o.p1_rhs(p.body_V))
        ns, st, I, path = o.p1_trace(u, r0 * dirs, tp, want_path=True)
        assert np.all(ns == steps) and np.all(st == 0)
        end = path[:, steps]
        assert np.max(np.abs(np.linalg.norm(end, axis=1) - r1)) < 1e-2
        assert np.max(np.linalg.norm(np.cross(end, dirs), axis=1)) < 1e-2
        errs.append(np.max(np.abs(I - exact)) / exact)
    assert errs[-1] < 2e-3 and errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


def test_matrix_against_brute_force_rows(oracle_mod):
    """Rows of Eq. Matrix on a level-1 sphere: each entry is a sum of the closed
    forms / 7-point values over the vertex's triangles; with every triangle
    integrated by the brute force instead the rows agree to the 7-point rule's
    error on regular pairs (eta = 6: below 1e-7 relative)."""
    p = sphere_problem(1)
    o = oracle_mod.Oracle(p)
    A = o.p1_assemble()
    nv = p.n_vert
    for i in (0, 7, nv - 1):
        ref = np.zeros(nv)
        for t in p.tri:
            h, _, _ = brute_hats(p.vert[i], *p.vert[t], nv=96, nu=16)
            ref[t] += h
        assert np.max(np.abs(A[i, :nv] - ref)) <= 1e-7 * np.max(np.abs(ref)), i


def test_sphere_nodal_convergence(oracle_mod):
    """Conductor sphere at V0: u -> V0/R, second order in h; potential V0 R/|x|
    outside and V0 inside."""
    errs, perr = [], []
    V0 = 1.0
    for level in (2, 3, 4):
        p = sphere_problem(level)
        o = oracle_mod.Oracle(p)
        A = o.p1_assemble()
        b = o.p1_rhs(p.body_V * V0)
        u = np.linalg.solve(A, b)
        errs.append(np.max(np.abs(u - V0)) / V0)
        pts = np.array([[0.0, 0.0, 3.0], [2.0, -1.0, 0.5], [0.1, 0.2, -0.3], [0.0, 0.0, 0.0]])
        phi = o.p1_potential(u, pts)
        r = np.linalg.norm(pts, axis=1)
        exact = np.where(r > 1.0, V0 / np.maximum(r, 1e-300), V0)
        perr.append(np.max(np.abs(phi - exact)) / V0)
    assert errs[-1] < 2e-3
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs
    assert perr[-1] < 2e-3 and perr[0] / perr[2] > 8.0, perr


def test_floating_shell_nodal(oracle_mod):
    g = GOLDEN["floating_shell"]
    errs = []
    for level in (2, 3):
        p = floating_shell_problem(level, a=g["a"], b1=g["b1"], b2=g["b2"])
        o = oracle_mod.Oracle(p, constraint_form=1)   # the net-charge row
        A = o.p1_assemble()
        u = np.linalg.solve(A, o.p1_rhs(p.body_V))
        nv = p.n_vert
        errs.append(abs(u[nv] - g["Vf_over_V0"]))
        # the net charge of the floating body is zero (its constraint row)
        assert abs(A[nv] @ u) < 1e-12
    assert errs[-1] < 2e-4 and errs[0] / errs[1] > 4.0, errs


def test_nodal_rigid_motion_invariance(oracle_mod):
    """A rotation plus translation of the whole mesh changes no entry of the nodal
    matrix beyond rounding, and rotates the field of the solution with it."""
    import dataclasses
    p = floating_shell_problem(1, V0=2.0)
    o = oracle_mod.Oracle(p)
    A = o.p1_assemble()
    u = np.linalg.solve(A, o.p1_rhs(p.body_V))
    th = 0.7
    Rz = np.array([[np.cos(th), -np.sin(th), 0.0], [np.sin(th), np.cos(th), 0.0], [0.0, 0.0, 1.0]])
    Rx = np.array([[1.0, 0.0, 0.0], [0.0, np.cos(0.3), -np.sin(0.3)], [0.0, np.sin(0.3), np.cos(0.3)]])
    Q = Rx @ Rz
    shift = np.array([0.4, -1.1, 2.3])
    q = dataclasses.replace(p, vert=p.vert @ Q.T + shift)
    oq = oracle_mod.Oracle(q)
    Aq = oq.p1_assemble()
    assert np.max(np.abs(Aq - A)) <= 1e-12 * np.max(np.abs(A))
    uq = np.linalg.solve(Aq, oq.p1_rhs(q.body_V))
    assert np.max(np.abs(uq - u)) <= 1e-10 * np.max(np.abs(u))
    pts = np.array([[0.0, 0.0, 2.5], [1.2, 1.9, -0.4], [0.3, -0.2, 0.1]])
    _, E = o.p1_field(u, pts)
    _, Eq = oq.p1_field(uq, pts @ Q.T + shift)
    assert np.max(np.abs(Eq - E @ Q.T)) <= 1e-10 * np.max(np.abs(E))


def test_refuses_shared_vertices(oracle_mod):
    """A vertex in triangles of two bodies is refused (each body carries its own nodes;
    interface bodies are accepted, their rows are pinned in test_oracle_p1_interface)."""
    p = sphere_problem(1)
    tb = p.tri_body.copy()
    tb[: len(tb) // 2] = 1
    q = Problem(name="shared", vert=p.vert, tri=p.tri, tri_body=tb.astype(np.int32),
                body_kind=np.array([0, 0], dtype=np.int32), eps_plus=np.ones(2), eps_minus=np.ones(2),
                body_V=np.array([1.0, 0.0]), body_names=["a", "b"])
    with pytest.raises(ValueError):
        oracle_mod.Oracle(q).p1_assemble()
