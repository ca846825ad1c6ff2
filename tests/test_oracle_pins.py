"""Pins of the FP64 oracle against mathematics that does not come from the oracle.

Each test fixes one part of the oracle by something independent of it: exact
polynomial integrals, textbook closed forms, an independent brute-force
integrator (the paper's own near-singular recipe of Sec. 4: split at the
closest point, Duffy transformation, tensor Gauss-Legendre), Gauss's law,
symmetry and equivariance, a dense LU solve, and closed-form electrostatics
of spheres (Sec. 2 formulation).
"""

import json
import math
import os

import numpy as np
import pytest

from workloads import (coated_sphere_problem, coax_problem, floating_shell_problem, sphere_eval_points,
                       sphere_problem, sphere_sheet_problem, icosphere)
from workloads.meshes import Problem

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


# ----------------------------------------------------------------- helpers
def _gl(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def brute_SF(x, v1, v2, v3, nv=320, nu=32):
    """Independent brute-force S and F of a unit-density flat triangle.

    Splits the triangle at the projection rho of x into three signed
    sub-triangles with a corner at rho, maps each to the unit square by the
    Duffy transformation (which cancels the 1/r singularity at rho) and
    integrates with composite Gauss-Legendre, graded in the radial variable
    towards rho on the scale |w|.
    """
    x, v1, v2, v3 = map(np.asarray, (x, v1, v2, v3))
    n = np.cross(v2 - v1, v3 - v1)
    n /= np.linalg.norm(n)
    w = float(np.dot(x - v1, n))
    rho = x - w * n
    size = max(np.linalg.norm(v2 - v1), np.linalg.norm(v3 - v2), np.linalg.norm(v1 - v3))
    # radial breakpoints: geometric grading from |w| (or a tiny fraction of size) to 1
    base = max(abs(w) / (4 * size), 1e-6)
    bps = [0.0]
    b = base / 64
    while b < 1.0:
        bps.append(b)
        b *= 2.0
    bps.append(1.0)
    ug, uw = _gl(nu)
    vg, vw = _gl(nv)
    S = 0.0
    F = np.zeros(3)
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
            U, V = np.meshgrid(u, vg, indexing="ij")
            W = np.outer(wu, vw)
            d = (1 - V)[..., None] * pa + V[..., None] * pb            # in-plane direction
            y = rho + U[..., None] * d
            r = x - y
            R = np.linalg.norm(r, axis=-1)
            jac = U * J * W * sgn
            S += np.sum(jac / R)
            F += np.einsum("ij,ijk->k", jac / R ** 3, r)
    return S / (4 * math.pi), F / (4 * math.pi)


def _tri(seed):
    rng = np.random.default_rng(seed)
    while True:
        v = rng.standard_normal((3, 3))
        a = 0.5 * np.linalg.norm(np.cross(v[1] - v[0], v[2] - v[0]))
        L = max(np.linalg.norm(v[1] - v[0]), np.linalg.norm(v[2] - v[1]), np.linalg.norm(v[0] - v[2]))
        if a / L ** 2 > 0.15:
            return v


# ------------------------------------------------------------- quadrature
def test_quad7_exact_degree5(oracle_mod):
    bary, w = oracle_mod.quad7_rule()
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.all(bary >= 0) and np.allclose(bary.sum(axis=1), 1.0, atol=1e-15)
    # reference triangle (0,0),(1,0),(0,1): x = b2, y = b3, area 1/2
    xs, ys = bary[:, 1], bary[:, 2]
    for p in range(6):
        for q in range(6 - p):
            exact = math.factorial(p) * math.factorial(q) / math.factorial(p + q + 2)
            got = 0.5 * np.sum(w * xs ** p * ys ** q)
            assert abs(got - exact) < 1e-15, (p, q, got, exact)
    # and not exact at degree 6 (a degree-5 rule, not something higher)
    errs = []
    for p in range(7):
        q = 6 - p
        exact = math.factorial(p) * math.factorial(q) / math.factorial(8)
        errs.append(abs(0.5 * np.sum(w * xs ** p * ys ** q) - exact))
    assert max(errs) > 1e-6


# --------------------------------------------------------- panel geometry
def test_panel_geometry_circumcentre(oracle_mod):
    for s in range(20):
        v = _tri(s)
        g = oracle_mod.panel_geometry(*v)
        d = [np.linalg.norm(v[k] - g["circumcenter"]) for k in range(3)]
        assert np.allclose(d, g["circumradius"], rtol=1e-12)
        assert abs(np.dot(g["circumcenter"] - v[0], g["normal"])) < 1e-12   # in plane
        assert np.allclose(g["centroid"], v.mean(axis=0))
        assert abs(g["area"] - 0.5 * np.linalg.norm(np.cross(v[1] - v[0], v[2] - v[0]))) < 1e-14
        assert np.dot(np.cross(v[1] - v[0], v[2] - v[0]), g["normal"]) > 0


# ---------------------------------------------------- analytic integrals
def test_equilateral_centroid_closed_form(oracle_mod):
    for side in (1.0, 0.37, 5.0):
        v1 = np.array([0.0, 0.0, 0.0])
        v2 = np.array([side, 0.0, 0.0])
        v3 = np.array([0.5 * side, 0.5 * math.sqrt(3) * side, 0.0])
        c = (v1 + v2 + v3) / 3
        S, F = oracle_mod.tri_analytic(c, v1, v2, v3, on_plane=True)
        exact = math.sqrt(3) * side * math.log(2 + math.sqrt(3))
        assert abs(exact / side - GOLDEN["equilateral_centroid_int_invR"]["value_over_side"]) < 1e-9
        assert abs(4 * math.pi * S - exact) < 1e-13 * exact
        assert np.abs(F).max() < 1e-15        # centroid of an equilateral triangle: PV field is zero


@pytest.mark.parametrize("seed", range(6))
def test_analytic_vs_bruteforce_offplane(oracle_mod, seed):
    v = _tri(100 + seed)
    rng = np.random.default_rng(seed)
    n = np.cross(v[1] - v[0], v[2] - v[0])
    n /= np.linalg.norm(n)
    size = np.linalg.norm(v[1] - v[0])
    c = v.mean(axis=0)
    cases = []
    for wfrac in (0.5, 0.05, 0.01, -0.02, 1e-3):
        # projection inside, and outside beyond an edge
        b = rng.dirichlet([2, 2, 2])
        cases.append(b @ v + wfrac * size * n)
        cases.append(c + 1.3 * (v[0] - c) + 0.4 * (v[1] - v[0]) + wfrac * size * n)
    for x in cases:
        S, F = oracle_mod.tri_analytic(x, *v)
        Sb, Fb = brute_SF(x, *v)
        assert abs(S - Sb) <= 1e-12 * abs(Sb), (x, S, Sb)
        assert np.abs(F - Fb).max() <= 1e-12 * np.abs(Fb).max(), (x, F, Fb)


def test_analytic_vs_bruteforce_inplane_potential(oracle_mod):
    # in-plane S: the self (centroid, principal value) and outside points
    for s in range(4):
        v = _tri(200 + s)
        c = v.mean(axis=0)
        S, _ = oracle_mod.tri_analytic(c, *v, on_plane=True)
        Sb, _ = brute_SF(c, *v)
        assert abs(S - Sb) <= 1e-12 * abs(Sb)
        x = c + 2.0 * (v[1] - c)
        S, _ = oracle_mod.tri_analytic(x, *v)
        Sb, _ = brute_SF(x, *v)
        assert abs(S - Sb) <= 1e-11 * abs(Sb)


def test_field_is_minus_gradient(oracle_mod):
    for s in range(5):
        v = _tri(300 + s)
        rng = np.random.default_rng(s)
        for scale in (0.05, 0.5, 3.0):
            x = v.mean(axis=0) + scale * rng.standard_normal(3)
            _, F = oracle_mod.tri_analytic(x, *v)
            h = 1e-5 * max(scale, 0.1)
            g = np.zeros(3)
            for k in range(3):
                e = np.zeros(3)
                e[k] = h
                g[k] = (oracle_mod.tri_analytic(x + e, *v)[0] - oracle_mod.tri_analytic(x - e, *v)[0]) / (2 * h)
            assert np.abs(F + g).max() <= 1e-7 * np.abs(F).max()


def test_principal_value_inplane_field_is_tangential_gradient(oracle_mod):
    # at an interior in-plane point the PV field is minus the tangential gradient of S
    for s in range(4):
        v = _tri(400 + s)
        x = np.array([0.5, 0.3, 0.2]) @ v
        S0, F = oracle_mod.tri_analytic(x, *v, on_plane=True)
        n = np.cross(v[1] - v[0], v[2] - v[0])
        n /= np.linalg.norm(n)
        assert abs(np.dot(F, n)) < 1e-15
        t1 = (v[1] - v[0]) / np.linalg.norm(v[1] - v[0])
        t2 = np.cross(n, t1)
        h = 1e-5
        for t in (t1, t2):
            d = (oracle_mod.tri_analytic(x + h * t, *v, on_plane=True)[0]
                 - oracle_mod.tri_analytic(x - h * t, *v, on_plane=True)[0]) / (2 * h)
            assert abs(np.dot(F, t) + d) < 1e-7


def test_normal_jump_of_field(oracle_mod):
    # single-layer jump: n.(F(x + eps n) - F(x - eps n)) -> 1 for unit density (Eq. ADL)
    v = _tri(500)
    n = np.cross(v[1] - v[0], v[2] - v[0])
    n /= np.linalg.norm(n)
    x = np.array([0.2, 0.5, 0.3]) @ v
    for eps in (1e-6, 1e-9, 1e-12):
        Fp = oracle_mod.tri_analytic(x + eps * n, *v)[1]
        Fm = oracle_mod.tri_analytic(x - eps * n, *v)[1]
        assert abs(np.dot(Fp - Fm, n) - 1.0) < 1e-5
        _, F0 = oracle_mod.tri_analytic(x, *v, on_plane=True)
        assert np.abs(0.5 * (Fp + Fm) - F0).max() < 1e-4


def test_far_limit_and_quad7_convergence(oracle_mod):
    v = _tri(600)
    c = v.mean(axis=0)
    a = 0.5 * np.linalg.norm(np.cross(v[1] - v[0], v[2] - v[0]))
    d = np.array([0.3, -0.5, 0.8]) / np.linalg.norm([0.3, -0.5, 0.8])
    errs = []
    for dist in (5.0, 10.0, 20.0, 40.0):
        x = c + dist * d
        S, F = oracle_mod.tri_analytic(x, *v)
        Sq, Fq = oracle_mod.tri_quad7(x, *v)
        errs.append(abs(S - Sq) / abs(S))
        # monopole limit with no dipole term about the centroid: relative error O(1/dist^2)
        assert abs(4 * math.pi * S * dist / a - 1.0) < 2.0 / dist ** 2
    # degree-5 rule: the absolute error falls like dist^-7, the relative one like dist^-6
    rates = [math.log2(errs[k] / errs[k + 1]) for k in range(3)]
    assert min(rates) > 5.5, (errs, rates)


def test_gauss_law_solid_angles_closed_mesh(oracle_mod):
    # sum_j n_j . F_j(x) = -1 inside a closed outward-oriented surface, 0 outside
    vert, tri = icosphere(2)
    rng = np.random.default_rng(7)
    for x, want in ((0.3 * rng.standard_normal(3) * 0.5, -1.0), (np.array([1.7, -0.4, 0.9]), 0.0),
                    (np.array([0.0, 0.0, 0.97]), -1.0), (np.array([0.2, 0.1, 1.04]), 0.0)):
        tot = 0.0
        for t in tri:
            v = vert[t]
            n = np.cross(v[1] - v[0], v[2] - v[0])
            n /= np.linalg.norm(n)
            tot += np.dot(n, oracle_mod.tri_analytic(x, *v)[1])
        assert abs(tot - want) < 1e-12, (x, tot)


# ----------------------------------------------------------- classification
def test_classification_rule(oracle_mod):
    p = sphere_problem(2)
    o = oracle_mod.Oracle(p, eta=6.0)
    cen = p.vert[p.tri].mean(axis=1)
    reg = o.classify(cen)
    assert np.all(np.diag(reg) == 0)          # self pairs are never regular
    g = [oracle_mod.panel_geometry(*p.vert[t]) for t in p.tri]
    cc = np.array([x["circumcenter"] for x in g])
    R = np.array([x["circumradius"] for x in g])
    D = np.linalg.norm(cen[:, None, :] - cc[None, :, :], axis=-1)
    assert np.array_equal(reg == 1, D > 6.0 * R[None, :])
    assert 80 < (reg == 0).sum(axis=1).mean() < 100    # about 88-90 near pairs per row


# -------------------------------------------------------------- sphere physics
def _solve(oracle_mod, p, eta=6.0, form=0):
    o = oracle_mod.Oracle(p, eta=eta, constraint_form=form)
    A = o.assemble()
    b = o.rhs(p.body_V)
    return o, A, b, np.linalg.solve(A, b)


def test_sphere_closed_form_and_convergence(oracle_mod):
    errs = []
    for lev in (2, 3, 4):
        p = sphere_problem(lev)
        o, A, b, x = _solve(oracle_mod, p)
        pts = sphere_eval_points()
        phi, E = o.eval(x, pts)
        r = np.linalg.norm(pts, axis=1)
        Eex = pts / r[:, None] ** 3
        err = (np.linalg.norm(E - Eex, axis=1) / np.linalg.norm(Eex, axis=1)).max()
        errs.append(err)
        if lev == 3:
            assert np.abs(x - 1.0).max() <= 1.5e-2
            assert err <= 5e-3
            assert np.abs(phi - 1.0 / r).max() <= 5e-3
    assert errs[1] / errs[2] >= 3.0 and errs[0] / errs[1] >= 3.0, errs


def test_gmres_matches_lu(oracle_mod):
    p = sphere_problem(3)
    o, A, b, x = _solve(oracle_mod, p)
    xg, it, rr, rc = oracle_mod.gmres(A, b, tol=1e-13)
    assert rc == 0 and rr <= 1e-13
    assert np.abs(xg - x).max() <= 1e-11 * np.abs(x).max()
    # a system that needs restarts (small restart length)
    pc = coax_problem(0.012)
    o2, A2, b2, x2 = _solve(oracle_mod, pc)
    xg2, it2, rr2, rc2 = oracle_mod.gmres(A2, b2, tol=1e-12, restart=10, max_iter=5000)
    assert rc2 == 0 and it2 > 10
    assert np.abs(xg2 - x2).max() <= 1e-9 * np.abs(x2).max()
    # non-convergence is reported
    _, it3, rr3, rc3 = oracle_mod.gmres(A2, b2, tol=1e-12, restart=100, max_iter=3)
    assert rc3 == 1 and it3 == 3 and rr3 > 1e-12


def test_sphere_symmetry_and_equivariance(oracle_mod):
    p = sphere_problem(3)
    o, A, b, x = _solve(oracle_mod, p)
    cen = p.vert[p.tri].mean(axis=1)
    # 2-fold rotations about the coordinate axes and the 3-fold rotation about (1,1,1)
    # map this icosphere onto itself
    rots = [np.diag([1.0, -1.0, -1.0]), np.diag([-1.0, 1.0, -1.0]),
            np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0]])]
    for Rm in rots:
        rc = cen @ Rm.T
        d = np.linalg.norm(rc[:, None, :] - cen[None, :, :], axis=-1)
        perm = d.argmin(axis=1)
        assert d[np.arange(len(perm)), perm].max() < 1e-12
        assert np.abs(x[perm] - x).max() < 1e-12
    # rotation, translation and scaling of the whole problem
    rng = np.random.default_rng(11)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    for s, sh in ((1.0, np.array([3.0, -2.0, 0.5])), (2.5, np.zeros(3)), (0.2, np.array([0.1, 0.0, 0.0]))):
        q = p.transformed(scale=s, rotation=Q, shift=sh)
        _, _, _, xq = _solve(oracle_mod, q)
        assert np.abs(xq * s - x).max() < 1e-11


def test_linearity_in_potential(oracle_mod):
    p = coax_problem(0.012)
    o = oracle_mod.Oracle(p)
    A = o.assemble()
    x1 = np.linalg.solve(A, o.rhs(p.body_V))
    x2 = np.linalg.solve(A, o.rhs(2.5 * p.body_V))
    assert np.abs(x2 - 2.5 * x1).max() <= 1e-10 * np.abs(x2).max()     # LU rounding x cond


def test_coated_sphere_interface_rows(oracle_mod):
    gold = GOLDEN["coated_sphere"]
    q = gold["q_over_V0"]
    rng = np.random.default_rng(2)
    d = rng.standard_normal((200, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    out = d * rng.uniform(2.0, 3.0, 200)[:, None]
    mid = d * 1.25
    errs_in = []
    for lev in (2, 3):
        p = coated_sphere_problem(lev, a=gold["a"], b=gold["b"], eps_r=gold["eps_r"])
        o, A, b, x = _solve(oracle_mod, p)
        _, E = o.eval(x, out)
        r = np.linalg.norm(out, axis=1)
        Eex = q * out / r[:, None] ** 3
        err_out = (np.linalg.norm(E - Eex, axis=1) / np.linalg.norm(Eex, axis=1)).max()
        _, Em = o.eval(x, mid)
        Eexm = q / gold["eps_r"] * mid / 1.25 ** 3
        errs_in.append((np.linalg.norm(Em - Eexm, axis=1) / np.linalg.norm(Eexm, axis=1)).max())
    # first-order convergence of the interface rows on flat panels
    assert err_out < 1.5e-2 and errs_in[1] < 4.5e-2
    assert errs_in[0] / errs_in[1] > 1.4, errs_in
    # eps+ == eps- makes the interface invisible: the bare-sphere solution exactly
    p2 = coated_sphere_problem(3, a=gold["a"], b=gold["b"], eps_r=1.0)
    _, A2, b2, x2 = _solve(oracle_mod, p2)
    nin = (p2.tri_body == 0).sum()
    assert np.abs(x2[nin:]).max() == 0.0
    ps = sphere_problem(3, radius=gold["a"])
    _, _, _, xs = _solve(oracle_mod, ps)
    assert np.abs(x2[:nin] - xs).max() < 1e-13


def test_floating_shell(oracle_mod):
    gold = GOLDEN["floating_shell"]
    errs = []
    for lev in (2, 3):
        p = floating_shell_problem(lev, a=gold["a"], b1=gold["b1"], b2=gold["b2"])
        o, A, b, x = _solve(oracle_mod, p)
        N = p.n_tri
        errs.append(abs(x[N] - gold["Vf_over_V0"]))
        # the reduced (net charge) constraint: same limit, smaller error
        _, _, _, x1 = _solve(oracle_mod, p, form=1)
        assert abs(x1[N] - gold["Vf_over_V0"]) < 1e-3
    assert errs[1] < 1.5e-2 and errs[0] / errs[1] > 1.8, errs
    # net charge of the floating body: small for the literal row, zero for the reduced row
    area = 0.5 * np.linalg.norm(np.cross(p.vert[p.tri[:, 1]] - p.vert[p.tri[:, 0]],
                                         p.vert[p.tri[:, 2]] - p.vert[p.tri[:, 0]]), axis=1)
    m = p.tri_body == 1
    assert abs(np.sum(area[m] * x[:N][m])) < 5e-2 * np.sum(np.abs(area[m] * x[:N][m]))
    assert abs(np.sum(area[m] * x1[:N][m])) < 1e-12 * np.sum(np.abs(area[m] * x1[:N][m]))


@pytest.mark.parametrize("case", range(2))
def test_floating_sheet_closed_form(oracle_mod, case):
    """A thin floating sheet (Eq. sheets) between two dielectrics: its potential and the
    field outside converge to the closed form, and the physical charge of the sheet,
    sum_i a_i ((eps+ + eps-)/2 sigma_i + (eps+ - eps-) (K' sigma)_i), is zero."""
    gold = GOLDEN["sphere_sheet"]["cases"][case]
    errs, errE = [], []
    for lev in (2, 3):
        p = sphere_sheet_problem(lev, a=gold["a"], b=gold["b"], eps_in=gold["eps_in"], eps_out=gold["eps_out"])
        o, A, b, x = _solve(oracle_mod, p)
        N = p.n_tri
        assert x.shape[0] == N + 1
        errs.append(abs(x[N] - gold["Vf_over_V0"]))
        pts = sphere_eval_points(200, seed=2, rmin=3.0, rmax=4.0)
        _, E = o.eval(x, pts)
        r = np.linalg.norm(pts, axis=1)
        errE.append(np.max(np.abs(np.linalg.norm(E, axis=1) - gold["C_over_V0"] / r ** 2) / (gold["C_over_V0"] / r ** 2)))
        # the constraint row is the sheet's net charge (scaled): A[N] . x = 0 to rounding
        assert abs(A[N] @ x) < 1e-12 * np.abs(A[N]).sum() * np.abs(x[:N]).max()
        # the net-charge form of closed floating bodies does not apply to an open sheet
        _, A1, _, x1 = _solve(oracle_mod, p, form=1)
        assert np.array_equal(A1, A) and abs(x1[N] - x[N]) < 1e-13
    # converging (the K' term of the sheet row makes the potential's order below one on these
    # meshes); a dropped eps weighting would give 0.5, a swapped eps+ - eps- sign 0.2
    assert errs[1] < 1e-2 and errs[0] / errs[1] > 1.4, errs
    assert errE[1] < 2e-2 and errE[0] / errE[1] > 1.8, errE


def test_coax_floating_ring_maximum_principle(oracle_mod):
    p = coax_problem(0.012)
    o, A, b, x = _solve(oracle_mod, p)
    V = x[p.n_tri]
    assert 0.0 < V < 1.0
    # a ring at rho = 0.05 in an infinite coax would sit at ln(0.1/0.05)/ln(5)
    assert abs(V - math.log(2) / math.log(5)) < 0.05


# ------------------------------------------------------------------ evaluation
def test_eval_gauss_flux_and_gradient(oracle_mod):
    p = sphere_problem(3)
    o, A, b, x = _solve(oracle_mod, p)
    area = 0.5 * np.linalg.norm(np.cross(p.vert[p.tri[:, 1]] - p.vert[p.tri[:, 0]],
                                         p.vert[p.tri[:, 2]] - p.vert[p.tri[:, 0]]), axis=1)
    # flux through r = 2 (all pairs regular: seven point charges per panel) = total charge
    ct, wt = np.polynomial.legendre.leggauss(48)
    nphi = 96
    ph = (np.arange(nphi) + 0.5) * 2 * math.pi / nphi
    C, PH = np.meshgrid(ct, ph, indexing="ij")
    st = np.sqrt(1 - C ** 2)
    nrm = np.stack([st * np.cos(PH), st * np.sin(PH), C], -1).reshape(-1, 3)
    W = (np.outer(wt, np.full(nphi, 2 * math.pi / nphi))).reshape(-1) * 4.0
    _, E = o.eval(x, 2.0 * nrm)
    flux = np.sum(W * np.einsum("ij,ij->i", E, nrm))
    assert abs(flux - np.sum(area * x)) < 1e-10 * abs(flux)
    # E = -grad phi
    pts = sphere_eval_points(20, seed=9)
    _, E0 = o.eval(x, pts)
    h = 1e-5
    for k in range(3):
        e = np.zeros(3)
        e[k] = h
        gp, _ = o.eval(x, pts + e)
        gm, _ = o.eval(x, pts - e)
        assert np.abs(E0[:, k] + (gp - gm) / (2 * h)).max() < 1e-8


def test_on_surface_exterior_limit(oracle_mod):
    p = sphere_problem(3)
    o, A, b, x = _solve(oracle_mod, p)
    cen = p.vert[p.tri].mean(axis=1)
    nrm = np.cross(p.vert[p.tri[:, 1]] - p.vert[p.tri[:, 0]], p.vert[p.tri[:, 2]] - p.vert[p.tri[:, 0]])
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    idx = np.arange(0, p.n_tri, 37)
    phi, Es = o.eval(x, cen[idx], on_panel=idx)
    # potential on the collocation points is V0 (the Dirichlet rows)
    assert np.abs(phi - 1.0).max() < 1e-12
    # exterior limit agrees with points slightly outside
    _, Eo = o.eval(x, cen[idx] + 1e-7 * nrm[idx])
    assert np.abs(Es - Eo).max() < 1e-5 * np.abs(Es).max()
    # and is close to the closed form |E| = 1 on the unit sphere
    assert np.abs(np.linalg.norm(Es, axis=1) - 1.0).max() < 5e-2     # O(h) flat-panel surface error


# ------------------------------------------------------------------- tracing
def _alpha(E, a=1e-3, e0=25.0, p=2.0):
    return a * np.maximum(E - e0, 0.0) ** p


def test_trace_radial_point_charge(oracle_mod):
    # E = q x/|x|^3: straight radial lines; the integral is Simpson's rule of int alpha(q/r^2) dr
    q = 50.0
    start = np.array([[1.0, 0.0, 0.0], [0.0, 0.6, 0.8]])
    res = []
    for h in (4e-3, 2e-3, 1e-3):
        n = int(round(0.2 / h))
        tp = oracle_mod.trace_params(h=h, max_steps=n, e_min=1e-3)
        ns, st, I, path = oracle_mod.trace_charges([[0, 0, 0]], [q], start, tp, want_path=True)
        assert np.all(ns == n) and np.all(st == 0)
        r = np.linalg.norm(path[:, n], axis=1)
        assert np.abs(r - 1.2).max() < 1e-12
        res.append(I[0])
    rr = np.linspace(1.0, 1.2, 200001)
    f = _alpha(q / rr ** 2)
    exact = np.sum((f[1:] + f[:-1]) * 0.5 * np.diff(rr))       # trapezoid reference on a fine grid
    # refine the reference with Richardson to remove its O(dr^2) error
    rr2 = np.linspace(1.0, 1.2, 100001)
    f2 = _alpha(q / rr2 ** 2)
    exact2 = np.sum((f2[1:] + f2[:-1]) * 0.5 * np.diff(rr2))
    exact = (4 * exact - exact2) / 3
    e = [abs(x - exact) for x in res]
    assert e[2] < 1e-10
    assert 12.0 < e[0] / e[1] < 20.0 and 12.0 < e[1] / e[2] < 20.0, e


def test_trace_two_charges_rk4_order(oracle_mod):
    # field lines of two charges on the z axis conserve q1 cos(th1) + q2 cos(th2)
    c = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    qs = np.array([1.0, -0.5])

    def invariant(x):
        d1, d2 = x - c[0], x - c[1]
        return qs[0] * d1[2] / np.linalg.norm(d1) + qs[1] * d2[2] / np.linalg.norm(d2)

    start = np.array([[0.2, 0.1, 0.05]])
    errs = []
    for h in (0.02, 0.01, 0.005):
        n = int(round(0.6 / h))
        tp = oracle_mod.trace_params(h=h, max_steps=n, e_min=0.0, alpha_a=0.0)
        ns, st, I, path = oracle_mod.trace_charges(c, qs, start, tp, want_path=True)
        assert ns[0] == n
        errs.append(abs(invariant(path[0, n]) - invariant(path[0, 0])))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 12.0 < r1 < 22.0 and 12.0 < r2 < 22.0, errs


def test_trace_stop_codes_charges(oracle_mod):
    tp = oracle_mod.trace_params(h=1e-2, max_steps=50, e_min=1e-3)
    # |E| below e_min at the start: stop 4 with no step
    ns, st, I = oracle_mod.trace_charges([[0, 0, 0]], [1.0], [[100.0, 0, 0]], tp)
    assert ns[0] == 0 and st[0] == 4 and I[0] == 0.0
    # direction -1 runs towards a positive charge
    tp2 = oracle_mod.trace_params(h=1e-2, max_steps=50, e_min=1e-3, direction=-1)
    ns, st, I, path = oracle_mod.trace_charges([[0, 0, 0]], [1.0], [[1.0, 0, 0]], tp2, want_path=True)
    assert ns[0] == 50 and st[0] == 0 and abs(path[0, 50, 0] - 0.5) < 1e-12


def _mt_free_hit(x0, x1, v):
    """Plane-intersection + barycentric test (independent of Moeller-Trumbore)."""
    n = np.cross(v[1] - v[0], v[2] - v[0])
    d0, d1 = np.dot(x0 - v[0], n), np.dot(x1 - v[0], n)
    if d0 == d1:
        return None
    t = d0 / (d0 - d1)
    if t < 0 or t > 1:
        return None
    y = x0 + t * (x1 - x0)
    T = np.stack([v[1] - v[0], v[2] - v[0]], 1)
    uv, *_ = np.linalg.lstsq(T, y - v[0], rcond=None)
    if uv[0] < 0 or uv[1] < 0 or uv.sum() > 1:
        return None
    return t


def test_segment_hit_against_independent_test(oracle_mod):
    p = sphere_problem(1)
    o = oracle_mod.Oracle(p)
    rng = np.random.default_rng(3)
    agree = 0
    for _ in range(300):
        x0 = rng.uniform(-1.3, 1.3, 3)
        x1 = x0 + rng.standard_normal(3) * 0.3
        j, t = o.segment_hit(x0, x1)
        best = None
        for k, tr in enumerate(p.tri):
            tt = _mt_free_hit(x0, x1, p.vert[tr])
            if tt is not None and (best is None or tt < best[1]):
                best = (k, tt)
        if best is None:
            assert j == -1
        else:
            assert j == best[0] and abs(t - best[1]) < 1e-12
            agree += 1
    assert agree > 20


def test_sphere_bem_trace(oracle_mod):
    # V0 = 50 on the unit sphere: radial lines, 2000 steps of 1e-4 -> r = 1.2, code 0
    p = sphere_problem(3, V0=50.0)
    o, A, b, x = _solve(oracle_mod, p)
    from workloads import electrode_line_starts
    starts, panel, bary = electrode_line_starts(p, 4, seed=6)
    tp = oracle_mod.trace_params(h=1e-4, max_steps=2000)
    ns, st, I, path = o.trace(x, starts, tp, want_path=True)
    assert np.all(ns == 2000) and np.all(st == 0)
    r = np.linalg.norm(path[:, 2000], axis=1)
    assert np.all(np.abs(r - np.linalg.norm(starts, axis=1) - 0.2) < 2e-3)
    rr = np.linspace(1.0, 1.2, 20001)
    f = _alpha(50.0 / rr ** 2)
    exact = np.sum((f[1:] + f[:-1]) * 0.5 * np.diff(rr))
    assert np.abs(I / exact - 1.0).max() < 5e-2
    # a line started inward hits the sphere at once: code 1, no step
    tp_in = oracle_mod.trace_params(h=1e-4, max_steps=10, direction=-1)
    ns, st, I = o.trace(x, starts[:1], tp_in)
    assert ns[0] == 0 and st[0] == 1 and I[0] == 0.0
