"""Pins of the oracle's forward-mode (dual-number) derivative of the streamer integrals.

The dual oracle redoes geometry, the system of Eqs. Final1-Final4, the solve and
the RK4 field lines with the integral of Eq. Breakdowncrit in dual arithmetic.
It is pinned here by things that do not come from it:
  * its value part equals the plain oracle's streamer integrals,
  * its derivative equals central finite differences of the plain oracle
    (mesh, solve, line starts and lines all recomputed at the perturbed
    vertices, h = 1e-6), for conductor, floating-conductor (both constraint
    forms), thin-sheet and dielectric-interface rows, and for body potentials,
  * rigid motions of the whole mesh (line starts move with their panels) leave
    every integral unchanged, so the derivative along a translation or an
    infinitesimal rotation vanishes.
The coax case has coplanar panels, where a collocation point lies in the plane
of another panel outside it: the normal field is smooth there and its
derivative must not vanish with sign(w).
"""

import dataclasses

import numpy as np
import pytest

from workloads import (bushing_problem, coated_sphere_problem, coax_problem, electrode_line_starts, floating_shell_problem,
                       sphere_problem, sphere_sheet_problem, union_problem)


def _setup(oracle_mod, p, L, steps, h, constraint_form=0, seed=6):
    starts, panel, bary = electrode_line_starts(p, L, seed=seed)
    tp = oracle_mod.trace_params(h=h, max_steps=steps, e_min=1e-3)
    o = oracle_mod.Oracle(p, constraint_form=constraint_form)
    return starts, panel, bary, tp, o


def _plain_I(oracle_mod, p, vert, body_V, panel, bary, tp, constraint_form=0):
    """Plain oracle at (vert, body_V): assemble, dense solve, starts on the moved panels, trace."""
    q = dataclasses.replace(p, vert=vert)
    o = oracle_mod.Oracle(q, constraint_form=constraint_form)
    A = o.assemble()
    u = np.linalg.solve(A, o.rhs(body_V))
    a, b, c = (vert[q.tri[panel, k]] for k in range(3))
    cr = np.cross(b - a, c - a)
    nrm = cr / np.linalg.norm(cr, axis=1, keepdims=True)
    starts = bary[:, :1] * a + bary[:, 1:2] * b + bary[:, 2:3] * c + tp.start_offset * nrm
    ns, st, I = o.trace(u[:q.n_tri], starts, tp)
    return ns, st, I


def _sheet_and_shell():
    return union_problem(sphere_sheet_problem(1, V0=100.0, eps_in=4.0), floating_shell_problem(1, V0=50.0),
                         (6.0, 0.0, 0.0))


CASES = [
    # (problem, lines, steps, h, constraint form)
    ("sphere", lambda: sphere_problem(1, V0=50.0), 4, 60, 1e-2, 0),
    ("floating_shell", lambda: floating_shell_problem(1, V0=50.0), 4, 30, 5e-3, 0),
    ("floating_shell_reduced", lambda: floating_shell_problem(1, V0=50.0), 4, 30, 5e-3, 1),
    ("coated_sphere", lambda: coated_sphere_problem(1, V0=200.0), 4, 30, 5e-3, 0),
    # coplanar panels (disc faces, caps): collocation points in the plane of other panels
    ("coarse_coax", lambda: coax_problem(0.03, V0=30.0), 3, 60, 2e-4, 0),
    # a thin floating sheet between two dielectrics (Eq. sheets row, K' weighted by eps+ - eps-)
    ("sphere_sheet", lambda: sphere_sheet_problem(1, V0=100.0, eps_in=4.0), 4, 30, 5e-3, 0),
    # two floating bodies with different constraint rows: the sheet above and a closed shell,
    # the shell's row literal (form 0) or the net charge (form 1)
    ("sheet_and_shell", lambda: _sheet_and_shell(), 6, 30, 5e-3, 0),
    ("sheet_and_shell_reduced", lambda: _sheet_and_shell(), 6, 30, 5e-3, 1),
    # four floating sheets in one insulator (eps+ = eps-) and its interface; lines end on the first foil
    ("bushing", lambda: bushing_problem(0.08, V0=5.0), 6, 40, 2e-3, 0),
]


# Residual of the dual solves: 1e-15 where GMRES reaches it, else the smallest it reaches.  The
# default 1e-13 leaves ~cond(A) 1e-13 of solution error (cond ~ 5e2 on the two-device case),
# more than the 1e-12 value-part bar.
DUAL_TOL = {"coarse_coax": 1e-13, "bushing": 1e-14}


@pytest.mark.parametrize("name,make,L,steps,h,cf", CASES, ids=[c[0] for c in CASES])
def test_dual_matches_finite_differences(oracle_mod, name, make, L, steps, h, cf):
    p = make()
    starts, panel, bary, tp, o = _setup(oracle_mod, p, L, steps, h, cf)
    ns, st, I0 = _plain_I(oracle_mod, p, p.vert, p.body_V, panel, bary, tp, cf)
    assert np.all(I0 > 0.0), "the case must have a non-trivial integral"
    dv = np.random.default_rng(8).standard_normal(p.vert.shape)
    I, dI, u, du, rc = o.dual_streamer(dv, p.body_V, None, panel, bary, tp, ns, tol=DUAL_TOL.get(name, 1e-15))
    assert rc == 0
    # value part = the plain oracle
    assert np.max(np.abs(I - I0)) <= 1e-12 * np.max(np.abs(I0))
    hfd = 1e-6 if name != "coarse_coax" else 1e-7   # the coax mesh is ten times finer
    nsp, stp, Ip = _plain_I(oracle_mod, p, p.vert + hfd * dv, p.body_V, panel, bary, tp, cf)
    nsm, stm, Im = _plain_I(oracle_mod, p, p.vert - hfd * dv, p.body_V, panel, bary, tp, cf)
    assert np.array_equal(nsp, ns) and np.array_equal(nsm, ns), "step counts moved under the perturbation"
    fd = (Ip - Im) / (2 * hfd)
    assert np.max(np.abs(dI - fd)) <= 1e-6 * np.max(np.abs(fd))


def test_dual_body_potential(oracle_mod):
    """dI/dV of the driven body against central differences in V."""
    p = floating_shell_problem(1, V0=50.0)
    starts, panel, bary, tp, o = _setup(oracle_mod, p, 4, 30, 5e-3)
    ns, st, I0 = _plain_I(oracle_mod, p, p.vert, p.body_V, panel, bary, tp)
    dV = np.zeros(p.n_body)
    dV[0] = 1.0
    I, dI, u, du, rc = o.dual_streamer(None, p.body_V, dV, panel, bary, tp, ns)
    hfd = 1e-5
    _, _, Ip = _plain_I(oracle_mod, p, p.vert, p.body_V + hfd * dV, panel, bary, tp)
    _, _, Im = _plain_I(oracle_mod, p, p.vert, p.body_V - hfd * dV, panel, bary, tp)
    fd = (Ip - Im) / (2 * hfd)
    assert np.max(np.abs(dI - fd)) <= 1e-7 * np.max(np.abs(fd))
    # du is the solution for a unit potential on body 0 (linearity): A du = b(e_0)
    A = o.assemble()
    assert np.max(np.abs(A @ du - o.rhs(dV))) <= 1e-11


@pytest.mark.parametrize("motion", ["translation", "rotation"])
def test_dual_rigid_motion_is_zero(oracle_mod, motion):
    p = floating_shell_problem(1, V0=50.0)
    starts, panel, bary, tp, o = _setup(oracle_mod, p, 4, 30, 5e-3)
    ns, st, I0 = _plain_I(oracle_mod, p, p.vert, p.body_V, panel, bary, tp)
    if motion == "translation":
        dv = np.tile(np.array([0.3, -0.7, 0.5]), (len(p.vert), 1))
    else:
        w = np.array([0.2, 0.5, -0.4])
        dv = np.cross(w, p.vert)
    I, dI, u, du, rc = o.dual_streamer(dv, p.body_V, None, panel, bary, tp, ns)
    # scale: derivative along a generic direction of the same size
    g = np.random.default_rng(8).standard_normal(p.vert.shape)
    g *= np.linalg.norm(dv) / np.linalg.norm(g)
    _, dIg, _, _, _ = o.dual_streamer(g, p.body_V, None, panel, bary, tp, ns)
    assert np.max(np.abs(dI)) <= 1e-9 * np.max(np.abs(dIg))
