"""TEST INFRASTRUCTURE ONLY: ctypes wrapper of the plain FP64 CPU oracle.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the GPU library; both receive
the same seeded inputs from `workloads`.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_SRC_DUAL = os.path.join(_HERE, "oracle_dual.c")
_LIB = os.path.join(_HERE, "liboracle.so")

DIRICHLET, FLOATING, INTERFACE, SHEET = 0, 1, 2, 3


_FLAGS = ["-O3", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]


def build(force: bool = True) -> str:
    """Compile oracle.c and oracle_dual.c into liboracle.so (gcc -O3, no FMA contraction, no
    fast-math).  This in-tree build targets x86-64-v3 (AVX2), which every host it is shipped
    to runs; build_native() makes a copy tuned for the host it runs on."""
    stale = (not os.path.exists(_LIB)
             or os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC), os.path.getmtime(_SRC_DUAL)))
    if force or stale:
        tmp = _LIB + ".tmp"
        cmd = ["gcc", *_FLAGS, "-march=x86-64-v3", "-o", tmp, _SRC, _SRC_DUAL, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def build_native(out_dir: str) -> str:
    """Compile the oracle with -O3 -march=native for the CPU it runs on (the timed CPU
    baseline), into out_dir, and load that copy for this process.  Must be called before
    any other use of the oracle in the process."""
    global _lib
    if _lib is not None:
        raise RuntimeError("the oracle library is already loaded")
    os.makedirs(out_dir, exist_ok=True)
    path = os.path.join(out_dir, "liboracle_native.so")
    cmd = ["gcc", *_FLAGS, "-march=native", "-o", path, _SRC, _SRC_DUAL, "-lm"]
    subprocess.run(cmd, check=True)
    _lib = ctypes.CDLL(path)
    return path


def num_threads() -> int:
    """OpenMP threads the oracle's parallel loops use (omp_get_max_threads)."""
    return int(_load().orc_num_threads())


class _Problem(ctypes.Structure):
    _fields_ = [
        ("n_vert", ctypes.c_int64), ("vert", ctypes.c_void_p),
        ("n_tri", ctypes.c_int64), ("tri", ctypes.c_void_p), ("tri_body", ctypes.c_void_p),
        ("n_body", ctypes.c_int32), ("body_kind", ctypes.c_void_p),
        ("eps_plus", ctypes.c_void_p), ("eps_minus", ctypes.c_void_p),
        ("eta", ctypes.c_double), ("constraint_form", ctypes.c_int32),
    ]


class TraceParams(ctypes.Structure):
    _fields_ = [
        ("h", ctypes.c_double), ("e_min", ctypes.c_double), ("start_offset", ctypes.c_double),
        ("max_steps", ctypes.c_int32), ("direction", ctypes.c_int32),
        ("alpha_a", ctypes.c_double), ("alpha_e0", ctypes.c_double), ("alpha_p", ctypes.c_double),
        ("k_str", ctypes.c_double),
    ]


def trace_params(h=1e-4, e_min=1e-3, max_steps=2000, direction=1, alpha_a=1e-3, alpha_e0=25.0,
                 alpha_p=2.0, k_str=0.0, start_offset=1e-6) -> TraceParams:
    return TraceParams(h, e_min, start_offset, max_steps, direction, alpha_a, alpha_e0, alpha_p, k_str)


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = ctypes.CDLL(_LIB)
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else ctypes.c_void_p(0)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a.reshape(shape) if shape is not None else a


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class Oracle:
    """Holds one problem (mesh + body table + eta) for the oracle calls."""

    def __init__(self, problem, eta: float = 6.0, constraint_form: int = 0):
        self.lib = _load()
        self.problem = problem
        self._keep = [_f64(problem.vert), _i32(problem.tri), _i32(problem.tri_body), _i32(problem.body_kind),
                      _f64(problem.eps_plus), _f64(problem.eps_minus)]
        v, t, tb, bk, ep, em = self._keep
        self.p = _Problem(len(v), _ptr(v), len(t), _ptr(t), _ptr(tb), len(bk), _ptr(bk), _ptr(ep), _ptr(em),
                          float(eta), int(constraint_form))
        self.N = len(t)
        self.n = int(self.lib.orc_n_unknowns(ctypes.byref(self.p)))

    # -- geometry and single-pair integrals (module-level helpers below) --
    def assemble(self) -> np.ndarray:
        A = np.empty((self.n, self.n), dtype=np.float64)
        self.lib.orc_assemble(ctypes.byref(self.p), _ptr(A))
        return A

    def assemble_rows(self, rows) -> np.ndarray:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        out = np.empty((len(rows), self.n), dtype=np.float64)
        self.lib.orc_assemble_rows(ctypes.byref(self.p), ctypes.c_int64(len(rows)), _ptr(rows), _ptr(out))
        return out

    def rhs(self, body_V) -> np.ndarray:
        bv = _f64(body_V)
        b = np.empty(self.n, dtype=np.float64)
        self.lib.orc_rhs(ctypes.byref(self.p), _ptr(bv), _ptr(b))
        return b

    # -- nodal linear basis, vertex collocation (Sec. 3, Eq. Matrix) --
    @property
    def n_p1(self) -> int:
        return int(self.lib.orc_p1_n_unknowns(ctypes.byref(self.p)))

    def p1_assemble(self) -> np.ndarray:
        A = np.empty((self.n_p1, self.n_p1), dtype=np.float64)
        rc = self.lib.orc_p1_assemble(ctypes.byref(self.p), _ptr(A))
        if rc != 0:
            raise ValueError(f"orc_p1_assemble: {rc}")
        return A

    def p1_assemble_rows(self, rows) -> np.ndarray:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        out = np.empty((len(rows), self.n_p1), dtype=np.float64)
        rc = self.lib.orc_p1_assemble_rows(ctypes.byref(self.p), ctypes.c_int64(len(rows)), _ptr(rows), _ptr(out))
        if rc != 0:
            raise ValueError(f"orc_p1_assemble_rows: {rc}")
        return out

    def p1_rhs(self, body_V) -> np.ndarray:
        bv = _f64(body_V)
        b = np.empty(self.n_p1, dtype=np.float64)
        rc = self.lib.orc_p1_rhs(ctypes.byref(self.p), _ptr(bv), _ptr(b))
        if rc != 0:
            raise ValueError(f"orc_p1_rhs: {rc}")
        return b

    def p1_potential(self, u, pts) -> np.ndarray:
        u = _f64(u)
        pts = _f64(pts, (-1, 3))
        phi = np.empty(len(pts), dtype=np.float64)
        self.lib.orc_p1_potential(ctypes.byref(self.p), _ptr(u), ctypes.c_int64(len(pts)), _ptr(pts), _ptr(phi))
        return phi

    def p1_field(self, u, pts):
        """(phi [P], E [P, 3]) of the nodal density u at volume points."""
        u = _f64(u)
        pts = _f64(pts, (-1, 3))
        phi = np.empty(len(pts), dtype=np.float64)
        E = np.empty((len(pts), 3), dtype=np.float64)
        self.lib.orc_p1_field(ctypes.byref(self.p), _ptr(u), ctypes.c_int64(len(pts)), _ptr(pts), _ptr(phi), _ptr(E))
        return phi, E

    def classify(self, pts) -> np.ndarray:
        pts = _f64(pts, (-1, 3))
        out = np.empty((len(pts), self.N), dtype=np.int32)
        self.lib.orc_classify(ctypes.byref(self.p), ctypes.c_int64(len(pts)), _ptr(pts), _ptr(out))
        return out

    def eval(self, sigma, pts, on_panel=None):
        sigma = _f64(sigma)
        pts = _f64(pts, (-1, 3))
        P = len(pts)
        op = _i32(on_panel) if on_panel is not None else None
        phi = np.empty(P, dtype=np.float64)
        E = np.empty((P, 3), dtype=np.float64)
        self.lib.orc_eval(ctypes.byref(self.p), _ptr(sigma), ctypes.c_int64(P), _ptr(pts), _ptr(op), _ptr(phi),
                          _ptr(E))
        return phi, E

    def segment_hit(self, x0, x1):
        x0, x1 = _f64(x0), _f64(x1)
        panel = ctypes.c_int64(0)
        t = ctypes.c_double(0.0)
        self.lib.orc_segment_hit(ctypes.byref(self.p), _ptr(x0), _ptr(x1), ctypes.byref(panel), ctypes.byref(t))
        return int(panel.value), float(t.value)

    def trace(self, sigma, starts, params: TraceParams, want_path=False):
        sigma = _f64(sigma)
        starts = _f64(starts, (-1, 3))
        L = len(starts)
        ns = np.empty(L, dtype=np.int32)
        st = np.empty(L, dtype=np.int32)
        I = np.empty(L, dtype=np.float64)
        path = np.full((L, params.max_steps + 1, 3), np.nan) if want_path else None
        self.lib.orc_trace(ctypes.byref(self.p), _ptr(sigma), ctypes.c_int64(L), _ptr(starts), ctypes.byref(params),
                           _ptr(ns), _ptr(st), _ptr(I), _ptr(path))
        return (ns, st, I, path) if want_path else (ns, st, I)

    def p1_trace(self, u, starts, params: TraceParams, want_path=False):
        """Field lines and streamer integrals of the nodal density u (orc_p1_trace)."""
        u = _f64(u)
        starts = _f64(starts, (-1, 3))
        L = len(starts)
        ns = np.empty(L, dtype=np.int32)
        st = np.empty(L, dtype=np.int32)
        I = np.empty(L, dtype=np.float64)
        path = np.full((L, params.max_steps + 1, 3), np.nan) if want_path else None
        self.lib.orc_p1_trace(ctypes.byref(self.p), _ptr(u), ctypes.c_int64(L), _ptr(starts), ctypes.byref(params),
                              _ptr(ns), _ptr(st), _ptr(I), _ptr(path))
        return (ns, st, I, path) if want_path else (ns, st, I)

    def dual_streamer(self, dvert, body_V, dbody_V, start_panel, start_bary, params: TraceParams, n_steps,
                      tol=1e-13):
        """Forward-mode derivative of the streamer integrals along (dvert, dbody_V), with the
        classification and the per-line step counts n_steps held fixed.  Line l starts at
        sum_k bary_k v_k + params.start_offset * n of its panel.  Returns (I, dI, u, du, rc)."""
        dv = _f64(dvert, (-1, 3)) if dvert is not None else None
        bv = _f64(body_V)
        dbv = _f64(dbody_V) if dbody_V is not None else None
        sp = _i32(start_panel)
        sb = _f64(start_bary, (-1, 3))
        ns = _i32(n_steps)
        L = len(sp)
        I = np.empty(L)
        dI = np.empty(L)
        u = np.empty(self.n)
        du = np.empty(self.n)
        rc = self.lib.orc_dual_streamer(ctypes.byref(self.p), _ptr(dv), _ptr(bv), _ptr(dbv), ctypes.c_int64(L),
                                        _ptr(sp), _ptr(sb), ctypes.c_double(params.start_offset),
                                        ctypes.byref(params), _ptr(ns), ctypes.c_double(tol), _ptr(u), _ptr(du),
                                        _ptr(I), _ptr(dI))
        return I, dI, u, du, int(rc)


def gmres(A, b, tol=1e-13, restart=100, max_iter=10000):
    lib = _load()
    A = _f64(A)
    b = _f64(b)
    n = len(b)
    x = np.empty(n, dtype=np.float64)
    it = ctypes.c_int32(0)
    rr = ctypes.c_double(0.0)
    rc = lib.orc_gmres(ctypes.c_int64(n), _ptr(A), _ptr(b), ctypes.c_double(tol), ctypes.c_int32(restart),
                       ctypes.c_int32(max_iter), _ptr(x), ctypes.byref(it), ctypes.byref(rr))
    return x, int(it.value), float(rr.value), int(rc)


def panel_geometry(v1, v2, v3):
    lib = _load()
    v1, v2, v3 = _f64(v1), _f64(v2), _f64(v3)
    cen, nrm, cc = np.empty(3), np.empty(3), np.empty(3)
    area, R = ctypes.c_double(0), ctypes.c_double(0)
    lib.orc_panel_geometry(_ptr(v1), _ptr(v2), _ptr(v3), _ptr(cen), _ptr(nrm), ctypes.byref(area), _ptr(cc),
                           ctypes.byref(R))
    return dict(centroid=cen, normal=nrm, area=area.value, circumcenter=cc, circumradius=R.value)


def quad7_rule():
    lib = _load()
    bary = np.empty((7, 3))
    w = np.empty(7)
    lib.orc_quad7_rule(_ptr(bary), _ptr(w))
    return bary, w


def tri_analytic(x, v1, v2, v3, on_plane=False):
    lib = _load()
    x, v1, v2, v3 = _f64(x), _f64(v1), _f64(v2), _f64(v3)
    S = ctypes.c_double(0)
    F = np.empty(3)
    lib.orc_tri_analytic(_ptr(x), _ptr(v1), _ptr(v2), _ptr(v3), ctypes.c_int(int(on_plane)), ctypes.byref(S),
                         _ptr(F))
    return S.value, F


def tri_linear_analytic(x, v1, v2, v3, on_plane=False):
    """int lambda_k / (4 pi |x - y|) dS over the flat triangle for its three vertices."""
    lib = _load()
    out = np.empty(3, dtype=np.float64)
    a = [_f64(v) for v in (x, v1, v2, v3)]
    lib.orc_tri_linear_analytic(*[_ptr(v) for v in a], ctypes.c_int(1 if on_plane else 0), _ptr(out))
    return out


def tri_linear_field(x, v1, v2, v3):
    """int lambda_k (x - y) / (4 pi |x - y|^3) dS over the flat triangle, [3 vertices][3]."""
    lib = _load()
    out = np.empty((3, 3), dtype=np.float64)
    a = [_f64(v) for v in (x, v1, v2, v3)]
    lib.orc_tri_linear_field(*[_ptr(v) for v in a], _ptr(out))
    return out


def tri_duffy(x, v1, v2, v3):
    """The paper's near-singular rule (closest point, subdivision, Duffy, Gauss-Legendre) for a
    unit-density flat triangle: (S, F); F is NaN when x lies on the triangle."""
    lib = _load()
    S = ctypes.c_double(0.0)
    F = np.empty(3)
    lib.orc_tri_duffy(*(_ptr(_f64(a)) for a in (x, v1, v2, v3)), ctypes.byref(S), _ptr(F))
    return S.value, F


def quad_duffy(x, nodes):
    """The near-singular rule of Sec. 4 on a curved quadratic panel (six nodes: the corners,
    then the edge nodes of edges 1-2, 2-3, 3-1): (S, F) of unit density at x; F is NaN when x
    lies on the panel."""
    lib = _load()
    S = ctypes.c_double(0.0)
    F = np.empty(3)
    P = np.ascontiguousarray(np.asarray(nodes, dtype=np.float64).reshape(6, 3))
    lib.orc_quad_duffy(_ptr(_f64(x)), _ptr(P), ctypes.byref(S), _ptr(F))
    return S.value, F


def quad_closest(x, nodes):
    """Parameter point (s, t) of the reference triangle whose image on the quadratic panel is
    closest to x (step 1 of the rule)."""
    lib = _load()
    c = np.empty(2)
    P = np.ascontiguousarray(np.asarray(nodes, dtype=np.float64).reshape(6, 3))
    lib.orc_quad_closest(_ptr(P), _ptr(_f64(x)), _ptr(c))
    return c


def closest_point(x, v1, v2, v3):
    """Closest point of the closed triangle to x (step 1 of the near-singular rule)."""
    lib = _load()
    c = np.empty(3)
    lib.orc_closest_point(*(_ptr(_f64(a)) for a in (x, v1, v2, v3)), _ptr(c))
    return c


def tri_quad7(x, v1, v2, v3):
    lib = _load()
    x, v1, v2, v3 = _f64(x), _f64(v1), _f64(v2), _f64(v3)
    S = ctypes.c_double(0)
    F = np.empty(3)
    lib.orc_tri_quad7(_ptr(x), _ptr(v1), _ptr(v2), _ptr(v3), ctypes.byref(S), _ptr(F))
    return S.value, F


def trace_charges(centres, charges, starts, params: TraceParams, want_path=False):
    lib = _load()
    c = _f64(centres, (-1, 3))
    q = _f64(charges)
    starts = _f64(starts, (-1, 3))
    L = len(starts)
    ns = np.empty(L, dtype=np.int32)
    st = np.empty(L, dtype=np.int32)
    I = np.empty(L, dtype=np.float64)
    path = np.full((L, params.max_steps + 1, 3), np.nan) if want_path else None
    lib.orc_trace_charges(ctypes.c_int32(len(q)), _ptr(c), _ptr(q), ctypes.c_int64(L), _ptr(starts),
                          ctypes.byref(params), _ptr(ns), _ptr(st), _ptr(I), _ptr(path))
    return (ns, st, I, path) if want_path else (ns, st, I)
