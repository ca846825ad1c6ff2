"""MI355X (gfx950) indirect single-layer collocation BEM.

Python binding of the C ABI in include/bem.h.  Every numerical step runs in
the HIP kernels of libbem.so; this module only marshals arguments.  torch
supplies device memory and the stream.  There is no CPU fallback: without the
built library or a gfx950 GPU every call raises.
"""

from __future__ import annotations

import ctypes

import numpy as np

from . import _lib

DIRICHLET, FLOATING, INTERFACE, FLOATING_SHEET = 0, 1, 2, 3
FP64, MIXED = 0, 1
BASIS_CONSTANT, BASIS_LINEAR = 0, 1   # per-panel constants at centroids / vertex hats at vertices (Sec. 3)
STOP_NAMES = {0: "max_steps", 1: "dirichlet", 2: "floating", 3: "interface", 4: "weak_field", 5: "nonfinite"}


class BemError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_lib.STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _check(rc: int, lib):
    if rc != 0:
        raise BemError(rc, lib.bem_last_error().decode())


def _torch():
    import torch
    return torch


def _dev_ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def trace_params(h=1e-4, e_min=1e-3, max_steps=2000, direction=1, alpha_a=1e-3, alpha_e0=25.0, alpha_p=2.0,
                 k_str=float("inf"), start_offset=1e-6) -> _lib.TraceParams:
    return _lib.TraceParams(h, e_min, start_offset, max_steps, direction, alpha_a, alpha_e0, alpha_p, k_str)


class Context:
    """One assembled BEM problem on the current GPU (bem_create / bem_destroy)."""

    def __init__(self, vert, tri, tri_body, body_kind, eps_plus, eps_minus, precision=FP64, eta=6.0, restart=100,
                 constraint_form=0, stream=None, basis=BASIS_CONSTANT):
        torch = _torch()
        self.lib = _lib.load()
        self.device = torch.device("cuda", torch.cuda.current_device())
        self._vert = np.ascontiguousarray(vert, dtype=np.float64)
        self._tri = np.ascontiguousarray(tri, dtype=np.int32)
        self._tb = np.ascontiguousarray(tri_body, dtype=np.int32)
        kinds = np.asarray(body_kind, dtype=np.int32)
        ep = np.asarray(eps_plus, dtype=np.float64)
        em = np.asarray(eps_minus, dtype=np.float64)
        self.n_body = len(kinds)
        bodies = (_lib.Body * self.n_body)(*[_lib.Body(int(k), float(a), float(b)) for k, a, b in zip(kinds, ep, em)])
        opt = _lib.Options(int(precision), float(eta), int(restart), int(constraint_form), int(basis))
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._ctx = ctypes.c_void_p()
        rc = self.lib.bem_create(len(self._vert), self._vert.ctypes.data, len(self._tri), self._tri.ctypes.data,
                                 self._tb.ctypes.data, self.n_body, ctypes.addressof(bodies), ctypes.byref(opt),
                                 ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._ctx))
        _check(rc, self.lib)
        self.N = len(self._tri)
        self.n = int(self.lib.bem_n_unknowns(self._ctx))
        self.precision = int(precision)
        self.basis = int(basis)

    @classmethod
    def from_problem(cls, p, **kw):
        return cls(p.vert, p.tri, p.tri_body, p.body_kind, p.eps_plus, p.eps_minus, **kw)

    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            self.lib.bem_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------------ calls
    def assemble(self):
        _check(self.lib.bem_assemble(self._ctx), self.lib)

    @property
    def near_pairs(self) -> int:
        return int(self.lib.bem_near_pairs(self._ctx))

    def copy_rows(self, row0: int, n_rows: int):
        torch = _torch()
        out = torch.empty((n_rows, self.n), dtype=torch.float64, device=self.device)
        _check(self.lib.bem_copy_rows(self._ctx, row0, n_rows, _dev_ptr(out)), self.lib)
        return out

    def rhs(self, body_V):
        torch = _torch()
        bv = np.ascontiguousarray(np.atleast_2d(body_V), dtype=np.float64)
        out = torch.empty((bv.shape[0], self.n), dtype=torch.float64, device=self.device)
        _check(self.lib.bem_rhs(self._ctx, bv.shape[0], bv.ctypes.data, _dev_ptr(out)), self.lib)
        return out

    def matvec(self, x, transpose=False):
        torch = _torch()
        x2 = x.reshape(-1, self.n).contiguous()
        y = torch.empty_like(x2)
        _check(self.lib.bem_matvec(self._ctx, x2.shape[0], _dev_ptr(x2), _dev_ptr(y), int(bool(transpose))), self.lib)
        return y.reshape(x.shape)

    def matvec_noalloc(self, x, y, transpose=False):
        """bem_matvec_noalloc: y = A x (or A^T x) into the caller's y, with no device allocation."""
        _check(self.lib.bem_matvec_noalloc(self._ctx, x.reshape(-1, self.n).shape[0], _dev_ptr(x), _dev_ptr(y),
                                           int(bool(transpose))), self.lib)
        return y

    def compress(self, eps=1e-8, eta_adm=1.0, leaf=64):
        """bem_compress: the hierarchical-matrix operator in place of the dense one; returns its sizes."""
        info = _lib.CompressInfo()
        _check(self.lib.bem_compress(self._ctx, float(eps), float(eta_adm), int(leaf), ctypes.byref(info)), self.lib)
        return {k: int(getattr(info, k)) for k, _ in _lib.CompressInfo._fields_}

    def pair_integrals(self, pts, panel, rule=0):
        """bem_pair_integrals: S [P] and F [P, 3] (numpy) of unit density on panel[p] at pts[p];
        rule 0 closed forms, 1 the near-singular rule (closest point, subdivision, Duffy)."""
        torch = _torch()
        x = torch.as_tensor(np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3), device=self.device)
        pn = torch.as_tensor(np.ascontiguousarray(panel, dtype=np.int32).reshape(-1), device=self.device)
        P = pn.shape[0]
        S = torch.empty(P, dtype=torch.float64, device=self.device)
        F = torch.empty((P, 3), dtype=torch.float64, device=self.device)
        _check(self.lib.bem_pair_integrals(self._ctx, P, _dev_ptr(x), _dev_ptr(pn), int(rule), _dev_ptr(S),
                                           _dev_ptr(F)), self.lib)
        return S.cpu().numpy(), F.cpu().numpy()

    def quad_pair_integrals(self, pts, nodes, want_F=True):
        """bem_quad_pair_integrals: S [P] and F [P, 3] (numpy; F None when not wanted) of unit
        density on the curved quadratic panel nodes[p] (six nodes: corners, then the edge nodes of
        edges 1-2, 2-3, 3-1) at pts[p], by the near-singular rule of Sec. 4."""
        torch = _torch()
        x = torch.as_tensor(np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3), device=self.device)
        q = torch.as_tensor(np.ascontiguousarray(nodes, dtype=np.float64).reshape(-1, 6, 3), device=self.device)
        P = x.shape[0]
        if q.shape[0] != P:
            raise ValueError("pts and nodes disagree in length")
        S = torch.empty(P, dtype=torch.float64, device=self.device)
        F = torch.empty((P, 3), dtype=torch.float64, device=self.device) if want_F else None
        _check(self.lib.bem_quad_pair_integrals(self._ctx, P, _dev_ptr(x), _dev_ptr(q), _dev_ptr(S),
                                                _dev_ptr(F)), self.lib)
        return S.cpu().numpy(), (F.cpu().numpy() if F is not None else None)

    def solve(self, body_V, tol=1e-10, max_iter=10000, raise_on_noconv=True):
        """Returns (sol [nrhs, n] float64 on the GPU, info dict)."""
        torch = _torch()
        bv = np.ascontiguousarray(np.atleast_2d(body_V), dtype=np.float64)
        sol = torch.empty((bv.shape[0], self.n), dtype=torch.float64, device=self.device)
        info = _lib.SolveInfo()
        rc = self.lib.bem_solve_gmres(self._ctx, bv.shape[0], bv.ctypes.data, float(tol), int(max_iter),
                                      _dev_ptr(sol), ctypes.byref(info))
        if rc != 0 and (rc != _lib.BEM_ERR_NOCONV or raise_on_noconv):
            _check(rc, self.lib)
        return sol, dict(iters=info.iters, rel_residual=info.rel_residual, refinements=info.refinements,
                         converged=(rc == 0))

    def eval_field(self, sol, pts, on_panel=None, want_phi=True):
        torch = _torch()
        sol2 = sol.reshape(-1, self.n).contiguous()
        nrhs = sol2.shape[0]
        pts = torch.as_tensor(pts, dtype=torch.float64, device=self.device).reshape(-1, 3).contiguous()
        P = pts.shape[0]
        op = None
        if on_panel is not None:
            op = torch.as_tensor(on_panel, dtype=torch.int32, device=self.device).contiguous()
        phi = torch.empty((nrhs, P), dtype=torch.float64, device=self.device) if want_phi else None
        E = torch.empty((nrhs, P, 3), dtype=torch.float64, device=self.device)
        _check(self.lib.bem_eval_field(self._ctx, nrhs, _dev_ptr(sol2), P, _dev_ptr(pts), _dev_ptr(op),
                                       _dev_ptr(phi), _dev_ptr(E)), self.lib)
        return phi, E

    def potential(self, sol, pts):
        """phi at points (either basis; E is not computed).  Returns [nrhs, P] on the GPU."""
        torch = _torch()
        sol2 = sol.reshape(-1, self.n).contiguous()
        nrhs = sol2.shape[0]
        pts = torch.as_tensor(pts, dtype=torch.float64, device=self.device).reshape(-1, 3).contiguous()
        P = pts.shape[0]
        phi = torch.empty((nrhs, P), dtype=torch.float64, device=self.device)
        if self.basis == BASIS_CONSTANT:
            E = torch.empty((nrhs, P, 3), dtype=torch.float64, device=self.device)
        else:
            E = None
        _check(self.lib.bem_eval_field(self._ctx, nrhs, _dev_ptr(sol2), P, _dev_ptr(pts), None,
                                       _dev_ptr(phi), _dev_ptr(E)), self.lib)
        return phi

    def _line_args(self, sol, starts, line_rhs):
        torch = _torch()
        sol2 = sol.reshape(-1, self.n).contiguous()
        starts = torch.as_tensor(starts, dtype=torch.float64, device=self.device).reshape(-1, 3).contiguous()
        lr = None
        if line_rhs is not None:
            lr = torch.as_tensor(line_rhs, dtype=torch.int32, device=self.device).contiguous()
        return sol2, starts, lr

    def trace_lines(self, sol, starts, params=None, line_rhs=None, want_path=False):
        torch = _torch()
        params = params or trace_params()
        sol2, starts, lr = self._line_args(sol, starts, line_rhs)
        L = starts.shape[0]
        ns = torch.empty(L, dtype=torch.int32, device=self.device)
        st = torch.empty(L, dtype=torch.int32, device=self.device)
        path = (torch.full((L, params.max_steps + 1, 3), float("nan"), dtype=torch.float64, device=self.device)
                if want_path else None)
        _check(self.lib.bem_trace_lines(self._ctx, sol2.shape[0], _dev_ptr(sol2), L, _dev_ptr(lr), _dev_ptr(starts),
                                        ctypes.byref(params), _dev_ptr(ns), _dev_ptr(st), _dev_ptr(path)), self.lib)
        return ns, st, path

    def streamer_integral(self, sol, starts, params=None, line_rhs=None):
        torch = _torch()
        params = params or trace_params()
        sol2, starts, lr = self._line_args(sol, starts, line_rhs)
        L = starts.shape[0]
        I = torch.empty(L, dtype=torch.float64, device=self.device)
        ns = torch.empty(L, dtype=torch.int32, device=self.device)
        st = torch.empty(L, dtype=torch.int32, device=self.device)
        ex = torch.empty(L, dtype=torch.uint8, device=self.device)
        _check(self.lib.bem_streamer_integral(self._ctx, sol2.shape[0], _dev_ptr(sol2), L, _dev_ptr(lr),
                                              _dev_ptr(starts), ctypes.byref(params), _dev_ptr(I), _dev_ptr(ns),
                                              _dev_ptr(st), _dev_ptr(ex)), self.lib)
        return I, ns, st, ex

    def streamer_grad(self, sol, starts, dJ_dI, params=None, line_rhs=None, start_panel=None, start_bary=None,
                      tol=1e-12, want_dstart=False):
        """Gradient of J = sum_l dJ_dI[l] * I_l (bem_streamer_grad).  Returns
        (dJ_dvert [n_vert, 3], dJ_dV [nrhs, n_body], dJ_dstart [L, 3] or None), float64 on the GPU."""
        torch = _torch()
        params = params or trace_params()
        sol2, starts, lr = self._line_args(sol, starts, line_rhs)
        L = starts.shape[0]
        g = torch.as_tensor(dJ_dI, dtype=torch.float64, device=self.device).reshape(L).contiguous()
        sp = sb = None
        if start_panel is not None:
            sp = torch.as_tensor(start_panel, dtype=torch.int32, device=self.device).reshape(L).contiguous()
            sb = torch.as_tensor(start_bary, dtype=torch.float64, device=self.device).reshape(L, 3).contiguous()
        dvert = torch.empty((len(self._vert), 3), dtype=torch.float64, device=self.device)
        dV = torch.empty((sol2.shape[0], self.n_body), dtype=torch.float64, device=self.device)
        dstart = torch.empty((L, 3), dtype=torch.float64, device=self.device) if want_dstart else None
        _check(self.lib.bem_streamer_grad(self._ctx, sol2.shape[0], _dev_ptr(sol2), L, _dev_ptr(lr), _dev_ptr(starts),
                                          _dev_ptr(sp), _dev_ptr(sb), ctypes.byref(params), _dev_ptr(g),
                                          float(tol), _dev_ptr(dvert), _dev_ptr(dV), _dev_ptr(dstart)), self.lib)
        return dvert, dV, dstart

    def panel_points(self, panel, bary, offset=0.0):
        """Points sum_k bary_k v_k + offset * n on the given panels (bem_panel_points).
        Returns [L, 3] float64 on the GPU."""
        torch = _torch()
        pn = torch.as_tensor(np.asarray(panel), dtype=torch.int32, device=self.device).reshape(-1).contiguous()
        L = pn.shape[0]
        bc = torch.as_tensor(np.asarray(bary), dtype=torch.float64, device=self.device).reshape(L, 3).contiguous()
        out = torch.empty((L, 3), dtype=torch.float64, device=self.device)
        _check(self.lib.bem_panel_points(self._ctx, L, _dev_ptr(pn), _dev_ptr(bc), float(offset), _dev_ptr(out)),
               self.lib)
        return out

    def set_tuning(self, key: str, value: int):
        _check(self.lib.bem_set_tuning(self._ctx, key.encode(), int(value)), self.lib)

    def get_tuning(self, key: str) -> int:
        v = ctypes.c_int64(0)
        _check(self.lib.bem_get_tuning(self._ctx, key.encode(), ctypes.byref(v)), self.lib)
        return int(v.value)

    def autotune(self, cache_path=None) -> bool:
        """Time the tile-shape candidates (or load them from the JSON cache); True if cached."""
        fc = ctypes.c_int32(0)
        path = cache_path.encode() if cache_path is not None else None
        _check(self.lib.bem_autotune(self._ctx, path, ctypes.byref(fc)), self.lib)
        return bool(fc.value)

    # -------------------------------------------------------------- profiling
    def set_profiling(self, mode=1):
        """0 off, 1 every kernel, 2 only the field-line far pass (see bem_set_profiling)."""
        _check(self.lib.bem_set_profiling(self._ctx, int(mode)), self.lib)

    def kernel_stats(self, name: str):
        n = ctypes.c_int64(0)
        ms = ctypes.c_double(0.0)
        _check(self.lib.bem_kernel_stats(self._ctx, name.encode(), ctypes.byref(n), ctypes.byref(ms)), self.lib)
        return int(n.value), float(ms.value)

    def reset_stats(self):
        _check(self.lib.bem_reset_stats(self._ctx), self.lib)

    def counter(self, name: str) -> int:
        v = ctypes.c_int64(0)
        _check(self.lib.bem_get_counter(self._ctx, name.encode(), ctypes.byref(v)), self.lib)
        return int(v.value)


def _streamer_function():
    torch = _torch()

    class StreamerIntegral(torch.autograd.Function):
        """I = streamer integrals of the field lines of the BEM solution for vertex
        positions `vert` (tensor [n_vert, 3]) and body potentials `body_V` (tensor
        [n_body]), lines starting on panels (start_panel, start_bary, params.start_offset).
        Forward: assemble, GMRES, bem_streamer_integral.  Backward: bem_streamer_grad."""

        @staticmethod
        def forward(ctx, vert, body_V, problem, start_panel, start_bary, params, solve_tol, eta, constraint_form):
            v = vert.detach().cpu().numpy()
            bv = body_V.detach().cpu().numpy()
            bctx = Context(v, problem.tri, problem.tri_body, problem.body_kind, problem.eps_plus, problem.eps_minus,
                           precision=FP64, eta=eta, constraint_form=constraint_form)
            bctx.assemble()
            sol, _ = bctx.solve(bv, tol=solve_tol, max_iter=100000)
            starts = bctx.panel_points(start_panel, start_bary, params.start_offset)
            I, ns, st, _ = bctx.streamer_integral(sol, starts, params)
            ctx.bctx, ctx.sol, ctx.starts, ctx.params = bctx, sol, starts, params
            ctx.start_panel, ctx.start_bary = start_panel, start_bary
            ctx.dev_in = vert.device
            return I.to(vert.device)

        @staticmethod
        def backward(ctx, gI):
            bctx = ctx.bctx
            dvert, dV, _ = bctx.streamer_grad(ctx.sol, ctx.starts, gI.detach().to(bctx.device, torch.float64),
                                              ctx.params, start_panel=ctx.start_panel, start_bary=ctx.start_bary)
            bctx.close()
            return dvert.to(ctx.dev_in), dV[0].to(ctx.dev_in), None, None, None, None, None, None, None

    return StreamerIntegral


_SI = None


def streamer_integral(vert, body_V, problem, start_panel, start_bary, params=None, solve_tol=1e-12, eta=6.0,
                      constraint_form=0):
    """Differentiable streamer integrals (torch.autograd): see _streamer_function."""
    global _SI
    if _SI is None:
        _SI = _streamer_function()
    return _SI.apply(vert, body_V, problem, np.asarray(start_panel, dtype=np.int32),
                     np.asarray(start_bary, dtype=np.float64), params or trace_params(), solve_tol, eta,
                     constraint_form)
