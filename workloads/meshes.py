"""Synthetic surface meshes for the electrostatic BEM problems.

Every mesher returns a :class:`Problem`: vertices, triangles (counter-clockwise
about the normal that points into the eps+ side of the surface), a body tag per
triangle and a body table.  Body kinds follow the paper's Section 2 split of a
device into conductors on a prescribed potential, floating conductors and
insulators (dielectric interfaces):

    DIRICHLET = 0   conductor held at a prescribed potential
    FLOATING  = 1   conductor of unknown potential and zero net charge
    INTERFACE = 2   dielectric interface (no free surface charge)
    SHEET     = 3   thin floating conductive sheet, one (open) surface, zero net
                    charge counted over both of its sides (Eq. sheets)

The meshes are the stand-ins for the paper's industrial geometries, which are
not public: an icosphere (sphere closed forms), a conductor coated with a
dielectric shell, a conductor inside a thick floating shell, and a coaxial
rod-in-shell device with a floating torus and a dielectric spacer disc.
Units of the coax are metres.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np

DIRICHLET = 0
FLOATING = 1
INTERFACE = 2
SHEET = 3


@dataclasses.dataclass
class Problem:
    name: str
    vert: np.ndarray          # float64 [Nv, 3]
    tri: np.ndarray           # int32 [N, 3], CCW about the eps+ normal
    tri_body: np.ndarray      # int32 [N]
    body_kind: np.ndarray     # int32 [n_body]
    eps_plus: np.ndarray      # float64 [n_body]
    eps_minus: np.ndarray     # float64 [n_body]
    body_V: np.ndarray        # float64 [n_body]; prescribed potential (DIRICHLET only)
    body_names: list
    # triangles on which field lines may start (electrode panels that touch air)
    start_mask: np.ndarray | None = None

    @property
    def n_tri(self) -> int:
        return int(self.tri.shape[0])

    @property
    def n_vert(self) -> int:
        return int(self.vert.shape[0])

    @property
    def n_body(self) -> int:
        return int(self.body_kind.shape[0])

    @property
    def n_float(self) -> int:
        return int(np.count_nonzero((self.body_kind == FLOATING) | (self.body_kind == SHEET)))

    @property
    def n_unknowns(self) -> int:
        return self.n_tri + self.n_float

    def transformed(self, scale=1.0, rotation=None, shift=None) -> "Problem":
        """Copy with vertices mapped by x -> scale * R x + shift."""
        v = self.vert.copy()
        if rotation is not None:
            v = v @ np.asarray(rotation, dtype=np.float64).T
        v = v * float(scale)
        if shift is not None:
            v = v + np.asarray(shift, dtype=np.float64)
        return dataclasses.replace(self, vert=np.ascontiguousarray(v))


# ---------------------------------------------------------------------------
# small helpers (pure mesh bookkeeping)
# ---------------------------------------------------------------------------

class _Builder:
    """Accumulates vertices and triangles of several bodies."""

    def __init__(self):
        self.v = []
        self.t = []
        self.b = []

    def add_vertices(self, pts) -> np.ndarray:
        pts = np.asarray(pts, dtype=np.float64).reshape(-1, 3)
        base = sum(len(x) for x in self.v)
        self.v.append(pts)
        return np.arange(base, base + len(pts), dtype=np.int64)

    def add_triangles(self, tris, body: int):
        tris = np.asarray(tris, dtype=np.int64).reshape(-1, 3)
        self.t.append(tris)
        self.b.append(np.full(len(tris), body, dtype=np.int32))

    def finish(self):
        vert = np.ascontiguousarray(np.concatenate(self.v), dtype=np.float64)
        tri = np.ascontiguousarray(np.concatenate(self.t), dtype=np.int32)
        body = np.ascontiguousarray(np.concatenate(self.b), dtype=np.int32)
        return vert, tri, body


def _orient(vert, tris, want):
    """Flip triangles so that their right-hand normal points along want(centroid)."""
    tris = np.asarray(tris, dtype=np.int64).reshape(-1, 3).copy()
    a, b, c = vert[tris[:, 0]], vert[tris[:, 1]], vert[tris[:, 2]]
    nrm = np.cross(b - a, c - a)
    d = want((a + b + c) / 3.0)
    flip = np.einsum("ij,ij->i", nrm, d) < 0
    tris[flip] = tris[flip][:, [0, 2, 1]]
    return tris


def _zip_loops(ia, ta, ib, tb):
    """Triangulate the band between two closed loops of vertices.

    ia/ib are vertex indices, ta/tb their angles in [0, 2pi), both increasing.
    The loops may hold different numbers of points; the band is closed.
    """
    na, nb = len(ia), len(ib)
    ta = np.concatenate([ta, [ta[0] + 2 * math.pi]])
    tb = np.concatenate([tb, [tb[0] + 2 * math.pi]])
    tris = []
    i = j = 0
    while i < na or j < nb:
        adv_a = j >= nb or (i < na and ta[i + 1] <= tb[j + 1])
        if adv_a:
            tris.append((ia[i % na], ia[(i + 1) % na], ib[j % nb]))
            i += 1
        else:
            tris.append((ia[i % na], ib[(j + 1) % nb], ib[j % nb]))
            j += 1
    return tris


def _circle(b: _Builder, radius, z, n, phase=0.0):
    th = (np.arange(n) + phase) * (2 * math.pi / n)
    pts = np.stack([radius * np.cos(th), radius * np.sin(th), np.full(n, z)], axis=1)
    return b.add_vertices(pts), th


def _n_around(radius, h, minimum=8):
    return max(minimum, int(round(2 * math.pi * radius / h)))


def _levels(z0, z1, h, must=()):
    """Monotone z levels from z0 to z1 with spacing ~h, containing every value in must."""
    cuts = sorted({z0, z1, *[m for m in must if z0 < m < z1]})
    out = [cuts[0]]
    for a, c in zip(cuts[:-1], cuts[1:]):
        k = max(1, int(math.ceil((c - a) / h - 1e-9)))
        out.extend(a + (c - a) * (np.arange(1, k + 1) / k))
    return np.array(out)


# ---------------------------------------------------------------------------
# icosphere
# ---------------------------------------------------------------------------

def icosphere(level: int, radius: float = 1.0):
    """Icosahedron with `level` rounds of 4-way midpoint subdivision, re-projected.

    Level 3 gives 1280 triangles and 642 vertices.  Triangles are CCW seen from
    outside (normal pointing away from the centre).
    """
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, p, 0), (1, p, 0), (-1, -p, 0), (1, -p, 0),
         (0, -1, p), (0, 1, p), (0, -1, -p), (0, 1, -p),
         (p, 0, -1), (p, 0, 1), (-p, 0, -1), (-p, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(x, dtype=np.float64) / np.linalg.norm(x) for x in v]
    faces = list(f)
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    vert = np.array(verts) * radius
    tri = _orient(vert, faces, lambda c: c)
    return np.ascontiguousarray(vert), np.ascontiguousarray(tri, dtype=np.int32)


def sphere_problem(level: int = 3, radius: float = 1.0, V0: float = 1.0) -> Problem:
    """Conductor sphere at V0 in free space (eps_r = 1)."""
    vert, tri = icosphere(level, radius)
    n = tri.shape[0]
    return Problem(
        name=f"sphere_L{level}", vert=vert, tri=tri,
        tri_body=np.zeros(n, dtype=np.int32),
        body_kind=np.array([DIRICHLET], dtype=np.int32),
        eps_plus=np.array([1.0]), eps_minus=np.array([1.0]),
        body_V=np.array([V0], dtype=np.float64), body_names=["sphere"],
        start_mask=np.ones(n, dtype=bool))


def _concentric(level, radii_kinds):
    b = _Builder()
    for bid, (r, outward) in enumerate(radii_kinds):
        v, t = icosphere(level, r)
        idx = b.add_vertices(v)
        tt = idx[t]
        if not outward:
            tt = tt[:, [0, 2, 1]]
        b.add_triangles(tt, bid)
    return b.finish()


def coated_sphere_problem(level=3, a=1.0, b=1.5, eps_r=4.0, V0=1.0) -> Problem:
    """Conductor sphere (radius a, V0) coated by a dielectric shell up to radius b.

    The dielectric surface r = b has its normal pointing outward into vacuum
    (eps+ = 1, eps- = eps_r).
    """
    vert, tri, body = _concentric(level, [(a, True), (b, True)])
    return Problem(
        name=f"coated_sphere_L{level}", vert=vert, tri=tri, tri_body=body,
        body_kind=np.array([DIRICHLET, INTERFACE], dtype=np.int32),
        eps_plus=np.array([eps_r, 1.0]), eps_minus=np.array([1.0, eps_r]),
        body_V=np.array([V0, 0.0]), body_names=["conductor", "coating"],
        start_mask=body == 0)


def floating_shell_problem(level=3, a=1.0, b1=1.5, b2=2.0, V0=1.0) -> Problem:
    """Conductor sphere (radius a, V0) inside a thick floating conducting shell b1..b2.

    The floating body's normals point out of the metal: inward on r = b1,
    outward on r = b2.
    """
    vert, tri, body = _concentric(level, [(a, True), (b1, False), (b2, True)])
    body = np.where(body == 2, 1, body).astype(np.int32)
    return Problem(
        name=f"floating_shell_L{level}", vert=vert, tri=tri, tri_body=body,
        body_kind=np.array([DIRICHLET, FLOATING], dtype=np.int32),
        eps_plus=np.array([1.0, 1.0]), eps_minus=np.array([1.0, 1.0]),
        body_V=np.array([V0, 0.0]), body_names=["conductor", "floating_shell"],
        start_mask=body == 0)


def sphere_sheet_problem(level=3, a=1.0, b=2.0, eps_in=4.0, eps_out=1.0, V0=1.0) -> Problem:
    """Conductor sphere (radius a, V0) inside a thin floating spherical sheet at r = b.

    Dielectric eps_in fills a < r < b and eps_out the outside; the sheet is the only
    surface between them, so it is a SHEET body with eps+ = eps_out (its normal points
    outward) and eps- = eps_in.
    """
    vert, tri, body = _concentric(level, [(a, True), (b, True)])
    return Problem(
        name=f"sphere_sheet_L{level}", vert=vert, tri=tri, tri_body=body,
        body_kind=np.array([DIRICHLET, SHEET], dtype=np.int32),
        eps_plus=np.array([eps_in, eps_out]), eps_minus=np.array([1.0, eps_in]),
        body_V=np.array([V0, 0.0]), body_names=["conductor", "sheet"],
        start_mask=body == 0)


def union_problem(p: Problem, q: Problem, offset=(0.0, 0.0, 0.0)) -> Problem:
    """Both devices in one problem: q translated by offset, its bodies numbered after p's."""
    sm_p = p.start_mask if p.start_mask is not None else np.zeros(p.n_tri, dtype=bool)
    sm_q = q.start_mask if q.start_mask is not None else np.zeros(q.n_tri, dtype=bool)
    return Problem(
        name=f"{p.name}+{q.name}",
        vert=np.concatenate([p.vert, q.vert + np.asarray(offset, dtype=np.float64)]),
        tri=np.concatenate([p.tri, q.tri + p.n_vert]).astype(np.int32),
        tri_body=np.concatenate([p.tri_body, q.tri_body + p.n_body]).astype(np.int32),
        body_kind=np.concatenate([p.body_kind, q.body_kind]).astype(np.int32),
        eps_plus=np.concatenate([p.eps_plus, q.eps_plus]),
        eps_minus=np.concatenate([p.eps_minus, q.eps_minus]),
        body_V=np.concatenate([p.body_V, q.body_V]),
        body_names=list(p.body_names) + list(q.body_names),
        start_mask=np.concatenate([sm_p, sm_q]))


def _open_cylinder(b: _Builder, body, r, zlo, zhi, h):
    """Side surface only (no caps), normals pointing outward (+rho)."""
    n = _n_around(r, h)
    zs = _levels(zlo, zhi, h)
    loops = [_circle(b, r, z, n, phase=0.5 * (k % 2)) for k, z in enumerate(zs)]
    tris = []
    for (ia, ta), (ib, tb) in zip(loops[:-1], loops[1:]):
        tris += _zip_loops(ia, ta, ib, tb)
    vert = np.concatenate(b.v)

    def want(cen):
        d = np.zeros_like(cen)
        d[:, 0] = cen[:, 0]
        d[:, 1] = cen[:, 1]
        return d

    b.add_triangles(_orient(vert, tris, want), body)


BUSHING = dict(
    rod_r=0.02, rod_z=0.30,           # driven closed cylinder, z in [-0.30, 0.30]
    foil_r=(0.035, 0.050, 0.065, 0.080, 0.095),   # five coaxial foils, outermost grounded
    foil_z=(0.26, 0.22, 0.18, 0.14, 0.10),         # half lengths: shorter outward (field grading)
    ins_r=0.11, ins_z=0.32, ins_eps=4.0,           # insulator: closed cylinder around rod and foils
)


def bushing_problem(h: float, V0: float = 1.0) -> Problem:
    """Bushing-like device: a conductor on V0 wrapped by an insulator (eps_r 4) in which five
    thin coaxial conducting foils grade the field; the outermost foil is grounded and the
    other four float (SHEET bodies, eps+ = eps- = eps_r).  The insulator surface is a
    dielectric interface (normals outward into air).  Potential zero at infinity.

    Bodies (index: kind): 0 rod DIRICHLET (V0), 1-4 foils SHEET, 5 outer foil DIRICHLET (0),
    6 insulator INTERFACE.  Element size h (metres) on every surface.
    """
    g = BUSHING
    b = _Builder()
    _capped_cylinder(b, 0, g["rod_r"], -g["rod_z"], g["rod_z"], h, h, (), True)
    for k, (r, z) in enumerate(zip(g["foil_r"], g["foil_z"])):
        _open_cylinder(b, 1 + k, r, -z, z, h)
    _capped_cylinder(b, 6, g["ins_r"], -g["ins_z"], g["ins_z"], 1.5 * h, 1.5 * h, (), True)
    vert, tri, body = b.finish()
    e = g["ins_eps"]
    return Problem(
        name=f"bushing_h{h:g}", vert=vert, tri=tri, tri_body=body,
        body_kind=np.array([DIRICHLET, SHEET, SHEET, SHEET, SHEET, DIRICHLET, INTERFACE], dtype=np.int32),
        eps_plus=np.array([e, e, e, e, e, e, 1.0]), eps_minus=np.array([1.0, e, e, e, e, 1.0, e]),
        body_V=np.array([V0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0]),
        body_names=["rod", "foil1", "foil2", "foil3", "foil4", "foil5_grounded", "insulator"],
        start_mask=body == 0)


# ---------------------------------------------------------------------------
# coaxial rod-in-shell device
# ---------------------------------------------------------------------------

COAX = dict(
    shell_r=0.1, shell_z=0.25,        # grounded closed cylinder, z in [-0.25, 0.25]
    rod_r=0.02, rod_z=0.15,           # driven closed cylinder, z in [-0.15, 0.15]
    ring_R=0.05, ring_r=0.005, ring_z=0.08,   # floating torus
    disc_z=0.01, disc_eps=4.0,        # spacer annulus 0.02 <= rho <= 0.1, |z| <= 0.01
)


def _capped_cylinder(b: _Builder, body, r, zlo, zhi, h_side, h_cap, must, outward):
    n = _n_around(r, h_side)
    zs = _levels(zlo, zhi, h_side, must)
    loops = [_circle(b, r, z, n, phase=0.5 * (k % 2)) for k, z in enumerate(zs)]
    tris = []
    for (ia, ta), (ib, tb) in zip(loops[:-1], loops[1:]):
        tris += _zip_loops(ia, ta, ib, tb)
    # caps: concentric rings down to a centre point
    for (rim, zc) in ((loops[0], zlo), (loops[-1], zhi)):
        k = max(1, int(round(r / h_cap)))
        prev = rim
        for q in range(k - 1, 0, -1):
            rq = r * q / k
            cur = _circle(b, rq, zc, _n_around(rq, h_cap, minimum=6), phase=0.5 * (q % 2))
            tris += _zip_loops(prev[0], prev[1], cur[0], cur[1])
            prev = cur
        c = b.add_vertices([[0.0, 0.0, zc]])[0]
        ia, ta = prev
        for i in range(len(ia)):
            tris.append((ia[i], ia[(i + 1) % len(ia)], c))
    vert = np.concatenate(b.v)

    def want(cen):
        d = np.zeros_like(cen)
        side = (np.abs(cen[:, 2] - zlo) > 1e-9) & (np.abs(cen[:, 2] - zhi) > 1e-9)
        d[side, 0] = cen[side, 0]
        d[side, 1] = cen[side, 1]
        d[~side, 2] = np.sign(cen[~side, 2] - 0.5 * (zlo + zhi))
        return d if outward else -d

    b.add_triangles(_orient(vert, tris, want), body)
    return n


def _torus(b: _Builder, body, R, r, zc, h):
    nu = _n_around(R, h)
    nv = _n_around(r, h, minimum=8)
    u = np.arange(nu) * 2 * math.pi / nu
    v = np.arange(nv) * 2 * math.pi / nv
    U, V = np.meshgrid(u, v, indexing="ij")
    pts = np.stack([(R + r * np.cos(V)) * np.cos(U), (R + r * np.cos(V)) * np.sin(U),
                    zc + r * np.sin(V)], axis=-1).reshape(-1, 3)
    idx = b.add_vertices(pts).reshape(nu, nv)
    tris = []
    for i in range(nu):
        for j in range(nv):
            a, bb = idx[i, j], idx[(i + 1) % nu, j]
            c, d = idx[(i + 1) % nu, (j + 1) % nv], idx[i, (j + 1) % nv]
            tris += [(a, bb, c), (a, c, d)]
    vert = np.concatenate(b.v)

    def want(cen):
        rho = np.hypot(cen[:, 0], cen[:, 1])
        core = np.stack([R * cen[:, 0] / rho, R * cen[:, 1] / rho, np.full(len(cen), zc)], 1)
        return cen - core

    b.add_triangles(_orient(vert, tris, want), body)


def _annulus(b: _Builder, body, r0, r1, z, n0, n1, h0, h1, normal_sign):
    # radial rings with spacing graded linearly from h0 (inner) to h1 (outer)
    radii = [r0]
    while radii[-1] < r1 - 1e-12:
        t = (radii[-1] - r0) / (r1 - r0)
        radii.append(radii[-1] + h0 + (h1 - h0) * t)
    k = max(1, len(radii) - 1)
    radii = np.linspace(r0, r1, k + 1)
    loops = []
    for q, rq in enumerate(radii):
        if q == 0:
            n = n0
        elif q == k:
            n = n1
        else:
            hq = h0 + (h1 - h0) * (rq - r0) / (r1 - r0)
            n = _n_around(rq, hq)
        loops.append(_circle(b, rq, z, n, phase=0.5 * (q % 2)))
    tris = []
    for (ia, ta), (ib, tb) in zip(loops[:-1], loops[1:]):
        tris += _zip_loops(ia, ta, ib, tb)
    vert = np.concatenate(b.v)
    up = np.array([0.0, 0.0, float(normal_sign)])
    b.add_triangles(_orient(vert, tris, lambda c: np.broadcast_to(up, c.shape)), body)


def coax_problem(h: float, V0: float = 1.0) -> Problem:
    """Coaxial rod-in-shell device with floating torus and dielectric spacer disc.

    Bodies (index: kind):
      0 shell: grounded closed cylinder r=0.1, z in [-0.25, 0.25]; normals point
        into the gap (eps+ = 1).
      1 rod: closed cylinder r=0.02, z in [-0.15, 0.15] at V0; outward normals.
      2 ring: floating torus, major radius 0.05, minor 0.005, centred on the
        axis at z = 0.08; outward normals, eps+ = 1.
      3 disc: eps_r = 4 annulus 0.02 <= rho <= 0.1, |z| <= 0.01.  Only its two
        flat faces are interface panels; they point into air (eps+ = 1,
        eps- = 4).  Its cylindrical faces coincide with the conductors.
    `h` is the rod's target edge length; the ring uses 0.85 h, the shell 2.6 h
    and the disc is graded from h (inner rim) to 2.6 h (outer rim).
    """
    g = COAX
    b = _Builder()
    h_shell = 2.6 * h
    dz = g["disc_z"]
    n_shell = _capped_cylinder(b, 0, g["shell_r"], -g["shell_z"], g["shell_z"], h_shell,
                               h_shell, (-dz, dz), outward=False)
    n_rod = _capped_cylinder(b, 1, g["rod_r"], -g["rod_z"], g["rod_z"], h, h,
                             (-dz, dz), outward=True)
    _torus(b, 2, g["ring_R"], g["ring_r"], g["ring_z"], 0.85 * h)
    for zz, sgn in ((dz, +1), (-dz, -1)):
        _annulus(b, 3, g["rod_r"], g["shell_r"], zz, n_rod, n_shell, h, h_shell, sgn)
    vert, tri, body = b.finish()
    cen = vert[tri].mean(axis=1)
    rho = np.hypot(cen[:, 0], cen[:, 1])
    # rod panels that touch air: all but the side panels inside the spacer disc
    in_disc = (np.abs(cen[:, 2]) < dz) & (rho > 0.5 * g["rod_r"])
    start_mask = (body == 1) & ~in_disc
    return Problem(
        name=f"coax_h{h:.5f}", vert=vert, tri=tri, tri_body=body,
        body_kind=np.array([DIRICHLET, DIRICHLET, FLOATING, INTERFACE], dtype=np.int32),
        eps_plus=np.array([1.0, 1.0, 1.0, 1.0]),
        eps_minus=np.array([1.0, 1.0, 1.0, g["disc_eps"]]),
        body_V=np.array([0.0, V0, 0.0, 0.0]),
        body_names=["shell", "rod", "ring", "disc"], start_mask=start_mask)


def coax_conductors_problem(h: float, V0: float = 1.0) -> Problem:
    """The coaxial device without its spacer disc: grounded shell (body 0), rod at V0
    (body 1) and floating torus (body 2), all in air, with the element sizes of
    coax_problem.  Conductors only, so it also suits the nodal basis (every vertex on
    one body)."""
    g = COAX
    b = _Builder()
    h_shell = 2.6 * h
    _capped_cylinder(b, 0, g["shell_r"], -g["shell_z"], g["shell_z"], h_shell, h_shell, (), outward=False)
    _capped_cylinder(b, 1, g["rod_r"], -g["rod_z"], g["rod_z"], h, h, (), outward=True)
    _torus(b, 2, g["ring_R"], g["ring_r"], g["ring_z"], 0.85 * h)
    vert, tri, body = b.finish()
    return Problem(
        name=f"coax_conductors_h{h:.5f}", vert=vert, tri=tri, tri_body=body,
        body_kind=np.array([DIRICHLET, DIRICHLET, FLOATING], dtype=np.int32),
        eps_plus=np.ones(3), eps_minus=np.ones(3), body_V=np.array([0.0, V0, 0.0]),
        body_names=["shell", "rod", "ring"], start_mask=body == 1)


def coax_conductors_for_vertices(n_target: int, V0: float = 1.0, tol: float = 0.02) -> Problem:
    """coax_conductors_problem whose vertex count lies within n_target*(1 +- tol)
    (bisection on log h; deterministic)."""
    lo, hi = 1e-4, 2e-2
    best = None
    for _ in range(60):
        h = math.sqrt(lo * hi)
        p = coax_conductors_problem(h, V0)
        if best is None or abs(p.n_vert - n_target) < abs(best.n_vert - n_target):
            best = p
        if abs(p.n_vert - n_target) <= tol * n_target:
            return p
        if p.n_vert > n_target:
            lo = h
        else:
            hi = h
    return best


def coax_problem_for_size(n_target: int, V0: float = 1.0, tol: float = 0.05) -> Problem:
    """Coax mesh whose panel count lies within n_target*(1 +- tol).

    The rod edge length h is found by bisection on log h; the result is
    deterministic.
    """
    lo, hi = 1e-4, 2e-2
    best = None
    for _ in range(60):
        h = math.sqrt(lo * hi)
        p = coax_problem(h, V0)
        n = p.n_tri
        if best is None or abs(n - n_target) < abs(best.n_tri - n_target):
            best = p
        if abs(n - n_target) <= tol * n_target:
            return p
        if n > n_target:
            lo = h
        else:
            hi = h
    return best
