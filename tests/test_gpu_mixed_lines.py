"""Field lines in MIXED precision against the FP64 oracle (Sec. 1, Eq. Breakdowncrit).

In a MIXED context the far passes of the field-line tracer evaluate the
7-point rule in FP32 (panel records rounded to FP32, FP32 arithmetic, each
chunk's partial field summed in FP64), while near pairs, the RK4 update and
the integral stay FP64.  Every FP32 instance of the far pass is run: the
split kernels at 2, 4 and 8 waves per chunk, the unsplit ones at 64, 128 and
256 lines per block, and the few-line tail.

Errors are stated per result, on 16 coax lines (seed 21, h = 1e-3, <= 200
steps) that end on the shell or the ring or run out of steps:
- driven by the oracle's FP64 density (so only the FP32 far arithmetic
  differs): stop codes and step counts equal to the oracle's; integrals within
  1e-5 relative; path points within 1e-6 of the path length scale;
- driven by the MIXED solution (sigma within 1e-5 of the oracle's): stop codes
  equal; integrals within 1e-4 relative.  The bar is the 1e-5 bar on |E|
  times the slope of alpha_eff(E) = a (E - 25)^2 in relative terms,
  d(alpha)/alpha = 2 E / (E - 25) dE/E, which is about 10 at the rod surface
  (E = 31 for V0 = 1);
- |E| at the GPU path points from the MIXED field evaluation against the
  oracle's FP64 field: within 1e-5 (the workload's mixed-mode bar).
"""

import sys

import numpy as np
import pytest

import oracle
from workloads import coax_problem, electrode_line_starts

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KW = dict(h=1e-3, max_steps=200)
LAYOUTS = {
    "split2": dict(trace_splitk=2, trace_split=4096, trace_few=0),
    "split4": dict(trace_splitk=4, trace_split=4096, trace_few=0),
    "split8": dict(trace_splitk=8, trace_split=4096, trace_few=0),
    "tile64": dict(trace_tile=64, trace_split=0, trace_few=0),
    "tile128": dict(trace_tile=128, trace_split=0, trace_few=0),
    "tile256": dict(trace_tile=256, trace_split=0, trace_few=0),
    "few16": dict(trace_split=0, trace_few=16),
}


def _say(msg):
    print(f"[gpu-mixed-lines] {msg}", flush=True)
    sys.stdout.flush()


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_12663_amd as bem
    p = coax_problem(0.012)
    o = oracle.Oracle(p)
    A = o.assemble()
    x_ref = np.linalg.solve(A, o.rhs(p.body_V))
    starts, _, _ = electrode_line_starts(p, 16, seed=21)
    nso, sto, Io, patho = o.trace(x_ref, starts, oracle.trace_params(**KW), want_path=True)
    c = bem.Context.from_problem(p, precision=bem.MIXED)
    c.assemble()
    sm, info = c.solve(p.body_V, tol=1e-8)
    assert info["converged"]
    _say(f"coax N={p.n_tri}: mixed sigma error {rel(sm[0].cpu().numpy()[:p.n_tri], x_ref[:p.n_tri]):.2e}")
    yield bem, p, o, c, x_ref, sm, starts, (nso, sto, Io, patho)
    c.close()


@pytest.mark.parametrize("layout", list(LAYOUTS), ids=list(LAYOUTS))
def test_mixed_lines_fp64_density(setup, layout):
    bem, p, o, c, x_ref, sm, starts, (nso, sto, Io, patho) = setup
    for k, v in LAYOUTS[layout].items():
        c.set_tuning(k, v)
    sol = torch.tensor(x_ref, device="cuda")
    I, ns, st, _ = c.streamer_integral(sol, starts, bem.trace_params(**KW))
    ns2, st2, path = c.trace_lines(sol, starts, bem.trace_params(**KW), want_path=True)
    I, ns, st, path = I.cpu().numpy(), ns.cpu().numpy(), st.cpu().numpy(), path.cpu().numpy()
    assert np.array_equal(ns, ns2.cpu().numpy()) and np.array_equal(st, st2.cpu().numpy())
    assert np.array_equal(st, sto) and np.array_equal(ns, nso)
    eI = rel(I, Io)
    scale = max(np.abs(patho[l, :nso[l] + 1]).max() for l in range(len(starts)))
    eP = max(np.abs(path[l, :ns[l] + 1] - patho[l, :ns[l] + 1]).max() for l in range(len(starts))) / scale
    _say(f"{layout}: FP64 density, FP32 far passes: integral error {eI:.2e}, path error {eP:.2e}")
    assert eI <= 1e-5 and eP <= 1e-6
    c.set_tuning("trace_split", 64)
    c.set_tuning("trace_few", 8)


def test_mixed_lines_mixed_density(setup):
    bem, p, o, c, x_ref, sm, starts, (nso, sto, Io, patho) = setup
    I, ns, st, _ = c.streamer_integral(sm, starts, bem.trace_params(**KW))
    ns2, st2, path = c.trace_lines(sm, starts, bem.trace_params(**KW), want_path=True)
    I, ns, st, path = I.cpu().numpy(), ns.cpu().numpy(), st.cpu().numpy(), path.cpu().numpy()
    assert np.array_equal(st, sto)
    same = ns == nso              # a hit may move by a step; integrals are compared where it did not
    assert np.abs(ns - nso).max() <= 1 and same.sum() >= len(ns) - 1
    eI = rel(I[same], Io[same])
    # |E| at the GPU's own path points: MIXED field evaluation against the oracle's FP64 field
    pts = np.concatenate([path[l, :ns[l] + 1:10] for l in range(len(starts))])
    _, E = c.eval_field(sm, pts, want_phi=False)
    _, E_o = o.eval(x_ref, pts)
    eE = rel(np.linalg.norm(E[0].cpu().numpy(), axis=1), np.linalg.norm(E_o, axis=1))
    _say(f"MIXED density: integral error {eI:.2e}, |E| error at {len(pts)} path points {eE:.2e}, "
         f"step counts equal on {int(same.sum())}/{len(ns)} lines")
    assert eI <= 1e-4 and eE <= 1e-5
