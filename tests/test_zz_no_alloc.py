"""apfc_step_noalloc (the step on the library's static device scratch, for callers that cannot allocate)
against apfc_step on the same inputs, through the C ABI.  Both run the same kernels in the same order with
fixed-order reductions, so the results must agree bit for bit.  Needs an MI355X."""
import math

import numpy as np
import pytest

from oracle.apfc_oracle import tri_k
from paper_1902_09761_amd import apfc, inputs
from tests.gpu_util import H_TRI, from_dev, phi_of, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

KW = dict(rtol=1e-10, precision=apfc.APFC_MIXED, inner_kind=apfc.APFC_INNER_CHEB, mass_iters=5, diff_iters=3,
          restart=4, x0_order=3)


def _solver(mesh, dB, attach):
    lat = apfc.apfc_lattice_default(apfc.APFC_TRI2D)
    p = apfc.apfc_params_default(a1=0.5 * dB, **KW)
    return apfc.Solver([apfc.make_mesh(2, mesh.n, mesh.length)], lat, [p], attach_workspace=attach)


def _state(mesh, dB, seed, theta):
    return inputs.single_grain(mesh, tri_k(), phi_of(tri_k())(dB), math.radians(theta), 0.25 * mesh.length[0],
                               seed=seed)


def _pair(eta0):
    et = to_dev(eta0)
    return et, torch.zeros_like(et)


def _steps(fn, et, zt, n):
    out = []
    for _ in range(n):
        info = fn([et], [zt], 1.0)
        torch.cuda.synchronize()
        out.append((from_dev(et), from_dev(zt), info["iters"]))
    return out


def _same(a, b):
    for (ea, za, ia), (eb, zb, ib) in zip(a, b):
        assert ia == ib
        assert np.array_equal(ea, eb) and np.array_equal(za, zb)


def test_noalloc_step_matches_step():
    print("no-alloc: scratch bytes", apfc.apfc_noalloc_max_bytes(), flush=True)
    mA = inputs.Mesh(2, (96, 80, 1), (96 * H_TRI, 80 * H_TRI, 1.0))
    mB = inputs.Mesh(2, (48, 40, 1), (48 * H_TRI, 40 * H_TRI, 1.0))
    eA, eB = _state(mA, 0.02, 61, 6.0), _state(mB, 0.03, 62, 4.0)

    # first call sequence: a context without any workspace, three consecutive steps (the extrapolation
    # history stays in the scratch between them)
    na, ra = _solver(mA, 0.02, False), _solver(mA, 0.02, True)
    assert na.workspace is None and na.workspace_bytes <= apfc.apfc_noalloc_max_bytes()
    print("no-alloc: 96x80, 3 steps", flush=True)
    et, zt = _pair(eA)
    ra.init_zeta([et], [zt])                    # zeta^0 from the regular context (init_zeta needs a workspace)
    et2, zt2 = et.clone(), zt.clone()
    got = _steps(na.step_noalloc, et, zt, 3)
    ref = _steps(ra.step, et2, zt2, 3)
    _same(got, ref)

    # second call sequence with a smaller input: another context lays its tables out in the same scratch
    print("no-alloc: 48x40, 2 steps", flush=True)
    nb, rb = _solver(mB, 0.03, False), _solver(mB, 0.03, True)
    et, zt = _pair(eB)
    rb.init_zeta([et], [zt])
    et2, zt2 = et.clone(), zt.clone()
    _same(_steps(nb.step_noalloc, et, zt, 2), _steps(rb.step, et2, zt2, 2))

    # the first context again: its tables are laid out anew and its history restarts
    print("no-alloc: 96x80 again after the other context", flush=True)
    et = to_dev(got[-1][0])
    zt = to_dev(got[-1][1])
    et2, zt2 = et.clone(), zt.clone()
    ra.reset_history()
    _same(_steps(na.step_noalloc, et, zt, 1), _steps(ra.step, et2, zt2, 1))


def test_noalloc_and_workspace_calls_interleave():
    """A context with a workspace alternates apfc_step_noalloc and apfc_step: each switch restarts the
    extrapolation history, and every step equals a regular context's step after a history reset."""
    m = inputs.Mesh(2, (64, 64, 1), (64 * H_TRI, 64 * H_TRI, 1.0))
    e0 = _state(m, 0.025, 63, 5.0)
    s, r = _solver(m, 0.025, True), _solver(m, 0.025, True)
    et, zt = _pair(e0)
    s.init_zeta([et], [zt])
    et2, zt2 = et.clone(), zt.clone()
    for k, fn in enumerate([s.step_noalloc, s.step, s.step_noalloc, s.step_noalloc, s.step]):
        print("interleave step", k, flush=True)
        if k in (0, 1, 2, 4):                  # the switches onto and off the scratch
            r.reset_history()
        _same(_steps(fn, et, zt, 1), _steps(r.step, et2, zt2, 1))


def test_noalloc_rejects_a_context_too_large():
    n = 1024
    big = inputs.Mesh(2, (n, n, 1), (n * H_TRI, n * H_TRI, 1.0))
    s = _solver(big, 0.02, False)
    assert s.workspace_bytes > apfc.apfc_noalloc_max_bytes()
    et = torch.zeros((3, 2, n * n), dtype=torch.float64, device="cuda")
    zt = torch.zeros_like(et)
    with pytest.raises(apfc.APFCError) as ei:
        s.step_noalloc([et], [zt], 1.0)
    assert ei.value.status == apfc.APFC_ERR_WORKSPACE
    assert float(et.abs().max()) == 0.0
