"""apfc_run (several steps in one call) against apfc_step calls and the oracle.  Needs an MI355X."""
import math

import numpy as np
import pytest

from oracle.apfc_oracle import tri_k
from paper_1902_09761_amd import apfc, inputs
from tests.gpu_util import H_TRI, from_dev, oracle_for, phi_of, rel_l2, solver_for, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _case():
    m1 = inputs.Mesh(2, (48, 40, 1), (48 * H_TRI, 40 * H_TRI, 1.0))
    m2 = inputs.Mesh(2, (64, 64, 1), (64 * H_TRI, 64 * H_TRI, 1.0))
    e1 = inputs.single_grain(m1, tri_k(), phi_of(tri_k())(0.02), math.radians(6.0), 10 * H_TRI, seed=21)
    e2 = inputs.single_grain(m2, tri_k(), phi_of(tri_k())(0.035), math.radians(3.0), 14 * H_TRI, seed=22)
    return [m1, m2], [0.02, 0.035], [e1, e2]


@pytest.mark.parametrize("x0_order,precision", [(0, apfc.APFC_FP64), (3, apfc.APFC_FP64), (3, apfc.APFC_MIXED)])
def test_run_equals_repeated_steps_and_oracle(x0_order, precision):
    """6 steps in one apfc_run call give the same bits as 6 apfc_step calls on a fresh context, and
    match the oracle's direct solves."""
    meshes, dBs, etas = _case()
    kw = dict(rtol=1e-12, precision=precision, inner_kind=apfc.APFC_INNER_CHEB, mass_iters=5, diff_iters=3,
              restart=4, x0_order=x0_order)
    steps, dt = 6, 1.0
    outs = []
    for use_run in (False, True):
        s = solver_for(meshes, apfc.APFC_TRI2D, dBs, **kw)
        et = [to_dev(e) for e in etas]
        zt = [torch.zeros_like(e) for e in et]
        s.init_zeta(et, zt)
        if use_run:
            info = s.run(et, zt, dt, steps)
            assert len(info["step_max_iters"]) == steps and min(info["step_max_iters"]) > 0
            assert info["max_relres"] <= 1e-12
            assert info["total_iters"] == sum(info["iters"])
        else:
            per = [s.step(et, zt, dt) for _ in range(steps)]
        torch.cuda.synchronize()
        outs.append(([from_dev(e) for e in et], [from_dev(z) for z in zt]))
    if use_run:
        assert info["step_max_iters"] == [p["max_iters"] for p in per]
        assert info["total_iters"] == sum(p["total_iters"] for p in per)
    for b in range(2):
        assert np.array_equal(outs[0][0][b], outs[1][0][b])
        assert np.array_equal(outs[0][1][b], outs[1][1][b])
    for b, (m, dB, e) in enumerate(zip(meshes, dBs, etas)):
        o = oracle_for(m, tri_k(), dB)
        for _ in range(steps):
            _, e = o.step(e, dt)
        assert rel_l2(outs[1][0][b], e) < 1e-9


def test_run_failure_leaves_state_unchanged():
    """max_iters too small: NOT_CONVERGED from the first step, the caller's arrays untouched."""
    meshes, dBs, etas = _case()
    s = solver_for(meshes, apfc.APFC_TRI2D, dBs, rtol=1e-12, max_iters=2, restart=2)
    et = [to_dev(e) for e in etas]
    zt = [torch.zeros_like(e) for e in et]
    s.init_zeta(et, zt)
    before = [e.clone() for e in et], [z.clone() for z in zt]
    with pytest.raises(apfc.APFCNotConverged):
        s.run(et, zt, 1.0, 3)
    torch.cuda.synchronize()
    for a, b in zip(et + zt, before[0] + before[1]):
        assert torch.equal(a, b)
