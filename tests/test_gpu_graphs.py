"""hipGraph replay of restart cycles (apfc_set_graphs) against eager launches: the same kernels in the
same order, so every step must give the same bits.  Each step replays the captured cycle several
times, with the step's own eager kernels and host synchronisations between the replays.  Needs an
MI355X."""
import math

import numpy as np
import pytest

from oracle.apfc_oracle import bcc_k, tri_k
from paper_1902_09761_amd import apfc, inputs
from tests.gpu_util import H_TRI, from_dev, oracle_for, phi_of, rel_l2, solver_for, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _trajectory(s, eta0, dt, steps):
    et = [to_dev(eta0)]
    zt = [torch.zeros_like(et[0])]
    s.init_zeta(et, zt)
    out = []
    for _ in range(steps):
        info = s.step(et, zt, dt)
        torch.cuda.synchronize()
        out.append((from_dev(et[0]), info["max_iters"]))
    return out


@pytest.mark.parametrize("dim,precision,inner", [(2, apfc.APFC_MIXED, apfc.APFC_INNER_CHEB),
                                                 (2, apfc.APFC_FP64, apfc.APFC_INNER_PCG),
                                                 (3, apfc.APFC_MIXED, apfc.APFC_INNER_CHEB)])
def test_graph_replay_matches_eager(dim, precision, inner):
    if dim == 2:
        mesh = inputs.Mesh(2, (96, 80, 1), (96 * H_TRI, 80 * H_TRI, 1.0))
        k, kind, J = tri_k(), apfc.APFC_TRI2D, 3
        eta0 = inputs.single_grain(mesh, k, phi_of(k)(0.02), math.radians(6.0), 20 * H_TRI, seed=41)
    else:
        h = 60.0 * inputs.BCC_SPACING / 128.0
        mesh = inputs.Mesh(3, (16, 12, 10), (16 * h, 12 * h, 10 * h))
        k, kind, J = bcc_k(), apfc.APFC_BCC3D, 6
        eta0 = inputs.single_grain(mesh, k, phi_of(k)(0.02), math.radians(5.0), 4 * h, seed=42)
    kw = dict(rtol=1e-10, precision=precision, inner_kind=inner, restart=3, x0_order=2)
    if inner == apfc.APFC_INNER_CHEB:
        kw.update(mass_iters=5, diff_iters=3)
    runs = []
    for graphs in (False, True):
        s = solver_for([mesh], kind, [0.02], **kw)
        s.set_graphs(graphs)
        runs.append(_trajectory(s, eta0, 1.0, 5))
    for (e0, i0), (e1, i1) in zip(*runs):
        assert i0 == i1 and i0 > 3          # several replays per step
        assert np.array_equal(e0, e1)
    # and the replayed trajectory is the method's
    o = oracle_for(mesh, k, 0.02)
    ref = eta0
    for _ in range(5):
        _, ref = o.step(ref, 1.0)
    assert rel_l2(runs[1][-1][0], ref) < 1e-7


def test_graph_replay_uneven_batch_matches_eager():
    """Four uneven instances (sizes 48^2..96x80, Delta B 0.012..0.045) in one context: the systems converge
    at different cycles, so the replayed cycles run with per-system masks that differ from replay to
    replay.  Graph replay and eager launches must give the same bits at every step, and the batch must
    match the oracle instance by instance."""
    meshes = [inputs.Mesh(2, (48, 48, 1), (48 * H_TRI, 48 * H_TRI, 1.0)),
              inputs.Mesh(2, (64, 40, 1), (64 * H_TRI, 40 * H_TRI, 1.0)),
              inputs.Mesh(2, (96, 80, 1), (96 * H_TRI, 80 * H_TRI, 1.0)),
              inputs.Mesh(2, (72, 72, 1), (72 * H_TRI, 72 * H_TRI, 1.0))]
    dBs = [0.012, 0.025, 0.045, 0.035]
    etas = [inputs.single_grain(m, tri_k(), phi_of(tri_k())(dB), math.radians(2.0 + 2.5 * i), 0.25 * m.length[0],
                                seed=50 + i) for i, (m, dB) in enumerate(zip(meshes, dBs))]
    kw = dict(rtol=1e-10, precision=apfc.APFC_MIXED, inner_kind=apfc.APFC_INNER_CHEB, mass_iters=5, diff_iters=3,
              restart=3, x0_order=2)
    runs = []
    for graphs in (False, True):
        s = solver_for(meshes, apfc.APFC_TRI2D, dBs, **kw)
        s.set_graphs(graphs)
        et = [to_dev(e) for e in etas]
        zt = [torch.zeros_like(e) for e in et]
        s.init_zeta(et, zt)
        traj = []
        for _ in range(4):
            info = s.step(et, zt, 1.0)
            torch.cuda.synchronize()
            traj.append(([from_dev(e) for e in et], info["iters"]))
        runs.append(traj)
    uneven = False
    for (ea, ia), (eb, ib) in zip(*runs):
        assert ia == ib
        per_inst = [max(ia[3 * b:3 * b + 3]) for b in range(4)]
        uneven |= len(set(per_inst)) > 1
        for x, y in zip(ea, eb):
            assert np.array_equal(x, y)
    assert uneven                       # the instances did stop at different iterations
    for b, (m, dB) in enumerate(zip(meshes, dBs)):
        o = oracle_for(m, tri_k(), dB)
        ref = etas[b]
        for _ in range(4):
            _, ref = o.step(ref, 1.0)
        assert rel_l2(runs[1][-1][0][b], ref) < 1e-7
