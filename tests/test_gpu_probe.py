"""The kernel timing probe behind bench.py's roofline: sampled launches, their duration and their
algorithmic bytes counting only the systems each launch works on.  Needs an MI355X."""
import math

import numpy as np
import pytest

from oracle.apfc_oracle import tri_k
from paper_1902_09761_amd import apfc, inputs
from tests.gpu_util import H_TRI, phi_of, solver_for, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _apply_bytes(NT, nv, c=8, J=3):
    # z (2 halves) and nv basis vectors in the basis precision, w (2 FP64 halves), d shared by J amplitudes
    return NT * (2.0 * c * (1 + nv) + 32.0 + 8.0 / J)


def _probe_one_step(meshes, etas, restart):
    s = solver_for(meshes, apfc.APFC_TRI2D, [0.02] * len(meshes), rtol=1e-10, precision=apfc.APFC_MIXED,
                   inner_kind=apfc.APFC_INNER_CHEB, restart=restart)
    et = [to_dev(e) for e in etas]
    zt = [torch.zeros_like(e) for e in et]
    s.init_zeta(et, zt)
    s.probe_enable("apply", 1)
    info = s.step(et, zt, 1.0)
    torch.cuda.synchronize()
    n, ms, bpl = s.probe_read()
    again = s.probe_read()
    s.probe_enable(None, 1)
    return n, ms, bpl, info, again


def test_probe_counts_only_working_systems():
    """A 64^2 instance alone, then batched with an instance at eta = 0 (b = 0 and x0 = 0: solved before
    the first iteration, so every kernel skips it): the same launches are sampled and each moves the same
    bytes, which lie between the formula's values for 1 basis vector on one of the first instance's three
    systems and `restart` vectors on all of them; a read after the reset reports nothing."""
    m = inputs.Mesh(2, (64, 64, 1), (64 * H_TRI, 64 * H_TRI, 1.0))
    e1 = inputs.single_grain(m, tri_k(), phi_of(tri_k())(0.02), math.radians(6.0), 14 * H_TRI, seed=31)
    restart = 4
    n1, ms1, b1, info1, again = _probe_one_step([m], [e1], restart)
    n2, ms2, b2, info2, _ = _probe_one_step([m, m], [e1, np.zeros_like(e1)], restart)
    assert n1 > 0 and ms1 > 0.0 and ms2 > 0.0
    assert again == (0, 0.0, 0.0)
    assert info2["iters"][:3] == info1["iters"] and info2["iters"][3:] == [0, 0, 0]
    assert n2 == n1
    assert abs(b2 - b1) <= 1e-12 * b1
    NT1 = 3 * m.N
    assert _apply_bytes(NT1, 1) / 3 * (1 - 1e-12) <= b1 <= _apply_bytes(NT1, restart) * (1 + 1e-12)
