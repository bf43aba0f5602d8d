"""The multigrid inner solve (APFC_INNER_MG: one geometric V-cycle per diffusion solve of the block
preconditioner, the paper's multigrid variant of Sec. III) through the C ABI against the oracle's
MultigridL: the preconditioner element by element (1, 2 and 3 levels, 2D and 3D, batched instances whose
hierarchy stops at the shallowest one), and time steps against the oracle's direct solve.  Needs an
MI355X."""
import math

import numpy as np
import pytest

from oracle.apfc_oracle import bcc_k, tri_k
from paper_1902_09761_amd import apfc, inputs
from tests.gpu_util import H_TRI, from_dev, oracle_for, phi_of, rel_l2, solver_for, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _pinv(meshes, kind, k, precision, nu, dt, max_levels=None, seed=81):
    rng = np.random.default_rng(seed)
    J = len(k)
    ins = [(rng.normal(size=(J, m.N)) + 1j * rng.normal(size=(J, m.N)),
            rng.normal(size=(J, m.N)) + 1j * rng.normal(size=(J, m.N))) for m in meshes]
    s = solver_for(meshes, kind, [0.02] * len(meshes), inner_kind=apfc.APFC_INNER_MG, precision=precision,
                   mass_iters=5, diff_iters=nu)
    zo = [torch.zeros((J, 2, m.N), dtype=torch.float64, device="cuda") for m in meshes]
    eo = [torch.zeros_like(z) for z in zo]
    s.apply(apfc.APFC_OP_PINV, [to_dev(a) for a, _ in ins], [to_dev(b) for _, b in ins], zo, eo, dt)
    worst = 0.0
    for b, m in enumerate(meshes):
        o = oracle_for(m, k, 0.02)
        gz, ge = from_dev(zo[b]), from_dev(eo[b])
        opts = dict(nu=nu, coarse_min=16 if m.dim == 2 else 8, coarse_iters=24, max_levels=max_levels)
        for j in range(J):
            c1, c2 = o.precond_apply(j, ins[b][0][j], ins[b][1][j], dt, inner="mg", mass_iters=5, mg_options=opts)
            ref = np.concatenate([c1, c2])
            got = np.concatenate([gz[j], ge[j]])
            worst = max(worst, np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    return worst


@pytest.mark.parametrize("precision,tol", [(apfc.APFC_FP64, 1e-12), (apfc.APFC_MIXED, 2e-5)])
@pytest.mark.parametrize("n,nu", [((64, 64), 2), ((96, 64), 3), ((40, 28), 2), ((128, 64), 1)])
def test_mg_preconditioner_matches_oracle_2d(n, nu, precision, tol):
    """64^2: levels 64, 32, 16; 96 x 64: 96 x 64, 48 x 32, 24 x 16; 40 x 28: no coarser level (the whole
    solve on the coarsest-level kernel); 128 x 64 with one smoothing iteration."""
    mesh = inputs.Mesh(2, (n[0], n[1], 1), (n[0] * H_TRI, n[1] * H_TRI, 1.0))
    err = _pinv([mesh], apfc.APFC_TRI2D, tri_k(), precision, nu, 7.0)
    print("mg P^-1", n, nu, err)
    assert err <= tol


def test_mg_preconditioner_batched_levels_stop_together():
    """A 32^2, a 64 x 96 and a 128^2 instance in one context: the hierarchy coarsens all instances
    together, so it stops where the smallest one does (two levels below the fine one would need 32/4 >= 16:
    one coarser level); the oracle's cycle is capped at the same depth."""
    meshes = [inputs.Mesh(2, (32, 32, 1), (32 * H_TRI, 32 * H_TRI, 1.0)),
              inputs.Mesh(2, (64, 96, 1), (64 * H_TRI, 96 * H_TRI, 1.0)),
              inputs.Mesh(2, (128, 128, 1), (128 * H_TRI, 128 * H_TRI, 1.0))]
    err = _pinv(meshes, apfc.APFC_TRI2D, tri_k(), apfc.APFC_FP64, 2, 3.0, max_levels=2)
    assert err <= 1e-12


def test_mg_preconditioner_matches_oracle_3d():
    """bcc on a 16^3 hex mesh: levels 16^3 and 8^3."""
    h = 60.0 * inputs.BCC_SPACING / 128.0
    mesh = inputs.Mesh(3, (16, 16, 16), (16 * h,) * 3)
    err = _pinv([mesh], apfc.APFC_BCC3D, bcc_k(), apfc.APFC_FP64, 2, 2.0)
    assert err <= 1e-12


@pytest.mark.parametrize("precision", [apfc.APFC_FP64, apfc.APFC_MIXED])
def test_mg_steps_match_oracle(precision):
    """The 64^2 grain, 4 steps with dt = 5 (the large-step regime the multigrid solve is for)."""
    wl = inputs.small_grain_2d(tri_k(), phi_of(tri_k()), n=64, seed=1)
    o = oracle_for(wl.mesh, tri_k(), wl.dB)
    ref = wl.eta0
    for _ in range(4):
        _, ref = o.step(ref, 5.0)
    s = solver_for([wl.mesh], apfc.APFC_TRI2D, [wl.dB], rtol=1e-12, precision=precision,
                   inner_kind=apfc.APFC_INNER_MG, mass_iters=5, diff_iters=2, restart=8)
    et = to_dev(wl.eta0)
    zt = torch.zeros_like(et)
    s.init_zeta([et], [zt])
    its = []
    for _ in range(4):
        its.append(s.step([et], [zt], 5.0)["max_iters"])
    err = rel_l2(from_dev(et), ref)
    print("mg steps", precision, "iterations", its, "rel-L2", err)
    assert err < 1e-9
