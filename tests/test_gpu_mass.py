"""The separable mass inverse (APFC_MASS_SEPARABLE: step 1 of P^{-1} by the Kronecker product of the
truncated 1D inverses of the mass matrix, reading R18 of the oracle) on the GPU against the oracle's four
steps with the same operator, element by element, for every inner solver and tap count, in 2D (fused LDS
stage and standalone bricks) and 3D; and time steps with it against the oracle's steps.  Needs an MI355X."""
import math

import numpy as np
import pytest

from oracle.apfc_oracle import bcc_k, fcc_k, tri_k
from paper_1902_09761_amd import apfc, inputs
from tests.gpu_util import H_TRI, eq_of, from_dev, oracle_for, phi_of, rel_l2, solver_for, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

H_BCC = 60.0 * inputs.BCC_SPACING / 128.0
INNER = {apfc.APFC_INNER_PCG: "pcg", apfc.APFC_INNER_CHEB: "cheb", apfc.APFC_INNER_MG: "mg"}


def _rand_pair(J, N, seed):
    rng = np.random.default_rng(seed)
    return (rng.normal(size=(J, N)) + 1j * rng.normal(size=(J, N)),
            rng.normal(size=(J, N)) + 1j * rng.normal(size=(J, N)))


def _pinv_err(mesh, kind, k, inner, precision, R, diff, dt, tiles=None, seed=31):
    """Largest deviation of P^{-1} (both fields, every amplitude) from the oracle's, relative to the
    largest entry of the oracle's result."""
    J = len(k)
    zin, ein = _rand_pair(J, mesh.N, seed)
    o = oracle_for(mesh, k, 0.02)
    s = solver_for([mesh], kind, [0.02], inner_kind=inner, precision=precision, mass_kind=apfc.APFC_MASS_SEPARABLE,
                   mass_iters=R, diff_iters=diff)
    if tiles:
        s.set_tiles(*tiles)
    zo = torch.zeros((J, 2, mesh.N), dtype=torch.float64, device="cuda")
    eo = torch.zeros_like(zo)
    s.apply(apfc.APFC_OP_PINV, [to_dev(zin)], [to_dev(ein)], [zo], [eo], dt)
    gz, ge = from_dev(zo), from_dev(eo)
    worst = 0.0
    mg = dict(nu=diff, coarse_min=16 if mesh.dim == 2 else 8, coarse_iters=24) if inner == apfc.APFC_INNER_MG else None
    for j in range(J):
        c1, c2 = o.precond_apply(j, zin[j], ein[j], dt, inner=INNER[inner], mass_iters=R, diff_iters=diff,
                                 mass="sep", mg_options=mg)
        ref = np.concatenate([c1, c2])
        got = np.concatenate([gz[j], ge[j]])
        worst = max(worst, float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))))
    return worst


@pytest.mark.parametrize("precision,tol", [(apfc.APFC_FP64, 1e-12), (apfc.APFC_MIXED, 2e-5)])
@pytest.mark.parametrize("n,tiles,R", [((256, 192), (32, 3), 3), ((40, 28), (16, 0), 2), ((96, 80), (8, 1), 1),
                                       ((256, 192), (16, 5), 4), ((130, 70), (32, 2), 3), ((96, 80), (8, 4), 2)])
def test_fused_2d_stage_matches_oracle(precision, tol, n, tiles, R):
    """The fused 2D Chebyshev preconditioner with the separable stage 0: every region shape, ragged meshes
    (40 x 28, smaller than a region; 130 x 70), every tap count."""
    nx, ny = n
    mesh = inputs.Mesh(2, (nx, ny, 1), (nx * H_TRI, ny * H_TRI, 1.0))
    err = _pinv_err(mesh, apfc.APFC_TRI2D, tri_k(), apfc.APFC_INNER_CHEB, precision, R, 3, 0.7, tiles)
    print("fused sep", n, tiles, R, precision, err)
    assert err <= tol


@pytest.mark.parametrize("inner", [apfc.APFC_INNER_PCG, apfc.APFC_INNER_MG])
@pytest.mark.parametrize("precision,tol", [(apfc.APFC_FP64, 1e-12), (apfc.APFC_MIXED, 2e-5)])
def test_standalone_2d_bricks_match_oracle(inner, precision, tol):
    """The brick kernel in 2D (PCG and multigrid inner solvers): 136 x 100, ragged in x and y."""
    mesh = inputs.Mesh(2, (136, 100, 1), (136 * H_TRI, 100 * H_TRI, 1.0))
    diff = 5 if inner == apfc.APFC_INNER_PCG else 2
    err = _pinv_err(mesh, apfc.APFC_TRI2D, tri_k(), inner, precision, 3, diff, 1.5)
    print("2d bricks", inner, precision, err)
    assert err <= tol


@pytest.mark.parametrize("n,R,precision,tol", [((12, 10, 8), 3, apfc.APFC_FP64, 1e-12),
                                               ((12, 10, 8), 2, apfc.APFC_MIXED, 2e-5),
                                               ((70, 20, 36), 4, apfc.APFC_FP64, 1e-12),
                                               ((70, 20, 36), 1, apfc.APFC_MIXED, 2e-5),
                                               ((8, 6, 4), 3, apfc.APFC_FP64, 1e-12)])
def test_3d_bricks_match_oracle(n, R, precision, tol):
    """3D Chebyshev preconditioner with the separable mass inverse on bcc: a mesh inside one brick,
    a ragged multi-brick mesh (70 x 20 x 36: x, y and z bricks cut), and 8 x 6 x 4, where the taps wrap
    onto the same node in every direction."""
    mesh = inputs.Mesh(3, n, tuple(v * H_BCC for v in n))
    err = _pinv_err(mesh, apfc.APFC_BCC3D, bcc_k(), apfc.APFC_INNER_CHEB, precision, R, 3, 0.9)
    print("3d bricks", n, R, precision, err)
    assert err <= tol


@pytest.mark.parametrize("diff", [1, 2, 5])
@pytest.mark.parametrize("precision,tol", [(apfc.APFC_FP64, 1e-12), (apfc.APFC_MIXED, 2e-5)])
def test_3d_diffusion_iteration_counts(diff, precision, tol):
    """The three-term 3D L solves for every shape of the iteration sequence: one iteration (the start
    writes the result), two (the first iteration also forms step 4), five (plain iterations after the
    second); 20 x 12 x 18, ragged in every direction."""
    n = (20, 12, 18)
    mesh = inputs.Mesh(3, n, tuple(v * H_BCC for v in n))
    err = _pinv_err(mesh, apfc.APFC_BCC3D, bcc_k(), apfc.APFC_INNER_CHEB, precision, 3, diff, 0.9)
    print("3d diffusion iterations", diff, precision, err)
    assert err <= tol


@pytest.mark.parametrize("precision,tol", [(apfc.APFC_FP64, 1e-12), (apfc.APFC_MIXED, 2e-5)])
def test_deep_bricks_in_a_large_batch(precision, tol):
    """128 bcc systems of 16 x 16 x 32 (768 amplitude systems: 3072 bricks of 16 planes, which fill three
    rounds of the chip, so the 3D L solves and the mass inverse take the deep bricks): P^{-1} of systems 0,
    77 and 127, each with its own input, against the oracle's."""
    S, n, dt = 128, (16, 16, 32), 0.8
    mesh = inputs.Mesh(3, n, tuple(v * H_BCC for v in n))
    k = bcc_k()
    J = len(k)
    pairs = [_rand_pair(J, mesh.N, 100 + q) for q in range(S)]
    s = solver_for([mesh] * S, apfc.APFC_BCC3D, [0.02] * S, inner_kind=apfc.APFC_INNER_CHEB, precision=precision,
                   mass_kind=apfc.APFC_MASS_SEPARABLE, mass_iters=3, diff_iters=3)
    zo = [torch.zeros((J, 2, mesh.N), dtype=torch.float64, device="cuda") for _ in range(S)]
    eo = [torch.zeros_like(t) for t in zo]
    s.apply(apfc.APFC_OP_PINV, [to_dev(z) for z, _ in pairs], [to_dev(e) for _, e in pairs], zo, eo, dt)
    o = oracle_for(mesh, k, 0.02)
    worst = 0.0
    for q in (0, 77, 127):
        gz, ge = from_dev(zo[q]), from_dev(eo[q])
        zin, ein = pairs[q]
        for j in range(J):
            c1, c2 = o.precond_apply(j, zin[j], ein[j], dt, inner="cheb", mass_iters=3, diff_iters=3, mass="sep")
            ref = np.concatenate([c1, c2])
            worst = max(worst, float(np.max(np.abs(np.concatenate([gz[j], ge[j]]) - ref)) / np.max(np.abs(ref))))
    print("deep bricks", precision, worst)
    assert worst <= tol


@pytest.mark.parametrize("precision", [apfc.APFC_FP64, apfc.APFC_MIXED])
def test_steps_with_separable_mass_match_oracle(precision):
    """Three steps of the 64^2 grain (fused 2D path) and two of a bcc 12 x 10 x 8 grain (3D bricks) with
    the separable mass inverse: the result is the oracle's step to the solver tolerance."""
    wl = inputs.small_grain_2d(tri_k(), phi_of(tri_k()), n=64, seed=1)
    o = oracle_for(wl.mesh, tri_k(), wl.dB)
    ref = wl.eta0
    for _ in range(3):
        _, ref = o.step(ref, 1.0)
    s = solver_for([wl.mesh], apfc.APFC_TRI2D, [wl.dB], rtol=1e-12, precision=precision, inner_kind=apfc.APFC_INNER_CHEB,
                   mass_kind=apfc.APFC_MASS_SEPARABLE, mass_iters=3, diff_iters=3, restart=4, x0_order=3)
    et = to_dev(wl.eta0)
    zt = torch.zeros_like(et)
    s.init_zeta([et], [zt])
    for _ in range(3):
        s.step([et], [zt], 1.0)
    err = rel_l2(from_dev(et), ref)
    print("2d steps", precision, err)
    assert err < 1e-9

    mesh = inputs.Mesh(3, (12, 10, 8), (12 * H_BCC, 10 * H_BCC, 8 * H_BCC))
    eta0 = inputs.single_grain(mesh, bcc_k(), phi_of(bcc_k())(0.02), math.radians(5.0), 4 * H_BCC, seed=5)
    o = oracle_for(mesh, bcc_k(), 0.02)
    ref = eta0
    for _ in range(2):
        _, ref = o.step(ref, 1.0)
    s = solver_for([mesh], apfc.APFC_BCC3D, [0.02], rtol=1e-12, precision=precision, inner_kind=apfc.APFC_INNER_CHEB,
                   mass_kind=apfc.APFC_MASS_SEPARABLE, mass_iters=2, diff_iters=3, restart=4)
    et = to_dev(eta0)
    zt = torch.zeros_like(et)
    s.init_zeta([et], [zt])
    for _ in range(2):
        s.step([et], [zt], 1.0)
    err = rel_l2(from_dev(et), ref)
    print("3d steps", precision, err)
    assert err < 1e-9


def test_fcc_preconditioner_with_separable_mass():
    """FCC (7 amplitudes) on 10 x 12 x 9 in mixed precision."""
    mesh = inputs.Mesh(3, (10, 12, 9), tuple(v * 60.0 * inputs.FCC_SPACING / 128.0 for v in (10, 12, 9)))
    err = _pinv_err(mesh, apfc.APFC_FCC3D, fcc_k(), apfc.APFC_INNER_CHEB, apfc.APFC_MIXED, 3, 3, 1.0)
    assert err <= 2e-5
