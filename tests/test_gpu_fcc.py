"""The FCC lattice (J = 7: the <111> and <200> shells; the paper's 3D workload) through the C ABI against
the oracle: steps, preconditioner, energy and its gradient, adjoint step, the two-shell relaxed crystal
as a fixed point, and a full-size 128^3 certificate in the benchmark's launch configuration.  Needs an
MI355X."""
import math

import numpy as np
import pytest

from oracle.apfc_oracle import BulkEnergy, Grid, Oracle, Params, equilibrium_amplitudes, fcc_k
from paper_1902_09761_amd import apfc, inputs
from tests.gpu_util import eq_of, from_dev, oracle_for, rel_l2, solver_for, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

H = 60.0 * inputs.FCC_SPACING / 128.0      # mesh size of the 128^3 FCC sphere


def _small(n=(12, 10, 8)):
    mesh = inputs.Mesh(3, n, tuple(H * v for v in n))
    eta0 = inputs.single_grain(mesh, fcc_k(), eq_of(fcc_k())(0.02), math.radians(5.0), 4 * H, seed=71)
    return mesh, eta0


def _run(s, eta0, dt, steps):
    et = to_dev(eta0)
    zt = torch.zeros_like(et)
    s.init_zeta([et], [zt])
    for _ in range(steps):
        s.step([et], [zt], dt)
    torch.cuda.synchronize()
    return from_dev(et), from_dev(zt)


def test_library_lattice_and_relaxed_amplitudes():
    L = apfc.apfc_lattice_default(apfc.APFC_FCC3D)
    assert L.J == 7
    np.testing.assert_allclose(np.array(apfc.lattice_k(L, 3)), fcc_k(), atol=1e-15)
    for dB in (0.01, 0.03):
        got = apfc.apfc_equilibrium_amplitudes(L, apfc.apfc_params_default(a1=0.5 * dB))
        np.testing.assert_allclose(got, equilibrium_amplitudes(BulkEnergy(fcc_k(), Params.from_dB(dB))), rtol=1e-13)


@pytest.mark.parametrize("precision,inner", [(apfc.APFC_FP64, apfc.APFC_INNER_PCG), (apfc.APFC_MIXED, apfc.APFC_INNER_CHEB),
                                             (apfc.APFC_FP64, apfc.APFC_INNER_CHEB)])
def test_fcc_steps_match_oracle(precision, inner):
    """12 x 10 x 8 hex mesh, a rotated spherical grain in the two-shell relaxed crystal, two steps."""
    mesh, eta0 = _small()
    o = oracle_for(mesh, fcc_k(), 0.02)
    ref = eta0
    for _ in range(2):
        _, ref = o.step(ref, 1.0)
    kw = {"mass_iters": 4, "diff_iters": 4, "restart": 6} if inner == apfc.APFC_INNER_CHEB else {}
    s = solver_for([mesh], apfc.APFC_FCC3D, [0.02], rtol=1e-12, precision=precision, inner_kind=inner, **kw)
    got, _ = _run(s, eta0, 1.0, 2)
    err = rel_l2(got, ref)
    print("fcc rel-L2", err)
    assert err < 1e-9


@pytest.mark.parametrize("inner,precision,tol", [(apfc.APFC_INNER_CHEB, apfc.APFC_FP64, 1e-12),
                                                 (apfc.APFC_INNER_CHEB, apfc.APFC_MIXED, 2e-5),
                                                 (apfc.APFC_INNER_PCG, apfc.APFC_FP64, 1e-12)])
def test_fcc_preconditioner_matches_oracle(inner, precision, tol):
    """P^{-1} element by element; the <200> systems have kappa = 4 a0 / 3 (other Chebyshev bounds)."""
    mesh, _ = _small((8, 6, 6))
    rng = np.random.default_rng(72)
    zin = rng.normal(size=(7, mesh.N)) + 1j * rng.normal(size=(7, mesh.N))
    ein = rng.normal(size=(7, mesh.N)) + 1j * rng.normal(size=(7, mesh.N))
    o = oracle_for(mesh, fcc_k(), 0.02)
    its = (4, 4) if inner == apfc.APFC_INNER_CHEB else (3, 5)
    s = solver_for([mesh], apfc.APFC_FCC3D, [0.02], inner_kind=inner, precision=precision, mass_iters=its[0],
                   diff_iters=its[1])
    zo = torch.zeros((7, 2, mesh.N), dtype=torch.float64, device="cuda")
    eo = torch.zeros_like(zo)
    s.apply(apfc.APFC_OP_PINV, [to_dev(zin)], [to_dev(ein)], [zo], [eo], 0.9)
    gz, ge = from_dev(zo), from_dev(eo)
    for j in range(7):
        c1, c2 = o.precond_apply(j, zin[j], ein[j], 0.9, inner="cheb" if inner == apfc.APFC_INNER_CHEB else "pcg",
                                 mass_iters=its[0], diff_iters=its[1])
        ref = np.concatenate([c1, c2])
        got = np.concatenate([gz[j], ge[j]])
        assert np.max(np.abs(got - ref)) <= tol * np.max(np.abs(ref)), j


def test_fcc_energy_gradient_and_adjoint():
    mesh, eta = _small((8, 6, 6))
    o = oracle_for(mesh, fcc_k(), 0.02)
    s = solver_for([mesh], apfc.APFC_FCC3D, [0.02], rtol=1e-13)
    et = to_dev(eta)
    E = s.energy([et])[0]
    assert abs(E - o.energy(eta)) <= 1e-10 * abs(o.energy(eta))
    g = torch.zeros_like(et)
    ddB = s.energy_grad([et], [g])[0]
    assert rel_l2(from_dev(g), o.energy_grad(eta)) < 1e-10
    assert abs(ddB - o.energy_ddB(eta)) < 1e-10 * abs(o.energy_ddB(eta))
    rng = np.random.default_rng(73)
    lam = rng.normal(size=(7, mesh.N)) + 1j * rng.normal(size=(7, mesh.N))
    _, eta1 = o.step(eta, 0.8)
    gref, dref = o.step_adjoint(eta, eta1, 0.8, lam)
    out = torch.zeros((7, 2, mesh.N), dtype=torch.float64, device="cuda")
    d = s.step_adjoint([et], [to_dev(eta1)], 0.8, [to_dev(lam)], [out])[0]
    assert rel_l2(from_dev(out), gref) < 1e-9
    assert abs(d - dref) < 1e-9 * abs(dref)


def test_fcc_relaxed_crystal_is_a_fixed_point_at_full_size():
    """eta_j = phi_shell(j) (the library's two-shell relaxed amplitudes) is reproduced by a step on the
    128^3 mesh to rounding."""
    n = 128
    L = apfc.apfc_lattice_default(apfc.APFC_FCC3D)
    p = apfc.apfc_params_default(a1=0.01)
    phi = apfc.apfc_equilibrium_amplitudes(L, p)
    s = apfc.Solver([apfc.make_mesh(3, (n, n, n), (n * H,) * 3)], L, [p])
    et = torch.zeros((7, 2, n ** 3), dtype=torch.float64, device="cuda")
    for j in range(7):
        et[j, 0, :] = phi[j]
    zt = torch.zeros_like(et)
    s.step([et], [zt], 1.0)
    for j in range(7):
        assert float((et[j, 0, :] - phi[j]).abs().max()) < 1e-13
    assert float(et[:, 1, :].abs().max()) < 1e-13


def test_fcc128_full_size_steps_solve_the_oracle_system():
    """The 128^3 FCC sphere (7 amplitudes, 14.7 M amplitude DOF) in the benchmark's launch configuration
    (mixed precision, separable mass inverse of 3 taps and 3 Chebyshev diffusion iterations, restart 4,
    cubic extrapolated guess, autotuned bricks): three steps,
    the third certified against the oracle's block systems (Kronecker assembly)."""
    wl = inputs.sphere_3d(fcc_k(), eq_of(fcc_k()), n=128, seed=1, spacing=inputs.FCC_SPACING, name="fcc")
    p = apfc.apfc_params_default(a1=0.5 * wl.dB, rtol=1e-8, precision=apfc.APFC_MIXED,
                                 inner_kind=apfc.APFC_INNER_CHEB, restart=4,
                                 mass_kind=apfc.APFC_MASS_SEPARABLE, mass_iters=3, diff_iters=3, x0_order=3)
    s = apfc.Solver([apfc.make_mesh(3, wl.mesh.n, wl.mesh.length)], apfc.apfc_lattice_default(apfc.APFC_FCC3D), [p])
    s.autotune()
    et = to_dev(wl.eta0)
    zt = torch.zeros_like(et)
    s.init_zeta([et], [zt])
    for m in range(3):
        eta_in = from_dev(et)
        info = s.step([et], [zt], wl.dt)
    o = Oracle(Grid(3, wl.mesh.n, wl.mesh.length), fcc_k(), Params.from_dB(wl.dB), assembly="kron")
    d, h = o.nodal(eta_in)
    eta1, zeta1 = from_dev(et), from_dev(zt)
    worst = 0.0
    for j in range(7):
        b = o.rhs(j, eta_in[j], h[j], wl.dt)
        y1, y2 = o.apply_block(j, d, wl.dt, zeta1[j], eta1[j])
        worst = max(worst, np.linalg.norm(b - np.concatenate([y1, y2])) / np.linalg.norm(b))
    print("relres (oracle)", worst, "relres (GPU)", info["max_relres"], "iterations", info["max_iters"])
    assert worst <= 1.01e-8
    assert abs(worst - info["max_relres"]) <= 1e-11
