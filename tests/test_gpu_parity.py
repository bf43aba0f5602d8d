"""HIP path vs the CPU oracle, through the C ABI (needs an MI355X).

Tolerances: FP64 steps are solved to rtol 1e-12 so that the algebraic error stays far below
the 1e-9 relative-L2 parity bar on eta; the mixed path (FP32 preconditioner and Krylov basis Z
inside FP64 FGMRES, FP64 operator accumulation) reaches the same FP64 residual, so it is held
to the same bar.
"""
import math

import numpy as np
import pytest

from oracle.apfc_oracle import Grid, Oracle, Params, bcc_k, plane_wave, tri_k
from paper_1902_09761_amd import apfc, inputs
from tests.gpu_util import H_TRI, from_dev, oracle_for, phi_of, rel_l2, solver_for, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def run_gpu(solver, etas, dt, steps, zetas=None):
    et = [to_dev(e) for e in etas]
    zt = [torch.zeros_like(e) for e in et]
    solver.init_zeta(et, zt)
    infos = []
    for _ in range(steps):
        infos.append(solver.step(et, zt, dt))
    torch.cuda.synchronize()
    return [from_dev(e) for e in et], [from_dev(z) for z in zt], infos


@pytest.mark.parametrize("precision,inner", [(apfc.APFC_FP64, apfc.APFC_INNER_PCG), (apfc.APFC_MIXED, apfc.APFC_INNER_PCG),
                                             (apfc.APFC_FP64, apfc.APFC_INNER_CHEB), (apfc.APFC_MIXED, apfc.APFC_INNER_CHEB)])
def test_grain_64_matches_oracle(precision, inner):
    """64^2 triangular grain (radius 6 spacings, 5 degrees), dt = 1, 10 steps."""
    wl = inputs.small_grain_2d(tri_k(), phi_of(tri_k()), n=64, seed=1)
    o = oracle_for(wl.mesh, tri_k(), wl.dB)
    ref = wl.eta0
    for _ in range(wl.steps):
        _, ref = o.step(ref, wl.dt)
    kw = {"mass_iters": 4, "diff_iters": 4} if inner == apfc.APFC_INNER_CHEB else {}
    s = solver_for([wl.mesh], apfc.APFC_TRI2D, [wl.dB], rtol=1e-12, precision=precision, inner_kind=inner, **kw)
    got, _, infos = run_gpu(s, [wl.eta0], wl.dt, wl.steps)
    err = rel_l2(got[0], ref)
    print("rel-L2", err, "iters", [i["max_iters"] for i in infos])
    assert err < 1e-9


def test_ragged_nonsquare_mesh_and_zeta():
    """40 x 28 nodes (not multiples of the 64-wide tile or of any tile height): eta and zeta."""
    mesh = inputs.Mesh(2, (40, 28, 1), (40 * H_TRI, 28 * H_TRI, 1.0))
    eta0 = inputs.single_grain(mesh, tri_k(), phi_of(tri_k())(0.02), math.radians(7.0), 8 * H_TRI, seed=3)
    o = oracle_for(mesh, tri_k(), 0.02)
    z1, e1 = o.step(eta0, 0.7)
    z2, e2 = o.step(e1, 0.7)
    s = solver_for([mesh], apfc.APFC_TRI2D, [0.02], rtol=1e-12)
    got, zg, _ = run_gpu(s, [eta0], 0.7, 2)
    assert rel_l2(got[0], e2) < 1e-9
    assert rel_l2(zg[0], z2) < 1e-8


def test_picard_iterates():
    """K = 3 simplified-Newton iterates per step."""
    mesh = inputs.Mesh(2, (32, 32, 1), (32 * H_TRI, 32 * H_TRI, 1.0))
    eta0 = inputs.single_grain(mesh, tri_k(), phi_of(tri_k())(0.02), math.radians(5.0), 10 * H_TRI, seed=4)
    o = oracle_for(mesh, tri_k(), 0.02)
    _, ref = o.step(eta0, 1.0, picard=3)
    s = solver_for([mesh], apfc.APFC_TRI2D, [0.02], rtol=1e-12, picard_iters=3)
    got, _, _ = run_gpu(s, [eta0], 1.0, 1)
    assert rel_l2(got[0], ref) < 1e-9


def test_batch_uneven_instances():
    """Three instances of different sizes and Delta B in one batched context."""
    meshes = [inputs.Mesh(2, (32, 32, 1), (32 * H_TRI, 32 * H_TRI, 1.0)),
              inputs.Mesh(2, (48, 40, 1), (48 * H_TRI, 40 * H_TRI, 1.0)),
              inputs.Mesh(2, (64, 64, 1), (64 * H_TRI, 64 * H_TRI, 1.0))]
    dBs = [0.015, 0.03, 0.045]
    etas = [inputs.single_grain(m, tri_k(), phi_of(tri_k())(dB), math.radians(3.0 + 2 * i), 0.25 * m.length[0], seed=10 + i)
            for i, (m, dB) in enumerate(zip(meshes, dBs))]
    refs = []
    for m, dB, e in zip(meshes, dBs, etas):
        o = oracle_for(m, tri_k(), dB)
        for _ in range(3):
            _, e = o.step(e, 1.0)
        refs.append(e)
    s = solver_for(meshes, apfc.APFC_TRI2D, dBs, rtol=1e-12)
    got, _, _ = run_gpu(s, etas, 1.0, 3)
    for g, r in zip(got, refs):
        assert rel_l2(g, r) < 1e-9


@pytest.mark.parametrize("precision", [apfc.APFC_FP64, apfc.APFC_MIXED])
def test_bcc_3d_matches_oracle(precision):
    """bcc lattice, 6 amplitudes, 12 x 10 x 8 periodic hex mesh, rotated spherical grain."""
    h = 60.0 * inputs.BCC_SPACING / 128.0
    mesh = inputs.Mesh(3, (12, 10, 8), (12 * h, 10 * h, 8 * h))
    eta0 = inputs.single_grain(mesh, bcc_k(), phi_of(bcc_k())(0.02), math.radians(5.0), 4 * h, seed=5)
    o = oracle_for(mesh, bcc_k(), 0.02)
    ref = eta0
    for _ in range(2):
        _, ref = o.step(ref, 1.0)
    s = solver_for([mesh], apfc.APFC_BCC3D, [0.02], rtol=1e-12, precision=precision)
    got, _, _ = run_gpu(s, [eta0], 1.0, 2)
    assert rel_l2(got[0], ref) < 1e-9


def test_energy_and_gradient():
    mesh = inputs.Mesh(2, (32, 24, 1), (32 * H_TRI, 24 * H_TRI, 1.0))
    eta = inputs.single_grain(mesh, tri_k(), phi_of(tri_k())(0.02), math.radians(6.0), 9 * H_TRI, seed=6)
    o = oracle_for(mesh, tri_k(), 0.02)
    s = solver_for([mesh], apfc.APFC_TRI2D, [0.02])
    et = to_dev(eta)
    E = s.energy([et])[0]
    assert abs(E - o.energy(eta)) <= 1e-11 * abs(o.energy(eta))
    g = torch.zeros_like(et)
    ddB = s.energy_grad([et], [g])[0]
    gref = o.energy_grad(eta)
    assert rel_l2(from_dev(g), gref) < 1e-10
    assert abs(ddB - o.energy_ddB(eta)) < 1e-10 * abs(o.energy_ddB(eta))
    zt = torch.zeros_like(et)
    s.init_zeta([et], [zt])
    assert rel_l2(from_dev(zt), o.zeta_of(eta)) < 1e-11


def test_energy_bcc():
    h = 60.0 * inputs.BCC_SPACING / 128.0
    mesh = inputs.Mesh(3, (8, 8, 8), (8 * h, 8 * h, 8 * h))
    eta = inputs.single_grain(mesh, bcc_k(), phi_of(bcc_k())(0.02), math.radians(5.0), 3 * h, seed=7)
    o = oracle_for(mesh, bcc_k(), 0.02)
    s = solver_for([mesh], apfc.APFC_BCC3D, [0.02])
    E = s.energy([to_dev(eta)])[0]
    assert abs(E - o.energy(eta)) <= 1e-10 * abs(o.energy(eta))


@pytest.mark.parametrize("lattice", ["tri", "bcc"])
def test_adjoint_step_matches_oracle(lattice):
    if lattice == "tri":
        mesh = inputs.Mesh(2, (16, 16, 1), (16 * H_TRI, 16 * H_TRI, 1.0))
        k, kind = tri_k(), apfc.APFC_TRI2D
    else:
        h = 60.0 * inputs.BCC_SPACING / 128.0
        mesh = inputs.Mesh(3, (6, 6, 6), (6 * h, 6 * h, 6 * h))
        k, kind = bcc_k(), apfc.APFC_BCC3D
    J = len(k)
    rng = np.random.default_rng(8)
    eta0 = 0.12 + 0.04 * (rng.normal(size=(J, mesh.N)) + 1j * rng.normal(size=(J, mesh.N)))
    lam = rng.normal(size=(J, mesh.N)) + 1j * rng.normal(size=(J, mesh.N))
    o = oracle_for(mesh, k, 0.02)
    _, eta1 = o.step(eta0, 0.8)
    gref, dref = o.step_adjoint(eta0, eta1, 0.8, lam)
    s = solver_for([mesh], kind, [0.02], rtol=1e-13)
    out = torch.zeros((J, 2, mesh.N), dtype=torch.float64, device="cuda")
    ddB = s.step_adjoint([to_dev(eta0)], [to_dev(eta1)], 0.8, [to_dev(lam)], [out])[0]
    assert rel_l2(from_dev(out), gref) < 1e-9
    assert abs(ddB - dref) < 1e-9 * abs(dref)


def test_dispersion_plane_wave_on_gpu():
    """Linear problem (a2 = a3 = 0, one amplitude k = (0,1)) on a 16^2 mesh of side 40: one step
    multiplies the plane wave of mode (1,2) by 0.631922129131270 (closed form of the symbols)."""
    L = apfc.apfc_lattice()
    L.kind = apfc.APFC_CUSTOM
    L.J = 1
    L.k[0][1] = 1.0
    p = apfc.apfc_params_default(a2=0.0, a3=0.0, rtol=1e-14)
    s = apfc.Solver([apfc.make_mesh(2, (16, 16), (40.0, 40.0))], L, [p])
    g = Grid(2, (16, 16), (40.0, 40.0))
    e = plane_wave(g, (1, 2))[None, :]
    et = to_dev(e)
    zt = torch.zeros_like(et)
    s.step([et], [zt], 1.0)
    ratio = from_dev(et)[0] / e[0]
    np.testing.assert_allclose(ratio, 0.631922129131270, rtol=0, atol=1e-13)


def test_uniform_state_fixed_point_full_size():
    """eta_j = phi is a fixed point of the discrete step at the 1024^2 workload size."""
    n = 1024
    phi = phi_of(tri_k())(0.02)
    s = solver_for([inputs.mesh2d(n, n * 400.0 * inputs.TRI_SPACING / 1024.0)], apfc.APFC_TRI2D, [0.02])
    et = torch.full((3, 2, n * n), 0.0, dtype=torch.float64, device="cuda")
    et[:, 0, :] = phi
    zt = torch.zeros_like(et)
    s.step([et], [zt], 1.0)
    assert float((et[:, 0, :] - phi).abs().max()) < 1e-13
    assert float(et[:, 1, :].abs().max()) < 1e-13


def test_step_is_deterministic():
    wl = inputs.small_grain_2d(tri_k(), phi_of(tri_k()), n=64, seed=2)
    s = solver_for([wl.mesh], apfc.APFC_TRI2D, [wl.dB], rtol=1e-10)
    a, za, _ = run_gpu(s, [wl.eta0], 1.0, 2)
    b, zb, _ = run_gpu(s, [wl.eta0], 1.0, 2)
    assert np.array_equal(a[0], b[0]) and np.array_equal(za[0], zb[0])


def test_not_converged_leaves_state_untouched():
    wl = inputs.small_grain_2d(tri_k(), phi_of(tri_k()), n=64, seed=3)
    s = solver_for([wl.mesh], apfc.APFC_TRI2D, [wl.dB], rtol=1e-14, max_iters=1, restart=1)
    et = to_dev(wl.eta0)
    zt = torch.zeros_like(et)
    e_before, z_before = et.clone(), zt.clone()
    with pytest.raises(apfc.APFCNotConverged):
        s.step([et], [zt], 1.0)
    assert torch.equal(et, e_before) and torch.equal(zt, z_before)


def test_nonfinite_input_is_rejected():
    wl = inputs.small_grain_2d(tri_k(), phi_of(tri_k()), n=64, seed=4)
    s = solver_for([wl.mesh], apfc.APFC_TRI2D, [wl.dB])
    et = to_dev(wl.eta0)
    et[1, 0, 77] = float("nan")
    zt = torch.zeros_like(et)
    before = et.clone()
    with pytest.raises(apfc.APFCError) as ei:
        s.step([et], [zt], 1.0)
    assert ei.value.status == apfc.APFC_ERR_NONFINITE
    assert torch.equal(torch.nan_to_num(et, nan=7.0), torch.nan_to_num(before, nan=7.0))


def _rand_pair(J, N, seed):
    rng = np.random.default_rng(seed)
    return (rng.normal(size=(J, N)) + 1j * rng.normal(size=(J, N)),
            rng.normal(size=(J, N)) + 1j * rng.normal(size=(J, N)))


def test_operator_A_matches_oracle():
    """apfc_apply(APFC_OP_A) = the oracle's assembled block matrix times the same vector."""
    mesh = inputs.Mesh(2, (40, 28, 1), (40 * H_TRI, 28 * H_TRI, 1.0))
    lin = inputs.single_grain(mesh, tri_k(), phi_of(tri_k())(0.02), math.radians(7.0), 8 * H_TRI, seed=3)
    zin, ein = _rand_pair(3, mesh.N, 21)
    o = oracle_for(mesh, tri_k(), 0.02)
    d, _ = o.nodal(lin)
    s = solver_for([mesh], apfc.APFC_TRI2D, [0.02])
    zo, eo = torch.zeros((3, 2, mesh.N), dtype=torch.float64, device="cuda"), torch.zeros((3, 2, mesh.N), dtype=torch.float64, device="cuda")
    s.apply(apfc.APFC_OP_A, [to_dev(zin)], [to_dev(ein)], [zo], [eo], 0.7, lin_etas=[to_dev(lin)])
    gz, ge = from_dev(zo), from_dev(eo)
    for j in range(3):
        ref = o.block_matrix(j, d, 0.7) @ np.concatenate([zin[j], ein[j]])
        got = np.concatenate([gz[j], ge[j]])
        assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("inner,precision,tol", [(apfc.APFC_INNER_PCG, apfc.APFC_FP64, 1e-12),
                                                 (apfc.APFC_INNER_PCG, apfc.APFC_MIXED, 2e-5),
                                                 (apfc.APFC_INNER_CHEB, apfc.APFC_FP64, 1e-12),
                                                 (apfc.APFC_INNER_CHEB, apfc.APFC_MIXED, 2e-5)])
@pytest.mark.parametrize("n,tiles", [((40, 28), (16, 0)), ((256, 192), (8, 1)), ((256, 192), (32, 2)), ((96, 80), (4, 1)),
                                     ((256, 192), (16, 3)), ((96, 80), (8, 4))])
def test_preconditioner_matches_oracle(inner, precision, tol, n, tiles):
    """P^{-1} by its four steps on the GPU vs the oracle's four steps with the same inner solver
    (Jacobi-PCG 3/5 or Chebyshev 4/4), element by element: the largest deviation over all nodes of both
    fields, relative to the largest entry of the oracle's result, so that a wrong value on a single row or
    column at a tile or halo edge fails the test."""
    nx, ny = n
    mesh = inputs.Mesh(2, (nx, ny, 1), (nx * H_TRI, ny * H_TRI, 1.0))
    zin, ein = _rand_pair(3, mesh.N, 22)
    o = oracle_for(mesh, tri_k(), 0.02)
    its = (4, 4) if inner == apfc.APFC_INNER_CHEB else (3, 5)
    s = solver_for([mesh], apfc.APFC_TRI2D, [0.02], inner_kind=inner, precision=precision,
                   mass_iters=its[0], diff_iters=its[1])
    s.set_tiles(*tiles)
    zo, eo = torch.zeros((3, 2, mesh.N), dtype=torch.float64, device="cuda"), torch.zeros((3, 2, mesh.N), dtype=torch.float64, device="cuda")
    s.apply(apfc.APFC_OP_PINV, [to_dev(zin)], [to_dev(ein)], [zo], [eo], 0.7)
    gz, ge = from_dev(zo), from_dev(eo)
    for j in range(3):
        c1, c2 = o.precond_apply(j, zin[j], ein[j], 0.7, inner="cheb" if inner == apfc.APFC_INNER_CHEB else "pcg",
                                 mass_iters=its[0], diff_iters=its[1])
        ref = np.concatenate([c1, c2])
        got = np.concatenate([gz[j], ge[j]])
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        assert err <= tol, (j, err)


@pytest.mark.parametrize("inner,precision,tol", [(apfc.APFC_INNER_CHEB, apfc.APFC_FP64, 1e-12),
                                                 (apfc.APFC_INNER_CHEB, apfc.APFC_MIXED, 2e-5),
                                                 (apfc.APFC_INNER_PCG, apfc.APFC_FP64, 1e-12)])
def test_preconditioner_3d_matches_oracle(inner, precision, tol):
    """bcc lattice on a 12 x 10 x 8 hex mesh: the 3D preconditioner (one launch per Chebyshev
    iteration, or Jacobi-PCG) vs the oracle's four steps, element by element (largest deviation relative to
    the largest entry)."""
    h = 60.0 * inputs.BCC_SPACING / 128.0
    mesh = inputs.Mesh(3, (12, 10, 8), (12 * h, 10 * h, 8 * h))
    zin, ein = _rand_pair(6, mesh.N, 23)
    o = oracle_for(mesh, bcc_k(), 0.02)
    its = (4, 4) if inner == apfc.APFC_INNER_CHEB else (3, 5)
    s = solver_for([mesh], apfc.APFC_BCC3D, [0.02], inner_kind=inner, precision=precision,
                   mass_iters=its[0], diff_iters=its[1])
    zo = torch.zeros((6, 2, mesh.N), dtype=torch.float64, device="cuda")
    eo = torch.zeros_like(zo)
    s.apply(apfc.APFC_OP_PINV, [to_dev(zin)], [to_dev(ein)], [zo], [eo], 0.9)
    gz, ge = from_dev(zo), from_dev(eo)
    for j in range(6):
        c1, c2 = o.precond_apply(j, zin[j], ein[j], 0.9, inner="cheb" if inner == apfc.APFC_INNER_CHEB else "pcg",
                                 mass_iters=its[0], diff_iters=its[1])
        ref = np.concatenate([c1, c2])
        got = np.concatenate([gz[j], ge[j]])
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        assert err <= tol, (j, err)


@pytest.mark.parametrize("precision", [apfc.APFC_FP64, apfc.APFC_MIXED])
def test_bcc_3d_chebyshev_step_matches_oracle(precision):
    h = 60.0 * inputs.BCC_SPACING / 128.0
    mesh = inputs.Mesh(3, (12, 10, 8), (12 * h, 10 * h, 8 * h))
    eta0 = inputs.single_grain(mesh, bcc_k(), phi_of(bcc_k())(0.02), math.radians(5.0), 4 * h, seed=5)
    o = oracle_for(mesh, bcc_k(), 0.02)
    ref = eta0
    for _ in range(2):
        _, ref = o.step(ref, 1.0)
    s = solver_for([mesh], apfc.APFC_BCC3D, [0.02], rtol=1e-12, precision=precision,
                   inner_kind=apfc.APFC_INNER_CHEB, mass_iters=4, diff_iters=4, restart=6)
    got, _, _ = run_gpu(s, [eta0], 1.0, 2)
    assert rel_l2(got[0], ref) < 1e-9


@pytest.mark.parametrize("tile_rows", [4, 8, 16, 32])
def test_bcc_3d_ragged_bricks(tile_rows):
    """8 x 6 x 5 hex mesh: every brick height TY/4 in {1, 2, 4, 8} leaves a ragged last brick in z
    (and the 64 x 4 brick footprint is ragged in x and y); nz = 5 < TY/4 + 2 makes the plane march wrap
    around the periodic z direction more than once.  Operator apply, preconditioner and two Chebyshev
    steps against the oracle."""
    h = 60.0 * inputs.BCC_SPACING / 128.0
    mesh = inputs.Mesh(3, (8, 6, 5), (8 * h, 6 * h, 5 * h))
    o = oracle_for(mesh, bcc_k(), 0.02)
    s = solver_for([mesh], apfc.APFC_BCC3D, [0.02], rtol=1e-12, inner_kind=apfc.APFC_INNER_CHEB,
                   mass_iters=4, diff_iters=4, restart=6)
    s.set_tiles(tile_rows)
    assert s.get_tiles()[0] == tile_rows
    zin, ein = _rand_pair(6, mesh.N, 31)
    eta_lin = inputs.single_grain(mesh, bcc_k(), phi_of(bcc_k())(0.02), math.radians(5.0), 2 * h, seed=8)
    d, _ = o.nodal(eta_lin)
    for op in (apfc.APFC_OP_A, apfc.APFC_OP_PINV):
        zo = torch.zeros((6, 2, mesh.N), dtype=torch.float64, device="cuda")
        eo = torch.zeros_like(zo)
        s.apply(op, [to_dev(zin)], [to_dev(ein)], [zo], [eo], 0.9, [to_dev(eta_lin)])
        gz, ge = from_dev(zo), from_dev(eo)
        for j in range(6):
            if op == apfc.APFC_OP_A:
                ref = o.block_matrix(j, d, 0.9) @ np.concatenate([zin[j], ein[j]])
            else:
                c1, c2 = o.precond_apply(j, zin[j], ein[j], 0.9, inner="cheb", mass_iters=4, diff_iters=4)
                ref = np.concatenate([c1, c2])
            got = np.concatenate([gz[j], ge[j]])
            assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref)), (op, j)
    ref = eta_lin
    for _ in range(2):
        _, ref = o.step(ref, 1.0)
    got, _, _ = run_gpu(s, [eta_lin], 1.0, 2)
    assert rel_l2(got[0], ref) < 1e-9


@pytest.mark.parametrize("tile_rows", [8, 32])
@pytest.mark.parametrize("inner", [apfc.APFC_INNER_CHEB, apfc.APFC_INNER_PCG])
def test_tiles_taller_than_the_mesh(tile_rows, inner):
    """40 x 6 nodes with tiles of 8 or 32 rows: the column march starts past the last row and wraps the
    periodic y direction more than once; the fused preconditioner regions wrap as well."""
    mesh = inputs.Mesh(2, (40, 6, 1), (40 * H_TRI, 6 * H_TRI, 1.0))
    eta0 = inputs.single_grain(mesh, tri_k(), phi_of(tri_k())(0.02), math.radians(7.0), 3 * H_TRI, seed=13)
    o = oracle_for(mesh, tri_k(), 0.02)
    ref = eta0
    for _ in range(3):
        _, ref = o.step(ref, 1.0)
    kw = {"mass_iters": 4, "diff_iters": 4} if inner == apfc.APFC_INNER_CHEB else {}
    s = solver_for([mesh], apfc.APFC_TRI2D, [0.02], rtol=1e-12, inner_kind=inner, restart=5, **kw)
    s.set_tiles(tile_rows)
    got, _, _ = run_gpu(s, [eta0], 1.0, 3)
    assert rel_l2(got[0], ref) < 1e-9


@pytest.mark.parametrize("precision", [apfc.APFC_FP64, apfc.APFC_MIXED])
def test_second_gram_schmidt_pass(precision):
    """rtol 5e-14 sets the second-pass threshold to (100 eps / rtol)^2 = 0.19 (re-orthogonalise
    whenever the first pass removed more than 81% of |w|^2), so the second pass and its fused reduction
    run in many iterations; 4 steps of the 64^2 grain (mixed precision: 3 steps) against
    the oracle.  The timing probe on k_gs counts the launches in which some system took the second pass
    (launches where none did are left out of its count), which must be nonzero."""
    wl = inputs.small_grain_2d(tri_k(), phi_of(tri_k()), n=64, seed=1)
    o = oracle_for(wl.mesh, tri_k(), wl.dB)
    steps = 4 if precision == apfc.APFC_FP64 else 3
    ref = wl.eta0
    for _ in range(steps):
        _, ref = o.step(ref, wl.dt)
    rtol = 5e-14
    s = solver_for([wl.mesh], apfc.APFC_TRI2D, [wl.dB], rtol=rtol, precision=precision,
                   inner_kind=apfc.APFC_INNER_CHEB, mass_iters=5, diff_iters=3, restart=8, max_iters=2000)
    s.probe_enable("gs", 1)
    got, _, infos = run_gpu(s, [wl.eta0], wl.dt, steps)
    n_second, _, _ = s.probe_read()
    s.probe_enable(None, 1)
    # the probe keeps a k_gs launch only if some system took the second pass in it
    print("launches with a second pass", n_second)
    assert n_second > 0
    assert rel_l2(got[0], ref) < 1e-10
