"""The benchmark workloads at full size, in the launch configuration bench.py times (separable mass
inverse of 3 taps and 3 Chebyshev diffusion iterations as inner solves, restart 4, cubic extrapolated
initial guess, autotuned tiles): the 1024^2 triangular
polycrystal, the 128^3 bcc sphere and the 64-instance batch.  The oracle cannot factor these systems in
reasonable time, so it checks a property that holds at any size: with its own assembly and its own
nodal linearisation it forms every amplitude's block system Eq. (11) and verifies that the GPU's step
result solves it to the requested relative residual.  Needs an MI355X."""
import numpy as np
import pytest

from oracle.apfc_oracle import BulkEnergy, Grid, Oracle, Params, tri_k, uniform_amplitude
from paper_1902_09761_amd import apfc, inputs
from tests.gpu_util import from_dev, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

_ORACLE = {}


def _oracle_and_workload():
    if "o" not in _ORACLE:
        wl = inputs.voronoi_2d(tri_k(), lambda dB: uniform_amplitude(BulkEnergy(tri_k(), Params.from_dB(dB))),
                               n=1024, seed=1)
        o = Oracle(Grid(2, (1024, 1024), wl.mesh.length[:2]), tri_k(), Params.from_dB(wl.dB))
        _ORACLE["o"], _ORACLE["wl"] = o, wl
    return _ORACLE["o"], _ORACLE["wl"]


@pytest.mark.parametrize("precision", [apfc.APFC_FP64, apfc.APFC_MIXED])
def test_full_size_step_solves_the_oracle_system(precision):
    """Five steps with the cubic extrapolated initial guess (as bench.py runs them); the first and the
    last step are certified."""
    o, wl = _oracle_and_workload()
    p = apfc.apfc_params_default(a1=0.5 * wl.dB, rtol=wl.rtol, precision=precision, inner_kind=apfc.APFC_INNER_CHEB,
                                 restart=4, mass_kind=apfc.APFC_MASS_SEPARABLE, mass_iters=3,
                                 diff_iters=3, x0_order=3)
    s = apfc.Solver([apfc.make_mesh(2, wl.mesh.n, wl.mesh.length)], apfc.apfc_lattice_default(apfc.APFC_TRI2D), [p])
    s.autotune()
    et = to_dev(wl.eta0)
    zt = torch.zeros_like(et)
    s.init_zeta([et], [zt])
    checked = {}
    for m in range(5):
        eta_in = from_dev(et)
        info = s.step([et], [zt], wl.dt)
        if m in (0, 4):
            checked[m] = (eta_in, from_dev(et), from_dev(zt), info)
    for m, (eta_in, eta1, zeta1, info) in checked.items():
        d, h = o.nodal(eta_in)
        worst = 0.0
        for j in range(3):
            A = o.block_matrix(j, d, wl.dt).tocsr()
            b = o.rhs(j, eta_in[j], h[j], wl.dt)
            r = b - A @ np.concatenate([zeta1[j], eta1[j]])
            worst = max(worst, np.linalg.norm(r) / np.linalg.norm(b))
        print("step", m, "relres (oracle)", worst, "relres (GPU)", info["max_relres"], "iterations", info["iters"])
        assert worst <= 1.01 * wl.rtol
        assert abs(worst - info["max_relres"]) <= 1e-3 * wl.rtol


def _certify(o, dt, eta_in, eta1, zeta1):
    """Largest relative residual over the amplitudes of the block systems Eq. (11) the oracle forms
    from eta_in (its own nodal linearisation and right-hand side) at the GPU's result."""
    d, h = o.nodal(eta_in)
    worst = 0.0
    for j in range(o.J):
        b = o.rhs(j, eta_in[j], h[j], dt)
        y1, y2 = o.apply_block(j, d, dt, zeta1[j], eta1[j])
        worst = max(worst, np.linalg.norm(b - np.concatenate([y1, y2])) / np.linalg.norm(b))
    return worst


def test_bcc128_full_size_steps_solve_the_oracle_system():
    """The 128^3 bcc sphere (6 amplitudes) in the benchmark's launch configuration (mixed precision,
    separable mass inverse of 3 taps and 3 Chebyshev diffusion iterations, restart 4, cubic extrapolated
    guess, autotuned bricks): three steps, the third
    certified against the oracle's block systems (Kronecker assembly, equal to the element loop)."""
    from oracle.apfc_oracle import bcc_k
    wl = inputs.sphere_3d(bcc_k(), lambda dB: uniform_amplitude(BulkEnergy(bcc_k(), Params.from_dB(dB))), n=128,
                          seed=1)
    p = apfc.apfc_params_default(a1=0.5 * wl.dB, rtol=1e-8, precision=apfc.APFC_MIXED,
                                 inner_kind=apfc.APFC_INNER_CHEB, restart=4,
                                 mass_kind=apfc.APFC_MASS_SEPARABLE, mass_iters=3, diff_iters=3, x0_order=3)
    s = apfc.Solver([apfc.make_mesh(3, wl.mesh.n, wl.mesh.length)], apfc.apfc_lattice_default(apfc.APFC_BCC3D), [p])
    s.autotune()
    et = to_dev(wl.eta0)
    zt = torch.zeros_like(et)
    s.init_zeta([et], [zt])
    for m in range(3):
        eta_in = from_dev(et)
        info = s.step([et], [zt], wl.dt)
    o = Oracle(Grid(3, wl.mesh.n, wl.mesh.length), bcc_k(), Params.from_dB(wl.dB), assembly="kron")
    worst = _certify(o, wl.dt, eta_in, from_dev(et), from_dev(zt))
    print("relres (oracle)", worst, "relres (GPU)", info["max_relres"], "iterations", info["max_iters"])
    assert worst <= 1.01e-8
    assert abs(worst - info["max_relres"]) <= 1e-11


def test_batch64_full_size_every_instance():
    """The 64-instance batch (n^2, n in {128..512}) in the benchmark's launch configuration: two
    batched steps, then every instance certified against the oracle's block systems (Kronecker
    assembly, equal to the element loop)."""
    k = tri_k()
    wls = inputs.batch_2d(k, lambda dB: uniform_amplitude(BulkEnergy(k, Params.from_dB(dB))), count=64, seed=1)
    ps = [apfc.apfc_params_default(a1=0.5 * w.dB, rtol=1e-8, precision=apfc.APFC_MIXED,
                                   inner_kind=apfc.APFC_INNER_CHEB, restart=4,
                                   mass_kind=apfc.APFC_MASS_SEPARABLE, mass_iters=3, diff_iters=3, x0_order=3)
          for w in wls]
    s = apfc.Solver([apfc.make_mesh(2, w.mesh.n, w.mesh.length) for w in wls],
                    apfc.apfc_lattice_default(apfc.APFC_TRI2D), ps)
    s.autotune()
    ets = [to_dev(w.eta0) for w in wls]
    zts = [torch.zeros_like(e) for e in ets]
    s.init_zeta(ets, zts)
    for m in range(2):
        eta_in = [from_dev(e) for e in ets]
        info = s.step(ets, zts, wls[0].dt)
    for b, w in enumerate(wls):
        o = Oracle(Grid(2, w.mesh.n[:2], w.mesh.length[:2]), k, Params.from_dB(w.dB), assembly="kron")
        worst = _certify(o, w.dt, eta_in[b], from_dev(ets[b]), from_dev(zts[b]))
        print("instance", b, "n", w.mesh.n[0], "relres (oracle)", worst, flush=True)
        assert worst <= 1.01e-8, b
    assert info["max_relres"] <= 1e-8
