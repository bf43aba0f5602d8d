"""Gradients through several time steps (torch.autograd + checkpoint-recompute over the HIP adjoint)
against the CPU oracle's gradient and against central finite differences.  Needs an MI355X."""
import math

import numpy as np
import pytest

from oracle.apfc_oracle import Params, tri_k
from paper_1902_09761_amd import apfc, inputs
from tests.gpu_util import H_TRI, from_dev, oracle_for, phi_of, rel_l2, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _loss(eta_T, target, dB, cache, w):
    from paper_1902_09761_amd import autograd as ag
    return w * torch.sum((eta_T - target) ** 2) + ag.energy(eta_T, dB, cache)


def _oracle_loss_grad(mesh, eta0, target, dB, dt, steps):
    o = oracle_for(mesh, tri_k(), dB)
    traj = [eta0]
    for _ in range(steps):
        traj.append(o.step(traj[-1], dt)[1])
    eT = traj[-1]
    L = float(o.grid.w * np.sum(np.abs(eT - target) ** 2) + o.energy(eT))
    lam = 2.0 * o.grid.w * (eT - target) + o.energy_grad(eT)
    ddB = o.energy_ddB(eT)
    for m in range(steps, 0, -1):
        lam, dd = o.step_adjoint(traj[m - 1], traj[m], dt, lam)
        ddB += dd
    return L, lam, ddB


def test_autograd_checkpointed_gradient_matches_oracle():
    """24^2 two-grain case, 5 steps with a checkpoint every 2 steps: dL/d eta0 and dL/dDeltaB."""
    from paper_1902_09761_amd import autograd as ag
    n, dt, steps, dB = 24, 1.0, 5, 0.02
    wl = inputs.two_grains_2d(tri_k(), phi_of(tri_k()), n=n, seed=3, dB=dB)
    target = inputs.two_grains_2d(tri_k(), phi_of(tri_k()), n=n, seed=4, dB=0.03).eta0
    L_ref, g_ref, ddB_ref = _oracle_loss_grad(wl.mesh, wl.eta0, target, dB, dt, steps)

    cache = ag.SolverCache(apfc.make_mesh(2, wl.mesh.n, wl.mesh.length), apfc.apfc_lattice_default(apfc.APFC_TRI2D),
                           rtol=1e-13)
    eta0 = to_dev(wl.eta0).requires_grad_(True)
    dBt = torch.tensor(dB, dtype=torch.float64, device="cuda", requires_grad=True)
    etaT = ag.run(eta0, dBt, cache, dt, steps, checkpoint_every=2)
    L = _loss(etaT, to_dev(target), dBt, cache, wl.mesh.h ** 2)
    L.backward()
    assert abs(float(L.detach()) - L_ref) < 1e-10 * abs(L_ref)
    assert rel_l2(from_dev(eta0.grad), g_ref) < 1e-8
    assert abs(float(dBt.grad) - ddB_ref) < 1e-8 * abs(ddB_ref)


def test_checkpoint_cadence_gradient_matches_oracle():
    """The differentiation workload's recipe on a 64^2 mesh at its real cadence: 50 FP64 steps, a checkpoint
    every 10 steps, loss = w |eta(T) - target|^2 + E(eta(T)).  The oracle's gradient (direct solves and
    their conjugate transposes), the target (the oracle's run at Delta B = 0.03) and the loss are read from
    tests/golden/twograin64_gradient.npz, written by tests/golden/make_twograin_gradient.py."""
    import os
    from paper_1902_09761_amd import autograd as ag
    ref = np.load(os.path.join(os.path.dirname(__file__), "golden", "twograin64_gradient.npz"))
    n, dt, steps, dB = int(ref["n"]), float(ref["dt"]), int(ref["steps"]), float(ref["dB"])
    wl = inputs.two_grains_2d(tri_k(), phi_of(tri_k()), n=n, seed=int(ref["seed"]), dB=dB)
    cache = ag.SolverCache(apfc.make_mesh(2, wl.mesh.n, wl.mesh.length), apfc.apfc_lattice_default(apfc.APFC_TRI2D),
                           rtol=1e-13)
    eta0 = to_dev(wl.eta0).requires_grad_(True)
    dBt = torch.tensor(dB, dtype=torch.float64, device="cuda", requires_grad=True)
    etaT = ag.run(eta0, dBt, cache, dt, steps, checkpoint_every=10)
    L = _loss(etaT, to_dev(ref["target"]), dBt, cache, wl.mesh.h ** 2)
    L.backward()
    err_g = rel_l2(from_dev(eta0.grad), ref["grad_eta0"])
    err_d = abs(float(dBt.grad) - float(ref["grad_dB"])) / abs(float(ref["grad_dB"]))
    print("loss", float(L.detach()), "ref", float(ref["loss"]), "grad rel-L2", err_g, "dL/dDeltaB rel", err_d)
    assert abs(float(L.detach()) - float(ref["loss"])) < 1e-10 * abs(float(ref["loss"]))
    assert err_g < 1e-8
    assert err_d < 1e-8


def test_differentiation_workload_finite_differences():
    """256^2 two grains (+-4 degrees), 50 FP64 steps, checkpoint every 10; loss = |eta(T) - target|^2 + E(eta(T))
    with the target from a run at Delta B = 0.03.  Central differences (h = 1e-6) along Delta B and 3
    seeded directions in eta0 agree with the adjoint gradient to 1e-6."""
    from paper_1902_09761_amd import autograd as ag
    n, dt, steps, dB = 256, 1.0, 50, 0.02
    wl = inputs.two_grains_2d(tri_k(), phi_of(tri_k()), n=n, seed=1, dB=dB)
    mesh = apfc.make_mesh(2, wl.mesh.n, wl.mesh.length)
    lat = apfc.apfc_lattice_default(apfc.APFC_TRI2D)
    cache = ag.SolverCache(mesh, lat, rtol=1e-13)
    w = wl.mesh.h ** 2
    # target: seeded forward run at Delta B = 0.03
    with torch.no_grad():
        tgt = ag.run(to_dev(wl.eta0), torch.tensor(0.03, dtype=torch.float64, device="cuda"), cache, dt, steps, 10)

    def loss_value(e0, dBv):
        with torch.no_grad():
            dBt = torch.tensor(dBv, dtype=torch.float64, device="cuda")
            eT = ag.run(e0, dBt, cache, dt, steps, 10)
            return float(_loss(eT, tgt, dBt, cache, w))

    eta0 = to_dev(wl.eta0).requires_grad_(True)
    dBt = torch.tensor(dB, dtype=torch.float64, device="cuda", requires_grad=True)
    L = _loss(ag.run(eta0, dBt, cache, dt, steps, 10), tgt, dBt, cache, w)
    L.backward()
    g = eta0.grad.detach()
    eps = 1e-6
    fd = (loss_value(eta0.detach(), dB + eps) - loss_value(eta0.detach(), dB - eps)) / (2 * eps)
    print("dL/ddB adjoint", float(dBt.grad), "fd", fd)
    assert abs(fd - float(dBt.grad)) <= 1e-6 * abs(fd)
    gen = torch.Generator(device="cuda").manual_seed(7)
    for _ in range(3):
        v = torch.randn(eta0.shape, dtype=torch.float64, device="cuda", generator=gen)
        fd = (loss_value(eta0.detach() + eps * v, dB) - loss_value(eta0.detach() - eps * v, dB)) / (2 * eps)
        ad = float(torch.sum(g * v))
        print("directional adjoint", ad, "fd", fd)
        assert abs(fd - ad) <= 1e-6 * abs(fd)
