"""Differentiation through APFC time steps: torch.autograd.Function wrappers around the HIP
library's one-step adjoint (apfc_step_adjoint) and energy gradient (apfc_energy_grad), with
checkpoint-and-recompute across steps.

Amplitudes are float64 CUDA tensors of shape (J, 2, N) (real planar), so PyTorch's gradient of a
real loss with respect to them is (dL/dRe, dL/dIm) -- the convention the library uses.
Delta B (= 2 a1) is a 0-d float64 tensor; a context is built per distinct Delta B value.
"""
from __future__ import annotations

from typing import Dict, List, Optional, Tuple

import torch

from . import apfc


class SolverCache:
    """One apfc context per Delta B for a fixed mesh, lattice and solver setup."""

    def __init__(self, mesh: apfc.apfc_mesh, lattice: apfc.apfc_lattice, **params):
        self.mesh = mesh
        self.lattice = lattice
        self.params = params
        self._cache: Dict[float, apfc.Solver] = {}

    def get(self, dB: float) -> apfc.Solver:
        key = float(dB)
        if key not in self._cache:
            p = apfc.apfc_params_default(a1=0.5 * key, **self.params)
            self._cache[key] = apfc.Solver([self.mesh], self.lattice, [p])
        return self._cache[key]


def _forward_steps(solver: apfc.Solver, eta: torch.Tensor, zeta: torch.Tensor, dt: float, steps: int,
                   keep: bool) -> Tuple[torch.Tensor, torch.Tensor, List[torch.Tensor]]:
    # every segment starts a new trajectory for the extrapolated initial guess (x0_order > 0), so that the
    # backward pass recomputes a segment from the same initial guesses as the forward pass did
    solver.reset_history()
    e = eta.clone()
    z = zeta.clone()
    traj = [e.clone()] if keep else []
    for _ in range(steps):
        solver.step([e], [z], dt)
        if keep:
            traj.append(e.clone())
    return e, z, traj


class _Run(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eta0, dB, cache: SolverCache, dt: float, steps: int, every: int):
        solver = cache.get(float(dB))
        z0 = torch.zeros_like(eta0)
        solver.init_zeta([eta0.detach()], [z0])
        ckpts = []
        e, z = eta0.detach().clone(), z0
        done = 0
        while done < steps:
            ckpts.append((done, e.clone(), z.clone()))
            n = min(every, steps - done)
            e, z, _ = _forward_steps(solver, e, z, dt, n, keep=False)
            done += n
        ctx.cache, ctx.dt, ctx.dB = cache, dt, float(dB)
        ctx.ckpts = ckpts
        ctx.steps = steps
        return e

    @staticmethod
    def backward(ctx, grad_out):
        solver = ctx.cache.get(ctx.dB)
        lam = grad_out.detach().contiguous().clone()
        ddB = 0.0
        out = torch.empty_like(lam)
        for start, e0, z0 in reversed(ctx.ckpts):
            nxt = [c[0] for c in ctx.ckpts if c[0] > start]
            n = (nxt[0] - start) if nxt else ctx.steps - start
            _, _, traj = _forward_steps(solver, e0, z0, ctx.dt, n, keep=True)
            for m in range(n, 0, -1):
                ddB += solver.step_adjoint([traj[m - 1]], [traj[m]], ctx.dt, [lam], [out])[0]
                lam, out = out, lam
        g_dB = torch.tensor(ddB, dtype=torch.float64, device=grad_out.device)
        return lam, g_dB, None, None, None, None


def run(eta0: torch.Tensor, dB: torch.Tensor, cache: SolverCache, dt: float, steps: int,
        checkpoint_every: int = 10) -> torch.Tensor:
    """eta(T) after `steps` K=1 steps from eta0; differentiable in eta0 and dB.  Checkpoints of
    (eta, zeta) are kept every `checkpoint_every` steps and the steps in between recomputed during
    the backward pass."""
    return _Run.apply(eta0, dB, cache, float(dt), int(steps), int(checkpoint_every))


class _Energy(torch.autograd.Function):
    @staticmethod
    def forward(ctx, eta, dB, cache: SolverCache):
        solver = cache.get(float(dB))
        E = solver.energy([eta.detach()])[0]
        ctx.save_for_backward(eta.detach())
        ctx.cache, ctx.dB = cache, float(dB)
        return torch.tensor(E, dtype=torch.float64, device=eta.device)

    @staticmethod
    def backward(ctx, gE):
        (eta,) = ctx.saved_tensors
        solver = ctx.cache.get(ctx.dB)
        g = torch.empty_like(eta)
        ddB = solver.energy_grad([eta], [g])[0]
        return g * gE, torch.as_tensor(ddB, dtype=torch.float64, device=eta.device) * gE, None


def energy(eta: torch.Tensor, dB: torch.Tensor, cache: SolverCache) -> torch.Tensor:
    """E(eta) of Eq. (2) (without the 1/2), differentiable in eta and Delta B."""
    return _Energy.apply(eta, dB, cache)
