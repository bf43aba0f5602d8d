"""Helpers shared by the GPU tests: seeded workloads, oracle runs, tensor conversion."""
import math

import numpy as np

from oracle.apfc_oracle import BulkEnergy, Grid, Oracle, Params, bcc_k, tri_k, uniform_amplitude
from paper_1902_09761_amd import inputs

H_TRI = 20.0 * inputs.TRI_SPACING / 64.0          # mesh size of the 64^2 grain workload


def phi_of(k):
    return lambda dB: uniform_amplitude(BulkEnergy(k, Params.from_dB(dB)))


def to_dev(eta):
    import torch
    return torch.tensor(inputs.to_planar(eta), dtype=torch.float64, device="cuda")


def from_dev(t):
    return inputs.from_planar(t.detach().cpu().numpy())


def oracle_for(mesh: inputs.Mesh, k, dB):
    g = Grid(mesh.dim, tuple(mesh.n[: mesh.dim]), tuple(mesh.length[: mesh.dim]))
    return Oracle(g, k, Params.from_dB(dB))


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def solver_for(meshes, kind, dBs, **kw):
    from paper_1902_09761_amd import apfc
    lat = apfc.apfc_lattice_default(kind)
    ms = [apfc.make_mesh(m.dim, m.n, m.length) for m in meshes]
    ps = [apfc.apfc_params_default(a1=0.5 * dB, **kw) for dB in dBs]
    return apfc.Solver(ms, lat, ps)


def eq_of(k):
    """dB -> relaxed amplitude of every amplitude (one value per shell of |k_j|; FCC has two)."""
    from oracle.apfc_oracle import equilibrium_amplitudes
    return lambda dB: equilibrium_amplitudes(BulkEnergy(k, Params.from_dB(dB)))
