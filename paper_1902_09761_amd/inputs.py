"""Seeded synthetic initial states for the APFC workloads.

This module holds geometry and random numbers only: grain placement, lattice
rotation of the reciprocal vectors (rotated-crystal amplitudes, Eq. (13)),
Voronoi assignment and uniform noise.  It takes the reciprocal vectors k_j and
the relaxed amplitude phi from its caller and contains none of the solver's
arithmetic, so the CPU oracle and the HIP path can both be fed from it.

All arrays are numpy; amplitudes are returned as complex128 of shape (J, N)
with nodes in x-fastest lexicographic order on the periodic uniform grid
(node (ix, iy, iz) at position (ix*h, iy*h, iz*h), h = L/n).

Units: the triangular lattice spacing for |k|=1 is 4*pi/sqrt(3); the cubic
constant of the bcc lattice built from the unit <110> vectors is 2*pi*sqrt(2), that
of the fcc lattice built from the unit <111> vectors 2*pi*sqrt(3).

The relaxed amplitude phi is a number (every amplitude the same) or one value per
amplitude (lattices with several shells of |k_j|, such as fcc).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

TRI_SPACING = 4.0 * math.pi / math.sqrt(3.0)
BCC_SPACING = 2.0 * math.pi * math.sqrt(2.0)
FCC_SPACING = 2.0 * math.pi * math.sqrt(3.0)
NOISE_AMPLITUDE = 1e-3


@dataclasses.dataclass
class Mesh:
    """Periodic uniform Q1 mesh: n[d] nodes (= elements) per direction, side length[d]."""
    dim: int
    n: tuple
    length: tuple

    @property
    def N(self) -> int:
        return int(np.prod(self.n[: self.dim]))

    @property
    def h(self) -> float:
        return self.length[0] / self.n[0]


@dataclasses.dataclass
class Workload:
    name: str
    mesh: Mesh
    eta0: np.ndarray          # (J, N) complex128
    dB: float                 # Delta B = 2 a1
    dt: float
    steps: int
    rtol: float


def node_coords(mesh: Mesh) -> np.ndarray:
    """(N, dim) node coordinates, x fastest."""
    axes = [np.arange(mesh.n[d]) * (mesh.length[d] / mesh.n[d]) for d in range(mesh.dim)]
    grids = np.meshgrid(*axes[::-1], indexing="ij")          # slowest axis first
    return np.stack([g.reshape(-1) for g in grids[::-1]], axis=1)


def min_image(dr: np.ndarray, length: Sequence[float]) -> np.ndarray:
    L = np.asarray(length[: dr.shape[-1]], dtype=float)
    return dr - L * np.round(dr / L)


def rotation_matrix(dim: int, theta: float, axis=(0.0, 0.0, 1.0)) -> np.ndarray:
    """Counter-clockwise rotation by theta (2D) or about `axis` (3D, Rodrigues)."""
    c, s = math.cos(theta), math.sin(theta)
    if dim == 2:
        return np.array([[c, -s], [s, c]])
    a = np.asarray(axis, dtype=float)
    a = a / np.linalg.norm(a)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    return np.eye(3) + s * K + (1 - c) * (K @ K)


def delta_k(kvecs: np.ndarray, theta: float, axis=(0.0, 0.0, 1.0)) -> np.ndarray:
    """Reciprocal-vector change of a crystal rotated counter-clockwise by theta (Eq. (13))."""
    R = rotation_matrix(kvecs.shape[1], theta, axis)
    return kvecs @ R.T - kvecs


def amplitudes(phi, J: int) -> np.ndarray:
    """phi as a (J, 1) column: one number for every amplitude, or one value per amplitude."""
    a = np.asarray(phi, dtype=float).reshape(-1, 1)
    return np.broadcast_to(a, (J, 1)) if a.shape[0] == 1 else a


def rotated_grain(kvecs, phi, theta, centre, coords, length, axis=(0.0, 0.0, 1.0)):
    """eta_j = phi_j * exp(i dk_j . (r - c)), phase measured from the grain centre (minimum image)."""
    dr = min_image(coords - np.asarray(centre)[None, :], length)
    dk = delta_k(np.asarray(kvecs, float), theta, axis)
    return amplitudes(phi, len(kvecs)) * np.exp(1j * (dr @ dk.T)).T     # (J, N)


def add_noise(eta: np.ndarray, seed: int, amplitude: float = NOISE_AMPLITUDE) -> np.ndarray:
    """Independent U[-a, a] noise on Re and Im, drawn in the order (j, re/im, node)."""
    rng = np.random.default_rng(seed)
    J, N = eta.shape
    u = rng.uniform(-amplitude, amplitude, size=(J, 2, N))
    return eta + u[:, 0, :] + 1j * u[:, 1, :]


def single_grain(mesh: Mesh, kvecs, phi, theta, radius, centre=None, matrix="crystal",
                 axis=(0.0, 0.0, 1.0), seed: Optional[int] = None):
    """One rotated circular (2D) or spherical (3D) grain in an unrotated crystal or liquid matrix."""
    coords = node_coords(mesh)
    if centre is None:
        centre = [0.5 * mesh.length[d] for d in range(mesh.dim)]
    J = len(kvecs)
    grain = rotated_grain(kvecs, phi, theta, centre, coords, mesh.length, axis)
    if matrix == "crystal":
        eta = np.broadcast_to(amplitudes(phi, J), (J, mesh.N)).astype(np.complex128)
    else:
        eta = np.zeros((J, mesh.N), dtype=np.complex128)
    inside = np.linalg.norm(min_image(coords - np.asarray(centre)[None, :], mesh.length), axis=1) < radius
    eta[:, inside] = grain[:, inside]
    if seed is not None:
        eta = add_noise(eta, seed)
    return eta


def grains(mesh: Mesh, kvecs, phi, centres, thetas, radii, seed: Optional[int] = None,
           axis=(0.0, 0.0, 1.0)):
    """Several rotated grains of given radii in a liquid (eta = 0) background."""
    coords = node_coords(mesh)
    J = len(kvecs)
    eta = np.zeros((J, mesh.N), dtype=np.complex128)
    for c, th, R in zip(centres, thetas, radii):
        g = rotated_grain(kvecs, phi, th, c, coords, mesh.length, axis)
        inside = np.linalg.norm(min_image(coords - np.asarray(c)[None, :], mesh.length), axis=1) < R
        eta[:, inside] = g[:, inside]
    if seed is not None:
        eta = add_noise(eta, seed)
    return eta


def voronoi_polycrystal(mesh: Mesh, kvecs, phi, n_grains, max_theta_deg, seed: int):
    """Periodic Voronoi polycrystal: seeded centres U[0,L)^d, angles U[-max, max]."""
    rng = np.random.default_rng(seed + 1000)
    centres = rng.uniform(0.0, 1.0, size=(n_grains, mesh.dim)) * np.asarray(mesh.length[: mesh.dim])
    thetas = np.deg2rad(rng.uniform(-max_theta_deg, max_theta_deg, size=n_grains))
    coords = node_coords(mesh)
    J = len(kvecs)
    best = np.full(mesh.N, np.inf)
    owner = np.zeros(mesh.N, dtype=np.int64)
    for g in range(n_grains):
        dist = np.linalg.norm(min_image(coords - centres[g][None, :], mesh.length), axis=1)
        closer = dist < best
        best[closer] = dist[closer]
        owner[closer] = g
    eta = np.zeros((J, mesh.N), dtype=np.complex128)
    for g in range(n_grains):
        sel = owner == g
        eta[:, sel] = rotated_grain(kvecs, phi, thetas[g], centres[g], coords[sel], mesh.length)
    return add_noise(eta, seed)


# --------------------------------------------------------------------------------------
# The five workloads.  Each builder takes the lattice vectors and the relaxed amplitude
# (a callable dB -> phi) from its caller.
# --------------------------------------------------------------------------------------

def mesh2d(n: int, length: float) -> Mesh:
    return Mesh(2, (n, n, 1), (length, length, 1.0))


def mesh3d(n: int, length: float) -> Mesh:
    return Mesh(3, (n, n, n), (length, length, length))


def small_grain_2d(kvecs, phi_of_dB, n=64, seed=1, dB=0.02) -> Workload:
    """Triangular lattice, 64^2 periodic square of side 20 spacings, one grain of radius
    6 spacings rotated by 5 degrees in an unrotated matrix; dt=1, 10 steps, rtol 1e-10."""
    L = 20.0 * TRI_SPACING * (n / 64.0)
    mesh = mesh2d(n, L)
    eta = single_grain(mesh, kvecs, phi_of_dB(dB), math.radians(5.0), 6.0 * TRI_SPACING, seed=seed)
    return Workload("tri64_grain", mesh, eta, dB, 1.0, 10, 1e-10)


def voronoi_2d(kvecs, phi_of_dB, n=1024, seed=1, dB=0.02) -> Workload:
    """Triangular lattice, 1024^2 periodic square of side 400 spacings, 16 Voronoi grains
    rotated within +-10 degrees; dt=1, 100 steps, rtol 1e-8.  Smaller n keeps h fixed."""
    h = 400.0 * TRI_SPACING / 1024.0
    mesh = mesh2d(n, n * h)
    eta = voronoi_polycrystal(mesh, kvecs, phi_of_dB(dB), 16, 10.0, seed)
    return Workload(f"tri{n}_voronoi16", mesh, eta, dB, 1.0, 100, 1e-8)


BATCH_SIZES = (128, 192, 256, 384, 512)


def batch_2d(kvecs, phi_of_dB, count=64, seed=1, sizes=BATCH_SIZES) -> List[Workload]:
    """Independent triangular-lattice instances of seeded size n^2, n in `sizes`, each with
    one grain (radius L/4) rotated U[2,10] degrees and Delta B ~ U[0.01, 0.05]; h as the
    64^2 case; 50 steps, rtol 1e-8."""
    rng = np.random.default_rng(seed + 2000)
    h = 20.0 * TRI_SPACING / 64.0
    out = []
    for b in range(count):
        n = int(sizes[rng.integers(0, len(sizes))])
        theta = math.radians(rng.uniform(2.0, 10.0))
        dB = float(rng.uniform(0.01, 0.05))
        mesh = mesh2d(n, n * h)
        eta = single_grain(mesh, kvecs, phi_of_dB(dB), theta, 0.25 * n * h, seed=seed * 100 + b)
        out.append(Workload(f"tri{n}_inst{b}", mesh, eta, dB, 1.0, 50, 1e-8))
    return out


def sphere_3d(kvecs, phi_of_dB, n=128, seed=1, dB=0.02, spacing=BCC_SPACING, name="bcc") -> Workload:
    """Cubic lattice (bcc: unit <110> vectors; fcc with spacing=FCC_SPACING: the <111> and <200>
    shells), 128^3 periodic cube of side 60 cubic constants, spherical grain of radius 20 constants
    rotated 5 degrees about [001]; dt=1, 20 steps.  Smaller n keeps h fixed."""
    h = 60.0 * spacing / 128.0
    mesh = mesh3d(n, n * h)
    R = 20.0 * spacing * (n / 128.0)
    eta = single_grain(mesh, kvecs, phi_of_dB(dB), math.radians(5.0), R, seed=seed,
                       axis=(0.0, 0.0, 1.0))
    return Workload(f"{name}{n}_sphere", mesh, eta, dB, 1.0, 20, 1e-8)


def two_grains_2d(kvecs, phi_of_dB, n=256, seed=1, dB=0.02) -> Workload:
    """Triangular lattice, n^2 periodic square with h of the 64^2 case, two grains of radius
    0.2 L at (0.3L, 0.5L) rotated +4 degrees and (0.7L, 0.5L) rotated -4 degrees, in liquid;
    dt=1, 50 steps (the differentiation workload)."""
    h = 20.0 * TRI_SPACING / 64.0
    L = n * h
    mesh = mesh2d(n, L)
    eta = grains(mesh, kvecs, phi_of_dB(dB), [(0.3 * L, 0.5 * L), (0.7 * L, 0.5 * L)],
                 [math.radians(4.0), math.radians(-4.0)], [0.2 * L, 0.2 * L], seed=seed)
    return Workload(f"tri{n}_twograins", mesh, eta, dB, 1.0, 50, 1e-8)


def to_planar(eta: np.ndarray) -> np.ndarray:
    """(J, N) complex -> (J, 2, N) float64 [re, im] planar layout used by the C ABI."""
    return np.ascontiguousarray(np.stack([eta.real, eta.imag], axis=1))


def from_planar(x: np.ndarray) -> np.ndarray:
    return x[:, 0, :] + 1j * x[:, 1, :]
