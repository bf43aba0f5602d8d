"""Plain FP64 CPU oracle of the APFC time step -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the package smoke check and the benchmark's CPU-baseline leg
may import this module.  It shares no code with the HIP path: it assembles the
finite-element matrices element by element into scipy CSR and solves every block
system with a sparse direct factorisation (SuperLU).  It is deliberately slow and
obviously correct.

What it follows (Praetorius, Salvalaglio, Voigt, "An efficient numerical framework
for the amplitude expansion of the phase-field crystal model"):

* amplitude energy, Eq. (2); gradient flow, Eq. (3)-(4); bulk energy, Eq. (5);
  triangular lattice, Eq. (6)-(7); parameters a0..a3 of Sec. II;
* split weak form, Eq. (8)-(9); the matrices M, K, T, J, h of Sec. II.A
  (assembled here on a periodic uniform Q1 quad/hex mesh);
* backward Euler + simplified Newton with amplitude splitting, Algorithm 1 and the
  block system Eq. (10)/(11);
* the block preconditioner Eq. (12) and its four-step application (Sec. II.B),
  used only to pin the HIP preconditioner, never in the step itself.

Readings (where the paper is silent, garbled or self-contradictory):

R1  The RHS of the eta equation carries -kappa_j (Eq. (3)): J^j = kappa_j w diag(dF),
    h-vector = -kappa_j w h.  (Eq. (8)/(9) omit the factor.)
R2  Energy without the 1/2 of Eq. (2): E = int f^s + sum_j |G_j eta_j|^2, consistent
    with Eq. (4).
R3  The four preconditioner steps are implemented as printed; they invert the
    factorisation with +M^{-1}K in the upper factor (the printed -M^{-1}K would need
    a '+' in step 4).  Both give the same spectrum {1} u eig(S_P^{-1} S).
R4  dF_j is the Wirtinger derivative of F^s_j = d f^s / d eta_j^* with respect to
    eta_j at fixed eta_j^*; h_j = F^s_j - dF_j eta_j.
R5  K (Picard iterates) = 1 by default; all amplitudes use the previous iterate
    (Jacobi splitting).
R6  Nodal (trapezoidal) quadrature for every integral of the bulk energy and its
    derivatives: weight w = h^dim per node.
R7  Matrix entries [(a phi_i, phi_l)]: row = test function i, column = trial l.
R8  The block system is solved with eta^{m-1} (not eta^m) in the RHS.
R9  Periodic boundary conditions; zeta^0 = M^{-1} G eta^0.
R10 bcc lattice: k_j = the six unit <110>/sqrt(2) vectors; f^s is the zero-wave-vector
    part of (a1/a0) n^2 - a3/(3 a0) n^3 + a2/(3 a0) n^4 with n from Eq. (1).  For the
    triangular lattice this reproduces Eq. (5)-(6) exactly.
R16 FCC lattice (J = 7; the paper takes its vectors and bulk polynomial from another work): the
    first two shells of the fcc reciprocal lattice, four <111>/sqrt 3 vectors (one of each +- pair,
    chosen to sum to zero, |k| = 1) and three <200>/sqrt 3 vectors (|k| = 2/sqrt 3); f^s by the same
    enumeration as R10.
R17 Multigrid inner solve (the paper uses one algebraic V-cycle from a library): a geometric V-cycle on
    the structured mesh, coarse operators by rediscretisation (equal to the Galerkin products), symmetric
    Chebyshev-Jacobi smoothing; see MultigridL.
R18 Separable mass inverse (an alternative to the paper's iterative inner solve of step 1 of P^{-1}): on
    the uniform periodic mesh M is the Kronecker product of 1D mass matrices, so M^{-1} is the Kronecker
    product of their inverses, whose entries decay geometrically; truncated to R neighbours per
    direction; see separable_mass_inverse.
"""
from __future__ import annotations

import dataclasses
import itertools
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


# ---------------------------------------------------------------------------------------
# Parameters and lattices (Sec. II, Eq. (7); R10)
# ---------------------------------------------------------------------------------------

@dataclasses.dataclass
class Params:
    a0: float = 0.98
    a1: float = 0.01
    a2: float = 0.25
    a3: float = 0.5

    @staticmethod
    def from_dB(dB: float, a0=0.98, a2=0.25, a3=0.5) -> "Params":
        """Elder's Delta B maps to a1 = Delta B / 2 (B^x -> a0, 3v/4 -> a2, tau -> a3)."""
        return Params(a0=a0, a1=0.5 * dB, a2=a2, a3=a3)


def tri_k() -> np.ndarray:
    """Triangular reciprocal vectors, Eq. (7)."""
    s = math.sqrt(3.0) / 2.0
    return np.array([[-s, -0.5], [0.0, 1.0], [s, -0.5]])


def bcc_k() -> np.ndarray:
    """bcc reciprocal vectors (R10): one of each +-<110>/sqrt(2) pair."""
    v = np.array([[1, 1, 0], [1, -1, 0], [1, 0, 1], [1, 0, -1], [0, 1, 1], [0, 1, -1]], float)
    return v / math.sqrt(2.0)


def fcc_k() -> np.ndarray:
    """FCC reciprocal vectors (R16): <111>/sqrt 3 (summing to zero) and <200>/sqrt 3."""
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1], [2, 0, 0], [0, 2, 0], [0, 0, 2]], float)
    return v / math.sqrt(3.0)


def kappas(k: np.ndarray, p: Params) -> np.ndarray:
    """Mobility kappa_j = a0 |k_j|^2 (below Eq. (3))."""
    return p.a0 * np.sum(k * k, axis=1)


# ---------------------------------------------------------------------------------------
# Bulk energy polynomial (Eq. (1), (5), (6); R4, R10)
# ---------------------------------------------------------------------------------------

class BulkEnergy:
    """f^s as a polynomial in the 2J variables (eta_1..eta_J, eta_1^*..eta_J^*).

    Built by enumerating every ordered product of p factors of
    n = sum_j (eta_j e^{i k_j.r} + eta_j^* e^{-i k_j.r}) whose wave vectors sum to zero
    (the part of n^p that survives averaging over the fast lattice scale).
    """

    def __init__(self, k: np.ndarray, p: Params):
        self.k = np.asarray(k, float)
        self.J = J = len(k)
        self.p = p
        coef = {2: p.a1 / p.a0, 3: -p.a3 / (3.0 * p.a0), 4: p.a2 / (3.0 * p.a0)}
        self.terms: Dict[Tuple[int, ...], float] = {}
        for order, c in coef.items():
            for tup in itertools.product(range(2 * J), repeat=order):
                q = np.zeros(self.k.shape[1])
                for t in tup:
                    q += self.k[t % J] if t < J else -self.k[t % J]
                if np.max(np.abs(q)) < 1e-12:
                    e = [0] * (2 * J)
                    for t in tup:
                        e[t] += 1
                    e = tuple(e)
                    self.terms[e] = self.terms.get(e, 0.0) + c

    @staticmethod
    def _eval(terms, u):
        out = np.zeros(u.shape[1], dtype=np.complex128)
        for e, c in terms.items():
            t = np.full(u.shape[1], c, dtype=np.complex128)
            for v, m in enumerate(e):
                if m:
                    t = t * u[v] ** m
            out += t
        return out

    @staticmethod
    def _diff(terms, var):
        out = {}
        for e, c in terms.items():
            if e[var] > 0:
                e2 = list(e)
                e2[var] -= 1
                e2 = tuple(e2)
                out[e2] = out.get(e2, 0.0) + c * e[var]
        return out

    def _u(self, eta):
        return np.concatenate([eta, np.conj(eta)], axis=0)

    def f(self, eta: np.ndarray) -> np.ndarray:
        """Bulk energy density at every node (real)."""
        v = self._eval(self.terms, self._u(eta))
        assert np.max(np.abs(v.imag)) <= 1e-12 * max(1.0, np.max(np.abs(v.real)))
        return v.real

    def F(self, eta: np.ndarray) -> np.ndarray:
        """F^s_j = d f^s / d eta_j^*, shape (J, N)."""
        u = self._u(eta)
        return np.stack([self._eval(self._diff(self.terms, self.J + j), u) for j in range(self.J)])

    def dF(self, eta: np.ndarray) -> np.ndarray:
        """dF_j = d F^s_j / d eta_j (R4), shape (J, N)."""
        u = self._u(eta)
        return np.stack([self._eval(self._diff(self._diff(self.terms, self.J + j), j), u)
                         for j in range(self.J)])

    def h(self, eta: np.ndarray) -> np.ndarray:
        """h_j = F^s_j - dF_j eta_j (the explicit part of the linearised bulk force)."""
        return self.F(eta) - self.dF(eta) * eta

    def h_derivs(self, eta: np.ndarray):
        """Wirtinger derivatives of h_j: P[j,l] = dh_j/d eta_l, Q[j,l] = dh_j/d eta_l^*."""
        J = self.J
        u = self._u(eta)
        Fj = [self._diff(self.terms, J + j) for j in range(J)]
        dFj = [self._diff(Fj[j], j) for j in range(J)]
        dFv = [self._eval(dFj[j], u) for j in range(J)]
        P = np.zeros((J, J) + eta.shape[1:], dtype=np.complex128)
        Q = np.zeros_like(P)
        for j in range(J):
            for l in range(J):
                # h_j = F_j - dF_j * eta_j
                P[j, l] = self._eval(self._diff(Fj[j], l), u) - self._eval(self._diff(dFj[j], l), u) * eta[j]
                Q[j, l] = self._eval(self._diff(Fj[j], J + l), u) - self._eval(self._diff(dFj[j], J + l), u) * eta[j]
                if l == j:
                    P[j, l] -= dFv[j]
        return P, Q


def tri_bulk_closed_form(eta: np.ndarray, p: Params) -> np.ndarray:
    """Eq. (5)-(6) written out for the triangular lattice (J = 3)."""
    A = 2.0 * np.sum(np.abs(eta) ** 2, axis=0)
    g = -2.0 * p.a3 / p.a0 * (eta[0] * eta[1] * eta[2] + np.conj(eta[0] * eta[1] * eta[2]))
    return (p.a1 / p.a0 * A + p.a2 / p.a0 * (A ** 2 - 2.0 * np.sum(np.abs(eta) ** 4, axis=0)) + g).real


def uniform_amplitude(bulk: BulkEnergy) -> float:
    """Relaxed amplitude phi of the uniform crystal (all eta_j = phi real): the positive
    root of d f^s(phi)/d phi = 0 with f^s(phi) = c2 phi^2 + c3 phi^3 + c4 phi^4."""
    c = {2: 0.0, 3: 0.0, 4: 0.0}
    for e, v in bulk.terms.items():
        c[sum(e)] += v
    disc = 9.0 * c[3] ** 2 - 32.0 * c[2] * c[4]
    if disc < 0:
        return 0.0
    return (-3.0 * c[3] + math.sqrt(disc)) / (8.0 * c[4])


def equilibrium_amplitudes(bulk: BulkEnergy) -> np.ndarray:
    """Relaxed real amplitudes of the uniform crystal, one value per shell of equal |k_j| (the
    amplitudes of one shell are equivalent under the lattice's point group): a stationary point of
    f^s(phi_shell(j)) with every phi > 0, found by Newton's method on the shell gradient
    d f / d phi_s = sum_{j in s} 2 Re F^s_j, started from the single-shell root (a library root finder
    on the oracle's own polynomial).  One shell (triangular, bcc): uniform_amplitude.  Zeros when the
    single-shell root is the liquid."""
    import scipy.optimize
    k2 = np.round(np.sum(bulk.k * bulk.k, axis=1), 12)
    shells = sorted(set(k2.tolist()))
    phi0 = uniform_amplitude(bulk)
    if len(shells) == 1 or phi0 == 0.0:
        return np.full(bulk.J, phi0)
    which = np.array([shells.index(v) for v in k2])

    def grad(x):
        eta = x[which].astype(np.complex128)[:, None]
        F = bulk.F(eta)[:, 0]
        return np.array([2.0 * np.sum(F[which == s].real) for s in range(len(shells))])

    sol = scipy.optimize.root(grad, np.full(len(shells), phi0), method="hybr", tol=1e-13)
    assert np.max(np.abs(sol.fun)) < 1e-15 and np.all(sol.x > 0.0), sol
    return sol.x[which]


# ---------------------------------------------------------------------------------------
# Periodic uniform Q1 mesh and element-by-element assembly (Sec. II.A; R6, R7)
# ---------------------------------------------------------------------------------------

@dataclasses.dataclass
class Grid:
    dim: int
    n: Tuple[int, ...]          # nodes (= elements) per direction
    length: Tuple[float, ...]

    @property
    def N(self) -> int:
        return int(np.prod(self.n[: self.dim]))

    @property
    def h(self) -> float:
        return self.length[0] / self.n[0]

    @property
    def w(self) -> float:
        """Nodal quadrature weight (R6)."""
        return self.h ** self.dim

    def node(self, idx: Sequence[np.ndarray]) -> np.ndarray:
        """Global index of node (ix, iy[, iz]) with periodic wrap, x fastest."""
        g = np.zeros_like(idx[0])
        stride = 1
        for d in range(self.dim):
            g = g + (idx[d] % self.n[d]) * stride
            stride *= self.n[d]
        return g


def element_matrices(dim: int, h: float, kvec: np.ndarray):
    """Q1 element matrices on [0,h]^dim by 2-point Gauss per direction (exact here).

    Me[a,b] = int phi_a phi_b, Ke[a,b] = int grad phi_a . grad phi_b,
    Te[a,b] = int (2 k . grad phi_b) phi_a   (row a = test, column b = trial).
    Local node a has corner bits (a_x, a_y[, a_z]) with x fastest.
    """
    gp = np.array([0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0)]) * h
    gw = np.array([0.5, 0.5]) * h
    nloc = 2 ** dim
    corners = [[(a >> d) & 1 for d in range(dim)] for a in range(nloc)]

    def psi(bit, s):
        return s / h if bit else 1.0 - s / h

    def dpsi(bit):
        return 1.0 / h if bit else -1.0 / h

    Me = np.zeros((nloc, nloc))
    Ke = np.zeros((nloc, nloc))
    Te = np.zeros((nloc, nloc))
    for gidx in itertools.product(range(2), repeat=dim):
        x = [gp[i] for i in gidx]
        W = np.prod([gw[i] for i in gidx])
        val = np.array([np.prod([psi(c[d], x[d]) for d in range(dim)]) for c in corners])
        grad = np.array([[dpsi(c[d]) * np.prod([psi(c[e], x[e]) for e in range(dim) if e != d])
                          for d in range(dim)] for c in corners])
        Me += W * np.outer(val, val)
        Ke += W * grad @ grad.T
        Te += W * np.outer(val, 2.0 * grad @ kvec[:dim])
    return Me, Ke, Te, corners


def assemble(grid: Grid, kvecs: np.ndarray):
    """Global CSR matrices M, K and T_j (one per reciprocal vector), element by element."""
    dim = grid.dim
    origins = np.meshgrid(*[np.arange(grid.n[d]) for d in range(dim)], indexing="ij")
    origins = [o.reshape(-1) for o in origins]
    Me, Ke, _, corners = element_matrices(dim, grid.h, np.zeros(dim))
    glob = np.stack([grid.node([origins[d] + c[d] for d in range(dim)]) for c in corners])   # (nloc, nelem)
    nloc = len(corners)
    rows = np.repeat(glob, nloc, axis=0)            # (nloc*nloc, nelem): row a repeated per b
    cols = np.tile(glob, (nloc, 1))
    N = grid.N

    def build(E):
        vals = np.repeat(E.reshape(-1)[:, None], glob.shape[1], axis=1)
        return sp.csr_matrix((vals.reshape(-1), (rows.reshape(-1), cols.reshape(-1))), shape=(N, N))

    M = build(Me)
    K = build(Ke)
    T = []
    for kv in kvecs:
        _, _, Te, _ = element_matrices(dim, grid.h, np.asarray(kv, float))
        T.append(build(Te))
    return M, K, T


def kron_matrices(grid: Grid, kvecs: np.ndarray):
    """The same matrices from 1D periodic stencils and Kronecker products (for pinning the
    element loop): m = h/6 [1 4 1], k = 1/h [-1 2 -1], d = 1/2 [-1 0 1]."""
    def circ(n, lo, mid, hi):
        A = sp.diags([np.full(n, mid), np.full(n - 1, hi), np.full(n - 1, lo)], [0, 1, -1], format="lil")
        A[0, n - 1] += lo
        A[n - 1, 0] += hi
        return A.tocsr()
    h = grid.h
    m1 = [circ(grid.n[d], h / 6, 4 * h / 6, h / 6) for d in range(grid.dim)]
    k1 = [circ(grid.n[d], -1 / h, 2 / h, -1 / h) for d in range(grid.dim)]
    d1 = [circ(grid.n[d], -0.5, 0.0, 0.5) for d in range(grid.dim)]

    def kron_dirs(ops):           # ops[d] acts in direction d; x fastest => kron(z, y, x)
        out = ops[grid.dim - 1]
        for d in range(grid.dim - 2, -1, -1):
            out = sp.kron(out, ops[d], format="csr")
        return out
    M = kron_dirs(m1)
    K = sum(kron_dirs([k1[e] if e == d else m1[e] for e in range(grid.dim)]) for d in range(grid.dim))
    T = []
    for kv in kvecs:
        T.append(sum(2.0 * kv[d] * kron_dirs([d1[e] if e == d else m1[e] for e in range(grid.dim)])
                     for d in range(grid.dim)))
    return M, K, T


# ---------------------------------------------------------------------------------------
# The time step (Algorithm 1, Eq. (10)/(11); R1, R5, R6, R8)
# ---------------------------------------------------------------------------------------

class Oracle:
    def __init__(self, grid: Grid, kvecs: np.ndarray, params: Params, assembly: str = "element"):
        """assembly = "element" (element loop, the default) or "kron" (the same matrices from 1D
        stencils, pinned equal to the element loop; for meshes too large for the element loop)."""
        self.grid = grid
        self.k = np.asarray(kvecs, float)
        self.J = len(self.k)
        self.params = params
        self.kappa = kappas(self.k, params)
        self.bulk = BulkEnergy(self.k, params)
        if assembly == "kron":
            self.M, self.K, self.T = kron_matrices(grid, self.k)
        else:
            self.M, self.K, self.T = assemble(grid, self.k)
        self.G = [(-self.K + 1j * Tj).tocsr() for Tj in self.T]
        self._Mlu = None

    # -- nodal nonlinearity ------------------------------------------------------------
    def nodal(self, eta):
        """d (real, (N,)) and h (J, N) of the simplified Newton linearisation (R4)."""
        dF = self.bulk.dF(eta)
        assert np.allclose(dF.imag, 0.0, atol=1e-13) and np.allclose(dF, dF[0:1], atol=1e-13)
        return dF[0].real, self.bulk.h(eta)

    def block_matrix(self, j: int, d: np.ndarray, dt: float):
        """A_j = [[M, -G_j], [kappa_j G_j, M/dt + kappa_j w diag(d)]] (Eq. (11); R1, R6)."""
        w = self.grid.w
        kap = self.kappa[j]
        B = (self.M / dt + kap * w * sp.diags(d)).astype(np.complex128)
        return sp.bmat([[self.M.astype(np.complex128), -self.G[j]], [kap * self.G[j], B]], format="csc")

    def apply_block(self, j: int, d: np.ndarray, dt: float, zeta_j, eta_j):
        """A_j [zeta_j; eta_j] block by block (Eq. (11)), without forming the 2N x 2N matrix:
        (M zeta - G eta, kappa G zeta + M eta/dt + kappa w d eta)."""
        kap, w = self.kappa[j], self.grid.w
        y1 = self.M @ zeta_j - self.G[j] @ eta_j
        y2 = kap * (self.G[j] @ zeta_j) + self.M @ eta_j / dt + (kap * w) * d * eta_j
        return y1, y2

    def rhs(self, j: int, eta_prev_j, h_j, dt: float, source_j=None):
        """b_j = [0 ; M eta_j^{m-1}/dt - kappa_j w h_j (+ M s_j)] (R1, R8)."""
        b2 = self.M @ eta_prev_j / dt - self.kappa[j] * self.grid.w * h_j
        if source_j is not None:
            b2 = b2 + self.M @ source_j
        return np.concatenate([np.zeros(self.grid.N, np.complex128), b2])

    def step(self, eta: np.ndarray, dt: float, picard: int = 1, source=None):
        """One time step of Algorithm 1: returns (zeta^m, eta^m), each (J, N) complex."""
        N = self.grid.N
        it = eta.copy()
        zeta = np.zeros_like(eta)
        for _ in range(picard):
            d, h = self.nodal(it)
            new = np.zeros_like(eta)
            for j in range(self.J):
                A = self.block_matrix(j, d, dt)
                b = self.rhs(j, eta[j], h[j], dt, None if source is None else source[j])
                x = spla.splu(A).solve(b)
                zeta[j], new[j] = x[:N], x[N:]
            it = new
        return zeta, it

    def run(self, eta, dt, steps, picard=1):
        for _ in range(steps):
            _, eta = self.step(eta, dt, picard)
        return eta

    # -- energy (Eq. (2) with R2, R6) -----------------------------------------------------
    def mass_solve(self, b):
        if self._Mlu is None:
            self._Mlu = spla.splu(self.M.tocsc().astype(np.complex128))
        return self._Mlu.solve(b)

    def zeta_of(self, eta):
        """zeta_j = M^{-1} G_j eta_j (R9)."""
        return np.stack([self.mass_solve(self.G[j] @ eta[j]) for j in range(self.J)])

    def energy(self, eta) -> float:
        zeta = self.zeta_of(eta)
        grad_part = sum(np.vdot(zeta[j], self.M @ zeta[j]).real for j in range(self.J))
        return float(self.grid.w * np.sum(self.bulk.f(eta)) + grad_part)

    def energy_grad(self, eta):
        """Gradient of E in torch's convention (dE/dRe + i dE/dIm = 2 dE/d eta^*)."""
        zeta = self.zeta_of(eta)
        F = self.bulk.F(eta)
        return np.stack([2.0 * (self.grid.w * F[j] + self.G[j] @ zeta[j]) for j in range(self.J)])

    def energy_ddB(self, eta) -> float:
        """dE/d(Delta B) at fixed eta: f^s contains (a1/a0) A with a1 = Delta B/2."""
        A = 2.0 * np.sum(np.abs(eta) ** 2, axis=0)
        return float(self.grid.w * np.sum(A) / (2.0 * self.params.a0))

    # -- adjoint of one step (K = 1) ----------------------------------------------------
    def step_adjoint(self, eta_prev, eta_new, dt, lam_new):
        """Given lam_new = dL/d eta^m (torch convention), return (dL/d eta^{m-1}, dL/dDeltaB)
        for L depending on eta^{m-1} only through one K = 1 step.

        eta^m_j = E A_j(d(eta^{m-1}))^{-1} b_j(eta^{m-1}); the solve is adjoined with a direct
        conjugate-transpose solve; the nodal maps are real-linear (adjoint P^H mu + Q^T mu^*).
        """
        N, J, w = self.grid.N, self.J, self.grid.w
        d, _ = self.nodal(eta_prev)
        P, Q = self.bulk.h_derivs(eta_prev)
        grad = np.zeros_like(eta_prev)
        C = np.zeros(N)
        for j in range(J):
            A = self.block_matrix(j, d, dt)
            mu = spla.splu(A).solve(np.concatenate([np.zeros(N, np.complex128), lam_new[j]]), trans="H")
            mu_eta = mu[N:]
            grad[j] += self.M @ mu_eta / dt
            for l in range(J):
                # contribution of -kappa_j w h_j(eta) to b_j
                grad[l] += -self.kappa[j] * w * (np.conj(P[j, l]) * mu_eta + Q[j, l] * np.conj(mu_eta))
            # contribution of kappa_j w diag(d) eta^m_j in A_j
            C += self.kappa[j] * w * np.real(np.conj(mu_eta) * eta_new[j])
        p = self.params
        # d = 2 a1/a0 + 4 (a2/a0) A, A = 2 sum |eta|^2: dd = 16 a2/a0 Re(eta^* deta)
        for l in range(J):
            grad[l] += -16.0 * p.a2 / p.a0 * C * eta_prev[l]
        ddB = float(-np.sum(C) / p.a0)      # dd/dDeltaB = 1/a0
        return grad, ddB

    # -- preconditioner of Eq. (12), four steps (R3) ------------------------------------
    def jacobi_bounds(self, j, dt):
        """Exact extremes of the spectra of D^{-1} M and D^{-1} L (L = M/sqrt(dt) + sqrt(kappa_j) K)
        on the periodic uniform mesh: the symbols are multilinear in cos(theta_d), so the extremes
        are attained at theta_d in {0, pi} (whether or not those modes exist on the mesh)."""
        g = self.grid
        kap = self.kappa[j]
        DM = self.M.diagonal()[0]
        DL = (self.M / math.sqrt(dt) + math.sqrt(kap) * self.K).diagonal()[0]
        lm, ll = [], []
        for corner in itertools.product((0.0, math.pi), repeat=g.dim):
            Mh, Kh, _ = symbols_at(g, np.zeros(g.dim), corner)
            lm.append(Mh / DM)
            ll.append((Mh / math.sqrt(dt) + math.sqrt(kap) * Kh) / DL)
        return (min(lm), max(lm)), (min(ll), max(ll))

    def precond_apply(self, j, beta1, beta2, dt, inner=None, mass_iters=3, diff_iters=5, mg_options=None,
                      mass="iter"):
        """x = P^{-1} b by the four steps; inner=None uses exact (direct) inner solves,
        inner='pcg' uses fixed-count Jacobi-preconditioned CG from a zero start, inner='cheb'
        fixed-count Chebyshev iteration with the exact Jacobi spectral bounds, inner='mg' one multigrid
        V-cycle for each L solve (MultigridL with mg_options) and Chebyshev for the mass solve.
        mass='sep' replaces the mass solve of step 1 by the separable inverse with R = mass_iters
        neighbours per direction (R18)."""
        kap = self.kappa[j]
        L = (self.M / math.sqrt(dt) + math.sqrt(kap) * self.K).tocsc()
        if inner is None:
            solve_M = lambda b: spla.spsolve(self.M.tocsc().astype(complex), b)
            solve_L = lambda b: spla.spsolve(L.astype(complex), b)
        elif inner == "pcg":
            solve_M = lambda b: jacobi_pcg(self.M, b, mass_iters)
            solve_L = lambda b: jacobi_pcg(L, b, diff_iters)
        elif inner == "mg":
            bm, _ = self.jacobi_bounds(j, dt)
            mg = MultigridL(self.grid, kap, dt, **(mg_options or {}))
            solve_M = lambda b: chebyshev(self.M, b, mass_iters, *bm)
            solve_L = lambda b: mg.cycle(b)
        else:
            bm, bl = self.jacobi_bounds(j, dt)
            solve_M = lambda b: chebyshev(self.M, b, mass_iters, *bm)
            solve_L = lambda b: chebyshev(L.tocsr(), b, diff_iters, *bl)
        if mass == "sep":
            W = separable_mass_inverse(self.grid, mass_iters)
            solve_M = lambda b: W @ b
        b1p = solve_M(beta1)                                   # step 1
        b2p = solve_L(beta2 - kap * (self.G[j] @ b1p))         # step 2
        chi2 = solve_L(self.M @ b2p)                           # step 3
        chi1 = b1p - (b2p - chi2 / math.sqrt(dt)) / math.sqrt(kap)   # step 4
        return chi1, chi2

    def precond_matrix(self, j, dt):
        """P with the upper factor [[I, +M^{-1}K], [0, M^{-1} L]] that the four steps invert
        (R3), as a dense matrix (small meshes only)."""
        kap = self.kappa[j]
        M = self.M.toarray()
        K = self.K.toarray()
        G = self.G[j].toarray()
        L = M / math.sqrt(dt) + math.sqrt(kap) * K
        N = M.shape[0]
        lower = np.block([[M, np.zeros((N, N))], [kap * G, L]])
        Minv = np.linalg.inv(M)
        upper = np.block([[np.eye(N), Minv @ K], [np.zeros((N, N)), Minv @ L]])
        return lower @ upper


# ---------------------------------------------------------------------------------------
# Separable approximate inverse of the mass matrix (R18)
# ---------------------------------------------------------------------------------------

def separable_mass_inverse(grid: Grid, R: int) -> sp.csr_matrix:
    """W ~ M^{-1} for step 1 of P^{-1} (R18).

    The 1D linear-element mass matrix on a uniform mesh is (h/6) tridiag(1, 4, 1).  On an unbounded
    line its inverse is the Toeplitz matrix with entries (sqrt(3)/h) rho^|i-l|, where rho = sqrt(3) - 2
    is the root of modulus below one of rho^2 + 4 rho + 1 = 0 (the recurrence the rows of the inverse
    satisfy away from the diagonal; the diagonal row fixes the factor: (h/6)(4 + 2 rho) sqrt(3)/h = 1).
    The Q1 mass matrix of the uniform quad/hex mesh is the Kronecker product of the 1D mass matrices of
    the directions, so W = kron of the 1D operators, each truncated to |i - l| <= R and wrapped
    periodically (taps that land on the same node add up)."""
    rho = math.sqrt(3.0) - 2.0
    c = math.sqrt(3.0) / grid.h

    def one(n):
        rows, cols, vals = [], [], []
        for i in range(n):
            for k in range(-R, R + 1):
                rows.append(i)
                cols.append((i + k) % n)
                vals.append(c * rho ** abs(k))
        return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))   # duplicates are summed

    W = one(grid.n[0])
    for d in range(1, grid.dim):                 # x fastest: kron(z, y, x)
        W = sp.kron(one(grid.n[d]), W)
    return W.tocsr()


# ---------------------------------------------------------------------------------------
# Multigrid V-cycle for the diffusion operator L (the multigrid inner solve of Sec. III; R17)
# ---------------------------------------------------------------------------------------

def coarse_grid(g: Grid) -> Grid:
    """The grid of twice the mesh size on the same periodic domain (n even in every direction)."""
    return Grid(g.dim, tuple(v // 2 for v in g.n[: g.dim]), tuple(g.length[: g.dim]))


def interpolation(gc: Grid) -> sp.csr_matrix:
    """Prolongation from the coarse grid gc to the grid of half its mesh size: the Q1 interpolant, i.e.
    the embedding of the coarse finite-element space in the fine one.  Per direction fine node 2i takes
    coarse node i and fine node 2i + 1 the mean of coarse nodes i and i + 1 (periodic); tensor product,
    x fastest.  Restriction is its transpose."""
    def one(nc):
        rows, cols, vals = [], [], []
        for i in range(nc):
            rows += [2 * i, 2 * i + 1, 2 * i + 1]
            cols += [i, i, (i + 1) % nc]
            vals += [1.0, 0.5, 0.5]
        return sp.csr_matrix((vals, (rows, cols)), shape=(2 * nc, nc))
    ops = [one(n) for n in gc.n[: gc.dim]]
    out = ops[gc.dim - 1]
    for d in range(gc.dim - 2, -1, -1):
        out = sp.kron(out, ops[d], format="csr")
    return out


class MultigridL:
    """One V-cycle, from a zero initial guess, for L = M/sqrt(dt) + sqrt(kappa) K (R17).

    Levels: the fine grid, then coarser grids of twice the mesh size while every n is even and n/2 >=
    coarse_min (and at most max_levels levels in all).  Each level's L is the finite-element L assembled on that level's grid, which equals the
    Galerkin product P^T L P for the Q1 interpolation P (nested spaces; pinned by a test).  Smoother:
    nu Chebyshev-Jacobi iterations for the upper part [lam_max/alpha, lam_max] of the spectrum of D^{-1}L
    (lam_max exact from the symbol), the same polynomial before and after the coarse-grid correction, so
    the cycle is symmetric.  Coarsest level: coarse_iters Chebyshev-Jacobi iterations over the whole
    spectrum [lam_min, lam_max].  The cycle:
      x = S(b);  r = b - L x;  x += P V(P^T r);  x += S(b - L x)."""

    def __init__(self, grid: Grid, kappa: float, dt: float, nu: int = 2, alpha: float = 4.0,
                 coarse_min: int = 16, coarse_iters: int = 24, max_levels: Optional[int] = None):
        self.nu, self.alpha, self.coarse_iters = nu, alpha, coarse_iters
        self.levels = []
        g = grid
        while True:
            M, K, _ = assemble(g, np.zeros((0, g.dim)))
            L = (M / math.sqrt(dt) + math.sqrt(kappa) * K).tocsr()
            lam = []
            D = L.diagonal()[0]
            for corner in itertools.product((0.0, math.pi), repeat=g.dim):
                Mh, Kh, _ = symbols_at(g, np.zeros(g.dim), corner)
                lam.append((Mh / math.sqrt(dt) + math.sqrt(kappa) * Kh) / D)
            self.levels.append({"grid": g, "L": L, "lam": (min(lam), max(lam))})
            more = max_levels is None or len(self.levels) < max_levels
            if more and all(v % 2 == 0 and v // 2 >= coarse_min for v in g.n[: g.dim]):
                gc = coarse_grid(g)
                self.levels[-1]["P"] = interpolation(gc)
                g = gc
            else:
                break

    def smooth(self, lev, b):
        lo, hi = lev["lam"]
        return chebyshev(lev["L"], b, self.nu, hi / self.alpha, hi)

    def cycle(self, b, level=0):
        lev = self.levels[level]
        if level == len(self.levels) - 1:
            return chebyshev(lev["L"], b, self.coarse_iters, *lev["lam"])
        L, P = lev["L"], lev["P"]
        x = self.smooth(lev, b)
        x = x + P @ self.cycle(P.T @ (b - L @ x), level + 1)
        return x + self.smooth(lev, b - L @ x)


def jacobi_pcg(A, b, iters):
    """Fixed-count CG with Jacobi preconditioner from x0 = 0 (Sec. III inner solver), with the
    Hermitian inner product; stops early only if the residual is exactly zero."""
    Dinv = 1.0 / A.diagonal()
    x = np.zeros_like(b)
    r = b.copy()
    z = Dinv * r
    p = z.copy()
    rho = np.vdot(r, z).real
    for it in range(iters):
        if rho == 0.0:
            break
        q = A @ p
        alpha = rho / np.vdot(p, q).real
        x = x + alpha * p
        r = r - alpha * q
        if it == iters - 1:
            break
        z = Dinv * r
        rho_new = np.vdot(r, z).real
        beta = rho_new / rho
        p = z + beta * p
        rho = rho_new
    return x


def chebyshev(A, b, iters, lam_min, lam_max):
    """Fixed-count Chebyshev iteration for A x = b preconditioned by D = diag(A), x0 = 0, for a
    spectrum of D^{-1} A inside [lam_min, lam_max] (Chebyshev acceleration, Saad, Iterative Methods
    for Sparse Linear Systems, Sec. 12.3): theta, delta = centre and half width, sigma = theta/delta,
    d_0 = D^{-1} r_0 / theta, rho_0 = 1/sigma, then x += d; r -= A d; rho' = 1/(2 sigma - rho);
    d = rho' rho d + (2 rho'/delta) D^{-1} r."""
    Dinv = 1.0 / A.diagonal()
    theta = 0.5 * (lam_max + lam_min)
    delta = 0.5 * (lam_max - lam_min)
    sigma = theta / delta
    x = np.zeros_like(b)
    r = b.copy()
    d = Dinv * r / theta
    rho = 1.0 / sigma
    for k in range(iters):
        x = x + d
        if k == iters - 1:
            break
        r = r - A @ d
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (Dinv * r)
        rho = rho_new
    return x


# ---------------------------------------------------------------------------------------
# Closed-form Fourier symbols on the periodic uniform mesh (pins for the operators)
# ---------------------------------------------------------------------------------------

def symbols_at(grid: "Grid", kvec, theta):
    """M^, K^ and G^ of the plane wave with phase increments theta_d = q_d h (see fourier_symbols)."""
    h = grid.h
    m = [(2.0 + math.cos(t)) / 3.0 for t in theta]
    Mh = h ** grid.dim * np.prod(m)
    Kh = 0.0
    Th = 0.0
    for d in range(grid.dim):
        other = np.prod([m[e] for e in range(grid.dim) if e != d])
        Kh += (2.0 - 2.0 * math.cos(theta[d])) * other
        Th += 2.0 * kvec[d] * 1j * math.sin(theta[d]) * other
    Kh *= h ** (grid.dim - 2)
    Th *= h ** (grid.dim - 1)
    return Mh, Kh, -Kh + 1j * Th


def fourier_symbols(grid: Grid, kvec, mode):
    """Eigenvalues of M, K, G_j on the plane wave e^{i q.r} with q = 2 pi mode / L.

    With theta_d = q_d h and m(theta) = (2 + cos theta)/3:
      M^ = h^dim prod_d m(theta_d)
      K^ = h^(dim-2) sum_d (2 - 2 cos theta_d) prod_{e != d} m(theta_e)
      T^ = h^(dim-1) sum_d 2 k_d (i sin theta_d) prod_{e != d} m(theta_e)
      G^ = -K^ + i T^
    """
    h = grid.h
    th = [2.0 * math.pi * mode[d] / grid.n[d] for d in range(grid.dim)]
    m = [(2.0 + math.cos(t)) / 3.0 for t in th]
    Mh = h ** grid.dim * np.prod(m)
    Kh = 0.0
    Th = 0.0
    for d in range(grid.dim):
        other = np.prod([m[e] for e in range(grid.dim) if e != d])
        Kh += (2.0 - 2.0 * math.cos(th[d])) * other
        Th += 2.0 * kvec[d] * 1j * math.sin(th[d]) * other
    Kh *= h ** (grid.dim - 2)
    Th *= h ** (grid.dim - 1)
    return Mh, Kh, -Kh + 1j * Th


def plane_wave(grid: Grid, mode):
    idx = np.meshgrid(*[np.arange(grid.n[d]) for d in range(grid.dim)][::-1], indexing="ij")
    idx = [i.reshape(-1) for i in idx[::-1]]
    ph = sum(2.0 * math.pi * mode[d] * idx[d] / grid.n[d] for d in range(grid.dim))
    return np.exp(1j * ph)


def model_spectrum(q: np.ndarray, k: float = 1.0, kappa: float = 1.0, tau: float = 1.0):
    """Eigenvalues of A P^{-1} for the 1D symbols of Sec. II.B (J = 0, M = 1):
    A = [[1, q^2+2qk], [-kappa (q^2+2qk), 1/tau]],
    P = [[1, 0], [-kappa (q^2+2qk), 1/sqrt(tau) + sqrt(kappa) q^2]] [[1, -q^2], [0, 1/sqrt(tau) + sqrt(kappa) q^2]]."""
    out = []
    for qq in q:
        g = qq * qq + 2.0 * qq * k
        A = np.array([[1.0, g], [-kappa * g, 1.0 / tau]])
        s = 1.0 / math.sqrt(tau) + math.sqrt(kappa) * qq * qq
        P = np.array([[1.0, 0.0], [-kappa * g, s]]) @ np.array([[1.0, -qq * qq], [0.0, s]])
        out.append(np.linalg.eigvals(A @ np.linalg.inv(P)))
    return np.array(out)


# ---------------------------------------------------------------------------------------
# Local lattice rotation and the refinement indicator (Sec. II.C, Eq. (13)-(17))
# ---------------------------------------------------------------------------------------

def nodal_gradient(grid: Grid, f: np.ndarray) -> np.ndarray:
    """Central differences on the periodic grid: (f(x + h e_d) - f(x - h e_d)) / (2h), shape (dim, ...)."""
    shape = tuple(grid.n[: grid.dim][::-1])            # numpy order (z, y, x) / (y, x)
    F = f.reshape(f.shape[:-1] + shape)
    out = []
    for d in range(grid.dim):
        ax = F.ndim - 1 - d
        out.append(((np.roll(F, -1, axis=ax) - np.roll(F, 1, axis=ax)) / (2.0 * grid.h)).reshape(f.shape))
    return np.stack(out)


def rotation_field(grid: Grid, k: np.ndarray, eta: np.ndarray, tiny: float = 1e-12):
    """Rotation omega_ab = (du_a/dx_b - du_b/dx_a)/2 (Eq. (14)) of the displacement u defined by
    k_j . u = arg eta_j (Eq. (15)).  Phase gradients avoid unwrapping:
    grad arg eta_j = Im(conj(eta_j) grad eta_j)/|eta_j|^2 with central differences; the per-node
    system k_j . (du/dx_b) = d arg eta_j/dx_b is solved in the least-squares sense over the
    amplitudes with |eta_j|^2 > tiny (reading: the paper cites explicit formulas elsewhere).
    Returns omega with shape (N,) in 2D (omega_12) and (3, N) in 3D (omega_23, omega_31, omega_12)."""
    dim = grid.dim
    J = len(k)
    kk = np.asarray(k, float)[:, :dim]
    grad_eta = nodal_gradient(grid, eta)                          # (dim, J, N)
    mag2 = np.abs(eta) ** 2
    ok = mag2 > tiny
    dtheta = np.where(ok[None], np.imag(np.conj(eta)[None] * grad_eta) / np.where(ok, mag2, 1.0)[None], 0.0)
    N = eta.shape[1]
    Gu = np.zeros((N, dim, dim))                                  # Gu[n, a, b] = du_a/dx_b
    for n in range(N):
        sel = ok[:, n]
        if sel.sum() < dim:
            continue
        Ks = kk[sel]
        Ainv = np.linalg.inv(Ks.T @ Ks)
        for b in range(dim):
            Gu[n, :, b] = Ainv @ (Ks.T @ dtheta[b, sel, n])
    if dim == 2:
        return 0.5 * (Gu[:, 0, 1] - Gu[:, 1, 0])
    return np.stack([0.5 * (Gu[:, 1, 2] - Gu[:, 2, 1]), 0.5 * (Gu[:, 2, 0] - Gu[:, 0, 2]),
                     0.5 * (Gu[:, 0, 1] - Gu[:, 1, 0])])


def refinement_h(grid: Grid, k: np.ndarray, eta: np.ndarray, omega: np.ndarray, n_per_wavelength: float,
                 eps: float, A_min: float, h_int: float, h_max: float):
    """Target mesh size of Eq. (17): h_int where |grad A| >= eps; min(max(h_amp, h_int), h_max) where
    A > A_min; h_max elsewhere, with h_amp = min_j lambda_j(theta)/n (Eq. (16)), theta = asin of the
    largest rotation component, lambda_j(theta) = 2 pi/|dk_j(theta)| and |dk_j| = 2 |k_j| sin(theta/2)."""
    A = 2.0 * np.sum(np.abs(eta) ** 2, axis=0)
    gA = np.sqrt(np.sum(nodal_gradient(grid, A[None])[:, 0] ** 2, axis=0))
    om = np.abs(omega) if omega.ndim == 1 else np.max(np.abs(omega), axis=0)
    theta = np.arcsin(np.minimum(om, 1.0))
    kmax = np.max(np.linalg.norm(np.asarray(k, float), axis=1))
    with np.errstate(divide="ignore"):
        lam = np.where(theta > 0, 2.0 * np.pi / (2.0 * kmax * np.sin(0.5 * theta)), np.inf)
    h_amp = lam / n_per_wavelength
    return np.where(gA >= eps, h_int, np.where(A > A_min, np.minimum(np.maximum(h_amp, h_int), h_max), h_max))
