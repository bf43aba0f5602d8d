"""The split form of the bilinear element stencils that the fused 2D Chebyshev kernels evaluate,
checked against the oracle's element-by-element assembly (Sec. II.A): with P = [1 4 1],
Q = [-1 2 -1] = 6 delta - P and E = [-1 0 1] (x fastest, periodic),
    M = (h/6)^2 P(x)P,   K = (delta(x)P + P(x)delta) - P(x)P/3,   T_j = (h/6)(k0 E(x)P + k1 P(x)E),
and cM M + cK K = a (pA + pC) + b pB + c (uA + uC) + d uB over the rows A, B, C of the x pass p = P u
and the centre values u, with a = cM (h/6)^2 - cK/3, b = 4a + cK, c = cK, d = 4 cK."""
import numpy as np
import scipy.sparse as sp

from oracle.apfc_oracle import Grid, assemble, tri_k


def _circ(n, lo, mid, hi):
    A = sp.diags([np.full(n, mid), np.full(n - 1, hi), np.full(n - 1, lo)], [0, 1, -1], format="lil")
    A[0, n - 1] += lo
    A[n - 1, 0] += hi
    return A.tocsr()


def _xy(op_y, op_x):
    return sp.kron(op_y, op_x, format="csr")   # x fastest


def test_split_form_matches_element_assembly():
    nx, ny, h = 7, 5, 0.9
    grid = Grid(2, (nx, ny), (nx * h, ny * h))
    k = tri_k()
    M, K, T = assemble(grid, k)
    Px, Py = _circ(nx, 1.0, 4.0, 1.0), _circ(ny, 1.0, 4.0, 1.0)
    Ex, Ey = _circ(nx, -1.0, 0.0, 1.0), _circ(ny, -1.0, 0.0, 1.0)
    Ix, Iy = sp.identity(nx, format="csr"), sp.identity(ny, format="csr")
    PP = _xy(Py, Px)
    assert abs(M - (h / 6) ** 2 * PP).max() < 1e-13
    Ks = _xy(Py, Ix) + _xy(Iy, Px) - PP / 3.0
    assert abs(K - Ks).max() < 1e-13
    for j in range(len(k)):
        Ts = (h / 6) * (k[j][0] * _xy(Py, Ex) + k[j][1] * _xy(Ey, Px))
        assert abs(T[j] - Ts).max() < 1e-13
    # the row form of L = cM M + cK K used per node
    cM, cK = 0.7, 1.9
    a = cM * (h / 6) ** 2 - cK / 3.0
    b, c, d = 4.0 * a + cK, cK, 4.0 * cK
    Sy = _circ(ny, 1.0, 0.0, 1.0)                 # rows A + C
    Ls = _xy(a * Sy + b * Iy, Px) + _xy(c * Sy + d * Iy, Ix)
    assert abs((cM * M + cK * K) - Ls).max() < 1e-12
    # a plausible slip (the K part without the -P(x)P/3 term) is caught
    assert abs(K - (_xy(Py, Ix) + _xy(Iy, Px))).max() > 1.0
