"""Independent reference constructions used to pin the oracle.

Nothing here calls the oracle or the HIP library.  Each helper builds a
quantity from its mathematical definition by a different route than the
oracle takes (dense Kronecker matrices instead of stencil loops, a
Vandermonde solve instead of Lagrange-polynomial integration, closed-form
Pade approximants instead of the collocation matrix).
"""
from __future__ import annotations

import json
import os
from fractions import Fraction

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name: str):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def frac(pair) -> float:
    return float(Fraction(pair[0], pair[1]))


def lobatto5() -> np.ndarray:
    r = np.sqrt(3.0 / 7.0)
    return np.array([0.0, (1 - r) / 2, 0.5, (1 + r) / 2, 1.0])


def q_vandermonde(s: np.ndarray) -> np.ndarray:
    """Q[m, i] from exactness on monomials: sum_i Q[m,i] s_i^j = s_m^(j+1)/(j+1)."""
    nn = len(s)
    V = np.vander(s, nn, increasing=True)          # V[i, j] = s_i^j
    rhs = np.array([[sm ** (j + 1) / (j + 1) for j in range(nn)] for sm in s])
    # rows: Q[m,:] V = rhs[m,:]  ->  V^T Q[m,:]^T = rhs[m,:]^T
    return np.linalg.solve(V.T, rhs.T).T


def q_delta(s: np.ndarray) -> np.ndarray:
    """Backward-Euler matrix of eq. Qbe: Q_D[m, j] = s_j - s_{j-1} for 1 <= j <= m."""
    nn = len(s)
    Qd = np.zeros((nn, nn))
    for m in range(1, nn):
        for j in range(1, m + 1):
            Qd[m, j] = s[j] - s[j - 1]
    return Qd


def lap_1d(n: int):
    h2 = 1.0 / (n + 1) ** 2
    return sp.diags([np.ones(n - 1), -2 * np.ones(n), np.ones(n - 1)], [-1, 0, 1]) / h2


def lap_dense(dim: int, n: int) -> np.ndarray:
    """Kronecker-sum Laplacian, x fastest (matches C-order [z, y, x] flattening)."""
    L1 = lap_1d(n)
    I = sp.identity(n)
    if dim == 1:
        L = L1
    elif dim == 2:
        L = sp.kron(I, L1) + sp.kron(L1, I)
    else:
        L = sp.kron(sp.kron(I, I), L1) + sp.kron(sp.kron(I, L1), I) + sp.kron(sp.kron(L1, I), I)
    return L.toarray()


def mu(n: int, k) -> float:
    """Eigenvalue of the discrete Laplacian for the sine mode k (tuple over dims)."""
    h = 1.0 / (n + 1)
    return float(sum((2 * np.cos(kd * np.pi * h) - 2) / h ** 2 for kd in k))


def pade(z, num):
    """Diagonal Pade approximant with numerator coefficients num (Fractions as pairs)."""
    c = [frac(p) for p in num]
    N = sum(ck * z ** j for j, ck in enumerate(c))
    D = sum(ck * (-z) ** j for j, ck in enumerate(c))
    return N / D


def collocation_block(A: np.ndarray, Q: np.ndarray, dt: float, u0: np.ndarray, P: int):
    """Composite collocation solution: for each slice solve (I - dt Q (x) A) U = 1 (x) u0_p
    densely, u0_{p+1} = last node.  Returns list of (nn, D) arrays."""
    nn, D = Q.shape[0], A.shape[0]
    big = np.eye(nn * D) - dt * np.kron(Q, A)
    lu = sla.lu_factor(big)
    out = []
    start = u0.copy()
    for _ in range(P):
        U = sla.lu_solve(lu, np.tile(start, nn)).reshape(nn, D)
        out.append(U)
        start = U[-1].copy()
    return out


def rel_err(a, b) -> float:
    a = np.asarray(a); b = np.asarray(b)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def kron_sum(L1: np.ndarray, dim: int) -> np.ndarray:
    """sum over axes of I (x) .. L1 .. (x) I, x fastest (C order [z, y, x])."""
    n = L1.shape[0]
    eye = np.eye(n)
    out = np.zeros((n ** dim, n ** dim))
    for ax in range(dim):              # ax = 0 is x, the fastest index
        term = np.ones((1, 1))
        for pos in range(dim):         # slowest factor first
            term = np.kron(term, L1 if pos == dim - 1 - ax else eye)
        out += term
    return out


def lap4_1d(n: int) -> np.ndarray:
    """Fourth-order second difference (-1, 16, -30, 16, -1)/(12 h^2) on the n
    interior points of [0, 1], with the value beyond the boundary the odd
    reflection of the first interior value (u_{-1} = -u_1, u_0 = 0): the two
    boundary rows carry -29 on the diagonal."""
    h2 = 1.0 / (n + 1) ** 2
    L = np.zeros((n, n))
    for i in range(n):
        for off, c in ((-2, -1.0), (-1, 16.0), (0, -30.0), (1, 16.0), (2, -1.0)):
            j = i + off
            if 0 <= j < n:
                L[i, j] += c
            elif j == -2:              # index -1 (1-based): odd image of index 1
                L[i, 0] -= c
            elif j == n + 1:           # index n+2 (1-based): odd image of index n
                L[i, n - 1] -= c
            # j == -1 or j == n: the Dirichlet boundary value 0
    return L / (12.0 * h2)


def lap4_dense(dim: int, n: int) -> np.ndarray:
    return kron_sum(lap4_1d(n), dim)


def prolong_dense(dim: int, nc: int) -> np.ndarray:
    """d-linear interpolation from nc to n = 2 nc + 1 interior points, zero
    boundary: the tensor product of the 1D matrix (coarse J -> fine 2J with
    weight 1, fine 2J +- 1 with weight 1/2, 1-based)."""
    n = 2 * nc + 1
    P1 = np.zeros((n, nc))
    for J in range(1, nc + 1):
        P1[2 * J - 1, J - 1] = 1.0
        P1[2 * J - 2, J - 1] = 0.5
        P1[2 * J, J - 1] = 0.5
    P = np.ones((1, 1))
    for _ in range(dim):
        P = np.kron(P, P1)
    return P


def red_mask(dim: int, n: int) -> np.ndarray:
    """Points whose 1-based index sum is even, flattened x fastest."""
    idx = np.indices((n,) * dim).reshape(dim, -1) + 1
    return (idx.sum(axis=0) % 2) == 0


def jor_pass(A: np.ndarray, diag: float, mask: np.ndarray, omega: float, b: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Relax the masked points together from the current u: u + omega (b - A u)/diag there."""
    r = b - A @ u
    out = u.copy()
    out[mask] += omega * r[mask] / diag
    return out


def dense_smooth(A, diag, dim, n, rb: bool, omega, b, u):
    if not rb:
        return jor_pass(A, diag, np.ones(n ** dim, bool), omega, b, u)
    red = red_mask(dim, n)
    return jor_pass(A, diag, ~red, omega, b, jor_pass(A, diag, red, omega, b, u))


def dense_vcycle(dim: int, n: int, alpha: float, b: np.ndarray, u: np.ndarray, rb: bool, omega: float,
                 nu1: int = 2, nu2: int = 2, fourth: bool = False) -> np.ndarray:
    """Two-grid recursion with dense matrices: nu1 smoothing passes on
    A = I - alpha L (L4 on this level when ``fourth``), full weighting
    R = P^T / 2^dim of the residual, the same recursion (second order) for
    the correction from zero, u += P e_c, nu2 passes; grids with n <= 2 are
    solved exactly.  The smoother's divisor is the interior stencil's centre
    coefficient, 1 + 2 dim alpha/h^2 (second order) or 1 + 2.5 dim alpha/h^2
    (fourth order)."""
    ih2 = float(n + 1) ** 2
    L = lap4_dense(dim, n) if fourth else lap_dense(dim, n)
    A = np.eye(n ** dim) - alpha * L
    if n <= 2:
        return np.linalg.solve(A, b)
    diag = 1.0 + (2.5 if fourth else 2.0) * dim * alpha * ih2
    for _ in range(nu1):
        u = dense_smooth(A, diag, dim, n, rb, omega, b, u)
    nc = (n + 1) // 2 - 1
    P = prolong_dense(dim, nc)
    bc = (P.T / 2 ** dim) @ (b - A @ u)
    ec = dense_vcycle(dim, nc, alpha, bc, np.zeros(nc ** dim), rb, omega, nu1, nu2, False)
    u = u + P @ ec
    for _ in range(nu2):
        u = dense_smooth(A, diag, dim, n, rb, omega, b, u)
    return u
