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
