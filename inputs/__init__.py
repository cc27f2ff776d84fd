"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

This module holds no arithmetic of the method: it only draws and evaluates
initial data for the heat equation u_t = nu * Laplace(u) on the unit
interval / cube with homogeneous Dirichlet data (the model problem of
Sec. 4 of arXiv:1407.6486).  Every array is float64, interior points
only, x fastest (numpy shape (n,) in 1D, (n, n, n) indexed [z, y, x] in 3D),
with mesh width h = 1/(n+1) and x_i = i*h, i = 1..n.

Workload recipes:
  * 1D: u0 = sin(pi x) + 0.1 sin(8 pi x)                       (heat_1d)
  * 3D: product of sines plus 32 random sine modes, amplitudes g/|k|^2
    with g ~ N(0,1), wave numbers drawn from 1..K, K = min(16, (n+1)/4),
    distinct and not (1,1,1); numpy PCG64 ``default_rng(seed)``  (random_fourier)
  * uneven batches: per problem q, ``default_rng([6486, q])`` draws n from
    {31, 63, 95, 127}, nu = 10**U(-1,1), dt = 10**U(-4,-2), then the data as
    above                                                        (batch_problem)
Each sine mode is an eigenvector of the discrete Laplacian, so every
initial condition here has a known modal decomposition (returned with it).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def grid_points(n: int) -> np.ndarray:
    return np.arange(1, n + 1, dtype=np.float64) / (n + 1)


@dataclass
class Modes:
    """u0 = sum_j amp[j] * prod_d sin(k[j, d] * pi * x_d)."""
    amp: np.ndarray      # (J,)
    k: np.ndarray        # (J, dim) integer wave numbers (x, y, z order)


def heat_1d(n: int = 127):
    x = grid_points(n)
    u = np.sin(np.pi * x) + 0.1 * np.sin(8 * np.pi * x)
    return u, Modes(np.array([1.0, 0.1]), np.array([[1], [8]]))


def sine_mode(n: int, k, dim: int = 3) -> np.ndarray:
    x = grid_points(n)
    if dim == 1:
        return np.sin(k[0] * np.pi * x)
    if dim == 2:
        return np.sin(k[1] * np.pi * x)[:, None] * np.sin(k[0] * np.pi * x)[None, :]
    sx = np.sin(k[0] * np.pi * x)
    sy = np.sin(k[1] * np.pi * x)
    sz = np.sin(k[2] * np.pi * x)
    return sz[:, None, None] * sy[None, :, None] * sx[None, None, :]


def draw_modes(rng: np.random.Generator, n: int, n_modes: int = 32, kmax: int | None = None) -> Modes:
    K = kmax if kmax is not None else min(16, (n + 1) // 4)
    K = max(K, 2)
    # small grids have fewer distinct modes than asked for: take them all
    n_modes = min(n_modes, K ** 3 - 1)
    seen = {(1, 1, 1)}
    ks = []
    while len(ks) < n_modes:
        k = tuple(int(v) for v in rng.integers(1, K + 1, size=3))
        if k in seen:
            continue
        seen.add(k)
        ks.append(k)
    g = rng.standard_normal(n_modes)
    karr = np.array(ks, dtype=np.int64)
    amp = g / (karr ** 2).sum(axis=1)
    return Modes(np.concatenate([[1.0], amp]), np.concatenate([[[1, 1, 1]], karr]))


def evaluate(n: int, modes: Modes, dim: int = 3) -> np.ndarray:
    u = np.zeros((n,) * dim)
    for a, k in zip(modes.amp, modes.k):
        u += a * sine_mode(n, k, dim)
    return u


def random_fourier(n: int, seed, n_modes: int = 32, kmax: int | None = None):
    rng = np.random.default_rng(seed)
    modes = draw_modes(rng, n, n_modes, kmax)
    return evaluate(n, modes), modes


@dataclass
class BatchProblem:
    n: int
    nu: float
    dt: float
    u0: np.ndarray
    modes: Modes


def batch_problem(q: int, sizes=(31, 63, 95, 127), materialise: bool = True) -> BatchProblem:
    rng = np.random.default_rng([6486, q])
    n = int(sizes[int(rng.integers(0, len(sizes)))])
    nu = float(10.0 ** rng.uniform(-1.0, 1.0))
    dt = float(10.0 ** rng.uniform(-4.0, -2.0))
    modes = draw_modes(rng, n)
    u0 = evaluate(n, modes) if materialise else None
    return BatchProblem(n, nu, dt, u0, modes)


def training_problem(r: int, n: int = 63):
    """Seeded problem for generating (rhs, solution) training pairs."""
    rng = np.random.default_rng([20000, r])
    dt = float(10.0 ** rng.uniform(-3.0, -2.0))
    modes = draw_modes(rng, n)
    return evaluate(n, modes), modes, dt


def random_field(shape, seed) -> np.ndarray:
    """Plain N(0,1) data for operator-level tests (not smooth)."""
    return np.random.default_rng(seed).standard_normal(shape)
