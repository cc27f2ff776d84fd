"""Pins for the oracle's fourth-order spatial discretisation (the paper's
fourth-order runs, Sec. 4.3): the 5-point-per-axis Laplacian with odd
reflection beyond the boundary, its multigrid solve, and IPFASST with it on
the fine level.

The pins come from outside the stencil code: the sine modes are the
operator's eigenvectors with a closed-form eigenvalue, so the direct solve
is a discrete sine transform, and the converged collocation end values are
the stability function applied mode by mode.
"""
import numpy as np
import pytest
from scipy.fft import dstn, idstn

import inputs
import oracle as O
from tests import pins
from tests.test_oracle_uniform_nodes import norsett

EXACT = dict(cycles=0, tol=1e-14, stall=0.999, max_cycles=100)


def lam4(n, k):
    """Eigenvalue of the fourth-order Laplacian on sine mode k (tuple):
    per axis (-2 cos(2 k pi h) + 32 cos(k pi h) - 30) / (12 h^2)."""
    h = 1.0 / (n + 1)
    return float(sum((-2 * np.cos(2 * kd * np.pi * h) + 32 * np.cos(kd * np.pi * h) - 30) / (12 * h * h) for kd in k))


@pytest.mark.parametrize("dim,n,k", [(1, 15, (1,)), (1, 15, (15,)), (1, 63, (7,)), (3, 15, (1, 2, 3)),
                                     (3, 15, (15, 1, 14)), (3, 31, (4, 9, 30))])
def test_sine_modes_are_eigenvectors(dim, n, k):
    phi = inputs.sine_mode(n, k, dim)
    out = O.lap4(dim, phi)
    lam = lam4(n, k)
    assert pins.rel_err(out, lam * phi) <= 1e-13


def test_fourth_order_accurate():
    """The eigenvalue of sin(pi x) sin(2 pi y) sin(3 pi z) tends to -14 pi^2
    with error O(h^4): halving h divides it by about 16."""
    errs = []
    for n in (15, 31, 63):
        phi = inputs.sine_mode(n, (1, 2, 3), 3)
        lam = np.sum(O.lap4(3, phi) * phi) / np.sum(phi * phi)
        errs.append(abs(lam + 14 * np.pi ** 2))
    for a, b in zip(errs, errs[1:]):
        assert 15.0 < a / b < 16.5, errs


def direct_solve(dim, alpha, b):
    """(I - alpha L4)^-1 b by the sine transform (DST-I diagonalises L4)."""
    n = b.shape[0]
    c = dstn(b, type=1)
    ks = np.arange(1, n + 1)
    h = 1.0 / (n + 1)
    l1 = (-2 * np.cos(2 * ks * np.pi * h) + 32 * np.cos(ks * np.pi * h) - 30) / (12 * h * h)
    lam = np.zeros((n,) * dim)
    for ax in range(dim):
        shp = [1] * dim
        shp[dim - 1 - ax] = n
        lam = lam + l1.reshape(shp)
    return idstn(c / (1.0 - alpha * lam), type=1)


@pytest.mark.parametrize("dim,n,sm,om", [(3, 15, O.RBGS, 1.0), (3, 31, O.JACOBI, 2.0 / 3.0), (1, 63, O.RBGS, 1.0)])
def test_full_solve_matches_sine_transform(dim, n, sm, om):
    alpha = 4.0 / (n + 1) ** 2
    b = inputs.random_field((n,) * dim, 31 + n)
    u, cycles, rr = O.mg_solve4(dim, alpha, b, np.zeros_like(b), O.policy(smoother=sm, omega=om, **EXACT))
    assert rr <= 1e-13 and cycles < 60
    assert pins.rel_err(u, direct_solve(dim, alpha, b)) <= 1e-11


@pytest.mark.parametrize("sm,om", [(O.RBGS, 1.0), (O.JACOBI, 2.0 / 3.0)])
def test_vcycle_contracts(sm, om):
    """A V(2,2) cycle whose finest level is fourth order reduces the error
    by a grid-independent factor (measured against the direct solve)."""
    for n, ah in ((15, 2.0), (31, 2.0), (31, 50.0), (63, 5.0)):
        alpha = ah / (n + 1) ** 2
        b = inputs.random_field((n,) * 3, 7 + n)
        x = direct_solve(3, alpha, b)
        u = np.zeros_like(b)
        e0 = np.max(np.abs(u - x))
        for _ in range(3):
            u = O.vcycle4(3, alpha, b, u, smoother=sm, omega=om)
        rate = (np.max(np.abs(u - x)) / e0) ** (1 / 3)
        assert rate < (0.35 if sm == O.RBGS else 0.6), (n, ah, rate)


@pytest.mark.parametrize("fam,interp", [(O.UNIFORM, 4), (O.LOBATTO, 2), (O.UNIFORM, 2)])
def test_heat1d_fourth_order_end_values(fam, interp):
    """1D heat (N=31, P=4, dt=0.01) with L4 on the fine level, coarse level
    second order, iterated to convergence: each slice's end value is
    sum_k a_k R(dt nu lambda4_k)^(p+1) phi_k, R the fine rule's stability
    function (Norsett for uniform nodes, the Pade (4,4) form for Lobatto)."""
    n, nu, dt, P = 31, 1.0, 0.01, 4
    u0, modes = inputs.heat_1d(n)
    pf = O.Pfasst(1, n, nu, dt, P, 5, 3, O.policy(smoother=O.RBGS, cycles=2), interp_order=interp,
                  node_family=fam, stencil_order=4)
    pf.set_initial(u0)
    it = 0
    while pf.iterate() > 1e-13 and it < 300:
        it += 1
    if fam == O.UNIFORM:
        R = lambda z: norsett([0.25, 0.5, 0.75, 1.0], z)
    else:
        g = pins.golden("lobatto_iiia.json")
        R = lambda z: pins.pade(z, g["pade44_num"])
    for p in range(P):
        want = sum(a * R(dt * nu * lam4(n, k)) ** (p + 1) * inputs.sine_mode(n, k, 1)
                   for a, k in zip(modes.amp, modes.k))
        assert pins.rel_err(pf.field(O.UF, p, 4), want) <= 1e-11, p


def test_fourth_order_rejects_mixed_precision():
    with pytest.raises(ValueError):
        O.Pfasst(3, 15, 1.0, 1e-3, 2, 5, 3, O.policy(cycles=1, mixed=1), stencil_order=4)
    with pytest.raises(ValueError):
        O.Pfasst(3, 15, 1.0, 1e-3, 2, 5, 3, O.policy(cycles=1), stencil_order=3)
