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


# ---- dense pins of the fourth-order smoother and V-cycle (Sec. 4.3's
# red-black JOR on the fine level): the operator, the colour order, the
# in-pass data dependence and the two-grid recursion are each rebuilt from
# dense matrices assembled independently of the stencil code.

@pytest.mark.parametrize("n", [5, 9, 15])
def test_dense_l4_has_the_sine_eigenpairs(n):
    """The dense 1D matrix (boundary rows by odd reflection) has the sine
    modes as eigenvectors with the closed-form eigenvalue."""
    L1 = pins.lap4_1d(n)
    for k in range(1, n + 1):
        phi = inputs.sine_mode(n, (k,), 1)
        assert pins.rel_err(L1 @ phi, lam4(n, (k,)) * phi) <= 1e-13


@pytest.mark.parametrize("dim,n", [(1, 5), (1, 9), (3, 3), (3, 5)])
def test_l4_and_residual_match_dense_matrix(dim, n):
    u = inputs.random_field((n,) * dim, 41)
    b = inputs.random_field((n,) * dim, 42)
    L = pins.lap4_dense(dim, n)
    assert pins.rel_err(O.lap4(dim, u).ravel(), L @ u.ravel()) <= 1e-14
    a = 0.03
    A = np.eye(n ** dim) - a * L
    assert pins.rel_err(O.resid4(dim, a, b, u).ravel(), b.ravel() - A @ u.ravel()) <= 1e-14


@pytest.mark.parametrize("dim,n,k", [(1, 15, (5,)), (1, 31, (29,)), (3, 7, (1, 6, 3)), (3, 15, (2, 9, 4))])
def test_jacobi4_damps_each_mode_by_closed_form(dim, n, k):
    """omega-Jacobi on L4 with b = 0 scales the sine mode k by
    1 - omega (1 - alpha lambda4_k)/(1 + 2.5 dim alpha/h^2)."""
    phi = inputs.sine_mode(n, k, dim)
    alpha, omega = 2e-3, 2.0 / 3.0
    g = 1 - omega * (1 - alpha * lam4(n, k)) / (1 + 2.5 * dim * alpha * (n + 1) ** 2)
    out = O.smooth4(dim, alpha, O.JACOBI, omega, np.zeros_like(phi), phi)
    assert pins.rel_err(out, g * phi) <= 1e-13


@pytest.mark.parametrize("dim,n,omega", [(1, 5, 1.0), (1, 7, 0.8), (3, 3, 1.0), (3, 5, 1.0), (3, 5, 0.7)])
def test_red_black_jor4_equals_dense_passes(dim, n, omega):
    """One red-black JOR pass on (I - alpha L4): the points with an even
    1-based index sum relax together from the values before the pass, then
    the odd points from the red-updated field."""
    a = 0.05 / (n + 1) ** 2 * 40
    A = np.eye(n ** dim) - a * pins.lap4_dense(dim, n)
    diag = 1.0 + 2.5 * dim * a * (n + 1) ** 2
    b = inputs.random_field((n,) * dim, 43).ravel()
    u = inputs.random_field((n,) * dim, 44).ravel()
    want = pins.dense_smooth(A, diag, dim, n, True, omega, b, u)
    got = O.smooth4(dim, a, O.RBGS, omega, b.reshape((n,) * dim), u.reshape((n,) * dim)).ravel()
    assert pins.rel_err(got, want) <= 1e-14
    # the pin separates the readings it rules out: black first, or black
    # from the pre-red values
    red = pins.red_mask(dim, n)
    swapped = pins.jor_pass(A, diag, red, omega, b, pins.jor_pass(A, diag, ~red, omega, b, u))
    simultaneous = u + omega * (b - A @ u) / diag
    assert pins.rel_err(got, swapped) > 1e-3 and pins.rel_err(got, simultaneous) > 1e-3


@pytest.mark.parametrize("dim,n,sm,om", [(1, 5, O.RBGS, 1.0), (1, 7, O.RBGS, 1.0), (1, 15, O.JACOBI, 2.0 / 3.0),
                                         (3, 3, O.RBGS, 1.0), (3, 7, O.RBGS, 1.0), (3, 7, O.JACOBI, 2.0 / 3.0)])
def test_vcycle4_equals_dense_two_grid_recursion(dim, n, sm, om):
    """V(2,2) with L4 on the finest level and the second-order rediscretised
    operator below it equals the same recursion written with dense matrices
    (dense L4 and L, interpolation matrix P, full weighting P^T/2^dim, exact
    solve on grids of at most two points)."""
    a = 3.0 / (n + 1) ** 2
    b = inputs.random_field((n,) * dim, 45)
    u = inputs.random_field((n,) * dim, 46)
    want = pins.dense_vcycle(dim, n, a, b.ravel(), u.ravel(), sm == O.RBGS, om, fourth=True)
    got = O.vcycle4(dim, a, b, u, smoother=sm, omega=om).ravel()
    assert pins.rel_err(got, want) <= 1e-13
