"""Pins for the oracle's stencil and multigrid routines (Sec. 4.1 / 4.2,
multigrid of Sec. 4.1.1 and Sec. 4.2.1)."""
import numpy as np
import pytest
import scipy.linalg as sla

import inputs
import oracle as O
from tests import pins


def mode(dim, n, k):
    return inputs.sine_mode(n, k, dim)


@pytest.mark.parametrize("dim,n,k", [(1, 15, (3,)), (1, 127, (8,)), (3, 7, (1, 2, 3)), (3, 15, (5, 1, 7))])
def test_laplacian_eigenmodes(dim, n, k):
    """L_h phi_k = mu_k phi_k with mu_k = sum_d (2 cos(k_d pi h) - 2)/h^2
    (Sec. 4.1, with the sign read so that modes decay)."""
    phi = mode(dim, n, k)
    Lphi = O.lap(dim, phi)
    assert pins.rel_err(Lphi, pins.mu(n, k) * phi) <= 1e-13
    alpha = 0.37
    assert pins.rel_err(O.helm(dim, alpha, phi), (1 - alpha * pins.mu(n, k)) * phi) <= 1e-13


@pytest.mark.parametrize("dim,n", [(1, 9), (3, 5)])
def test_operators_match_dense_kronecker(dim, n):
    u = inputs.random_field((n,) * dim, 1)
    b = inputs.random_field((n,) * dim, 2)
    L = pins.lap_dense(dim, n)
    assert pins.rel_err(O.lap(dim, u).ravel(), L @ u.ravel()) <= 1e-14
    a = 0.02
    H = np.eye(n ** dim) - a * L
    assert pins.rel_err(O.resid(dim, a, b, u).ravel(), b.ravel() - H @ u.ravel()) <= 1e-14


@pytest.mark.parametrize("dim,n,k", [(1, 31, (5,)), (3, 15, (2, 9, 4))])
def test_jacobi_damps_each_mode_by_closed_form(dim, n, k):
    """Weighted Jacobi on a mode with b = 0 multiplies it by
    1 - omega (1 - alpha mu_k)/(1 + 2 dim alpha/h^2)."""
    phi = mode(dim, n, k)
    alpha, omega = 3e-3, 2.0 / 3.0
    ih2 = (n + 1) ** 2
    g = 1 - omega * (1 - alpha * pins.mu(n, k)) / (1 + 2 * dim * alpha * ih2)
    out = O.smooth(dim, alpha, O.JACOBI, omega, np.zeros_like(phi), phi)
    assert pins.rel_err(out, g * phi) <= 1e-13


@pytest.mark.parametrize("dim,n", [(1, 7), (3, 5)])
def test_rbgs_equals_dense_gauss_seidel_in_red_black_order(dim, n):
    """Red-black Gauss-Seidel = forward Gauss-Seidel on the matrix with the
    unknowns ordered red first (1-based index sum even), then black."""
    a = 0.05
    L = pins.lap_dense(dim, n)
    H = np.eye(n ** dim) - a * L
    idx = np.indices((n,) * dim).reshape(dim, -1) + 1          # 1-based, [z,y,x] order
    red = (idx.sum(axis=0) % 2) == 0
    perm = np.concatenate([np.where(red)[0], np.where(~red)[0]])
    Hp = H[np.ix_(perm, perm)]
    b = inputs.random_field((n,) * dim, 3)
    u = inputs.random_field((n,) * dim, 4)
    bp, up = b.ravel()[perm], u.ravel()[perm]
    lower = np.tril(Hp)
    upper = Hp - lower
    new = sla.solve_triangular(lower, bp - upper @ up, lower=True)
    want = np.empty_like(new)
    want[perm] = new
    got = O.smooth(dim, a, O.RBGS, 1.0, b, u).ravel()
    assert pins.rel_err(got, want) <= 1e-14


@pytest.mark.parametrize("dim,n,k", [(1, 31, (5,)), (1, 31, (13,)), (3, 15, (3, 5, 6))])
def test_transfer_operators_on_sine_modes(dim, n, k):
    """Full weighting maps fine mode k to cos^2(k pi h/2) times the coarse mode;
    linear interpolation maps coarse mode k to c phi_k - s phi_{N+1-k} per
    dimension with c = cos^2(k pi h/2), s = sin^2(k pi h/2)."""
    h = 1.0 / (n + 1)
    nc = (n + 1) // 2 - 1
    phi = mode(dim, n, k)
    rc = O.restrict_fw(dim, phi)
    fac = np.prod([np.cos(kd * np.pi * h / 2) ** 2 for kd in k])
    assert pins.rel_err(rc, fac * mode(dim, nc, k)) <= 1e-13
    # prolongation of the coarse mode: tensor product of the 1D pair
    pc = O.prolong_add(dim, mode(dim, nc, k), np.zeros((n,) * dim))
    want = np.zeros((n,) * dim)
    for sel in np.ndindex(*(2,) * dim):
        kk = tuple((n + 1 - kd) if s else kd for kd, s in zip(k, sel))
        w = np.prod([(-np.sin(kd * np.pi * h / 2) ** 2) if s else np.cos(kd * np.pi * h / 2) ** 2
                     for kd, s in zip(k, sel)])
        want += w * mode(dim, n, kk)
    assert pins.rel_err(pc, want) <= 1e-13


@pytest.mark.parametrize("dim,n", [(1, 15), (3, 7)])
def test_restriction_is_scaled_transpose_of_prolongation(dim, n):
    nc = (n + 1) // 2 - 1
    Pm = np.stack([O.prolong_add(dim, e.reshape((nc,) * dim), np.zeros((n,) * dim)).ravel()
                   for e in np.eye(nc ** dim)], axis=1)
    Rm = np.stack([O.restrict_fw(dim, e.reshape((n,) * dim)).ravel() for e in np.eye(n ** dim)], axis=1)
    assert np.max(np.abs(Rm - Pm.T / 2 ** dim)) <= 1e-16


@pytest.mark.parametrize("dim,n", [(1, 1), (1, 2), (3, 1), (3, 2)])
def test_coarsest_exact(dim, n):
    a = 0.7
    b = inputs.random_field((n,) * dim, 5)
    H = np.eye(n ** dim) - a * pins.lap_dense(dim, n)
    u = O.coarsest(dim, a, b)
    assert pins.rel_err(u.ravel(), np.linalg.solve(H, b.ravel())) <= 1e-14


@pytest.mark.parametrize("dim,n,sm,om", [(1, 31, O.JACOBI, 2 / 3), (3, 15, O.RBGS, 1.0),
                                         (3, 7, O.JACOBI, 2 / 3), (3, 11, O.RBGS, 1.0)])
def test_full_solve_matches_dense_solve(dim, n, sm, om):
    a = 2e-3
    H = np.eye(n ** dim) - a * pins.lap_dense(dim, n)
    b = inputs.random_field((n,) * dim, 6)
    pol = O.policy(smoother=sm, omega=om, cycles=0, tol=1e-13, stall=0.99, max_cycles=100)
    u, ncyc, rr = O.mg_solve(dim, a, b, np.zeros_like(b), pol)
    assert rr <= 1e-13 and ncyc >= 2
    assert pins.rel_err(u.ravel(), np.linalg.solve(H, b.ravel())) <= 1e-12


def test_full_solve_of_sine_mode_closed_form():
    """u = b / (1 - alpha mu_k) for a single mode right-hand side."""
    dim, n, k, a = 3, 31, (2, 3, 5), 1e-3
    phi = mode(dim, n, k)
    pol = O.policy(smoother=O.RBGS, cycles=0, tol=1e-14, stall=0.99, max_cycles=60)
    u, _, _ = O.mg_solve(dim, a, phi, np.zeros_like(phi), pol)
    assert pins.rel_err(u, phi / (1 - a * pins.mu(n, k))) <= 1e-12


def _vcycle_error_matrix(dim, n, a, sm, om):
    cols = []
    for e in np.eye(n ** dim):
        cols.append(O.vcycle(dim, a, np.zeros((n,) * dim), e.reshape((n,) * dim), sm, om).ravel())
    return np.stack(cols, axis=1)


def test_vcycle_is_consistent_linear_iteration():
    """The exact solution is a fixed point and the error propagates by a
    fixed matrix E (V(u*+e, b) - u* = E e) with spectral radius well below 1."""
    dim, n, a = 3, 7, 5e-3
    H = np.eye(n ** dim) - a * pins.lap_dense(dim, n)
    b = inputs.random_field((n,) * dim, 7)
    ustar = np.linalg.solve(H, b.ravel()).reshape(b.shape)
    assert pins.rel_err(O.vcycle(dim, a, b, ustar), ustar) <= 1e-13
    e = inputs.random_field(b.shape, 8)
    E = _vcycle_error_matrix(dim, n, a, O.RBGS, 1.0)
    assert pins.rel_err((O.vcycle(dim, a, b, ustar + e) - ustar).ravel(), E @ e.ravel()) <= 1e-12
    rho = max(abs(np.linalg.eigvals(E)))
    assert rho < 0.15


@pytest.mark.parametrize("ah2,want", [(28.3, 0.0853), (53.6, 0.0874), (81.9, 0.0888)])
def test_vcycle_factor_1d_jacobi(ah2, want):
    """1D V(2,2), weighted Jacobi 2/3, N = 127: the spectral radius of the
    assembled error matrix.  Reference values: an independent dense
    computation of the same two-grid-recursive operator (parity unpinned by
    the paper, whose V-cycle figure is not available)."""
    n = 127
    a = ah2 / (n + 1) ** 2
    E = _vcycle_error_matrix(1, n, a, O.JACOBI, 2.0 / 3.0)
    rho = max(abs(np.linalg.eigvals(E)))
    assert abs(rho - want) < 1.5e-3


def test_mixed_precision_refinement_reaches_fp64_accuracy():
    """FP32 V-cycles inside FP64 iterative refinement converge to the FP64
    solution (the refinement residual is formed in FP64)."""
    dim, n, a = 3, 15, 4e-3
    b = inputs.random_field((n,) * dim, 9)
    pol64 = O.policy(cycles=0, tol=1e-14, stall=0.99, max_cycles=60)
    u64, _, _ = O.mg_solve(dim, a, b, np.zeros_like(b), pol64)
    pol = O.policy(cycles=12, mixed=1)
    u, _, rr = O.mg_solve(dim, a, b, np.zeros_like(b), pol)
    assert rr <= 1e-13
    assert pins.rel_err(u, u64) <= 1e-12
    # one FP32 cycle differs from the FP64 cycle only by FP32 rounding
    v64 = O.vcycle(dim, a, b, np.zeros_like(b))
    v32 = O.vcycle32(dim, a, b.astype(np.float32), np.zeros(b.shape, np.float32))
    assert pins.rel_err(v32, v64) <= 1e-5


def test_full_solve_stall_and_divergence_paths():
    """Policy of Sec. 4.2.1: a divergent smoother (Jacobi with omega 1.9)
    stops at the first cycle that fails to cut the residual below 75%."""
    dim, n, a = 1, 31, 1.0
    b = inputs.random_field((n,), 10)
    pol = O.policy(smoother=O.JACOBI, omega=1.9, cycles=0, tol=1e-12, stall=0.75, max_cycles=50)
    _, ncyc, rr = O.mg_solve(dim, a, b, np.zeros_like(b), pol)
    assert ncyc < 50
    pol_cap = O.policy(smoother=O.JACOBI, omega=2 / 3, cycles=0, tol=1e-30, stall=1.0, max_cycles=3)
    _, ncyc, _ = O.mg_solve(dim, a, b, np.zeros_like(b), pol_cap)
    assert ncyc == 3
    # zero data: zero cycles
    _, ncyc, rr = O.mg_solve(dim, a, np.zeros_like(b), np.zeros_like(b), pol)
    assert ncyc == 0 and rr == 0.0


@pytest.mark.parametrize("dim,nc", [(1, 3), (1, 15), (3, 3), (3, 7)])
def test_cubic_interpolation_exact_on_cubics_vanishing_at_the_boundary(dim, nc):
    # Four-point Lagrange interpolation reproduces every cubic; with the zero
    # boundary values among the points, cubics that vanish at x = 0 and 1 are
    # interpolated exactly everywhere, in tensor products too.
    n = 2 * (nc + 1) - 1
    cubics = [lambda x: x * (1 - x) * (0.3 + x), lambda x: x * (1 - x) * (2.0 - 3.0 * x), lambda x: x * (1 - x)]
    xc = np.arange(1, nc + 1) / (nc + 1)
    xf = np.arange(1, n + 1) / (n + 1)
    if dim == 1:
        ec, want = cubics[0](xc), cubics[0](xf)
    else:
        ec = cubics[2](xc)[:, None, None] * cubics[1](xc)[None, :, None] * cubics[0](xc)[None, None, :]
        want = cubics[2](xf)[:, None, None] * cubics[1](xf)[None, :, None] * cubics[0](xf)[None, None, :]
    u = O.prolong4_add(dim, ec, np.zeros((n,) * dim))
    assert np.max(np.abs(u - want)) <= 1e-15


def test_cubic_interpolation_is_fourth_order():
    # error of interpolating sin(pi x) falls by ~16 per halving of h (the
    # linear interpolation's by ~4)
    errs4, errs2 = [], []
    for nc in (15, 31, 63):
        n = 2 * (nc + 1) - 1
        xc = np.arange(1, nc + 1) / (nc + 1)
        xf = np.arange(1, n + 1) / (n + 1)
        u4 = O.prolong4_add(1, np.sin(np.pi * xc), np.zeros(n))
        u2 = O.prolong_add(1, np.sin(np.pi * xc), np.zeros(n))
        errs4.append(np.max(np.abs(u4 - np.sin(np.pi * xf))))
        errs2.append(np.max(np.abs(u2 - np.sin(np.pi * xf))))
    for a, b in zip(errs4, errs4[1:]):
        assert 14.0 < a / b < 18.0
    for a, b in zip(errs2, errs2[1:]):
        assert 3.6 < a / b < 4.4


@pytest.mark.parametrize("dim,n,sm,om", [(1, 7, O.RBGS, 1.0), (1, 15, O.JACOBI, 2.0 / 3.0), (3, 7, O.RBGS, 1.0),
                                         (3, 7, O.JACOBI, 2.0 / 3.0)])
def test_vcycle_equals_dense_two_grid_recursion(dim, n, sm, om):
    """The second-order V(2,2) cycle equals its recursion written with dense
    matrices (red-black Gauss-Seidel is the red-black JOR pass with weight 1
    for the 7-point stencil, whose same-colour points do not couple)."""
    a = 3.0 / (n + 1) ** 2
    b = inputs.random_field((n,) * dim, 47)
    u = inputs.random_field((n,) * dim, 48)
    want = pins.dense_vcycle(dim, n, a, b.ravel(), u.ravel(), sm == O.RBGS, om)
    got = O.vcycle(dim, a, b, u, smoother=sm, omega=om).ravel()
    assert pins.rel_err(got, want) <= 1e-13
