"""Pins for the oracle's SDC sweep, FAS coupling and PFASST iteration
(Sec. 2.2, 2.3, 3)."""
import numpy as np
import pytest

import inputs
import oracle as O
from tests import pins

EXACT = dict(cycles=0, tol=1e-15, stall=0.999, max_cycles=200)


def colloc_state(pf: O.Pfasst, dim, n, nu, dt, u0, P):
    """Set slices to the composite collocation solution (dense solve) and
    return it."""
    s = pins.lobatto5()
    Q = pins.q_vandermonde(s)
    A = nu * pins.lap_dense(dim, n)
    Us = pins.collocation_block(A, Q, dt, u0.ravel(), P)
    for p in range(P):
        for m in range(5):
            pf.set_field(O.UF, p, m, Us[p][m])
            pf.set_field(O.FF, p, m, A @ Us[p][m])
    return Us, A


def test_sweep_is_identity_on_collocation_solution():
    """Sec. 3: the SDC sweep acts as the identity on the collocation solution."""
    dim, n, nu, dt = 1, 15, 1.0, 0.02
    u0 = inputs.heat_1d(n)[0] + 0.3 * inputs.sine_mode(n, (11,), 1)
    pf = O.Pfasst(dim, n, nu, dt, 1, 5, 0, O.policy(smoother=O.RBGS, **EXACT))
    Us, _ = colloc_state(pf, dim, n, nu, dt, u0, 1)
    pf.sweep(0, 0)
    for m in range(5):
        assert pins.rel_err(pf.field(O.UF, 0, m), Us[0][m]) <= 1e-13


@pytest.mark.parametrize("k", [1, 6, 13])
def test_sweep_on_a_mode_is_the_sdc_error_map(k):
    """On one eigenmode with exact solves, one sweep maps the node values y^k
    to y^{k+1} solving (I - z Q_D) y^{k+1} = y0 + z (Q - Q_D) y^k (eq. lamdtI),
    z = dt nu mu_k, with Q_D of eq. Qbe."""
    dim, n, nu, dt = 1, 15, 1.0, 0.05
    phi = inputs.sine_mode(n, (k,), 1)
    z = dt * nu * pins.mu(n, (k,))
    s = pins.lobatto5()
    Q, Qd = pins.q_vandermonde(s), pins.q_delta(s)
    rng = np.random.default_rng(k)
    yk = np.concatenate([[1.0], rng.standard_normal(4)])
    pf = O.Pfasst(dim, n, nu, dt, 1, 5, 0, O.policy(smoother=O.JACOBI, omega=2 / 3, **EXACT))
    lam = nu * pins.mu(n, (k,))
    for m in range(5):
        pf.set_field(O.UF, 0, m, yk[m] * phi)
        pf.set_field(O.FF, 0, m, lam * yk[m] * phi)
    pf.sweep(0, 0)
    y1 = np.linalg.solve(np.eye(5) - z * Qd, np.ones(5) * yk[0] + z * (Q - Qd) @ yk)
    for m in range(5):
        got = pf.field(O.UF, 0, m)
        assert pins.rel_err(got, y1[m] * phi) <= 1e-12


@pytest.mark.parametrize("K,order,nts", [(1, 1, (8, 16)), (2, 2, (64, 128)), (3, 3, (128, 256)),
                                         (4, 4, (128, 256)), (40, 8, (2, 4))])
def test_sdc_order(K, order, nts):
    """K sweeps from the spread initial guess give order min(K, 2M) in time;
    converged 5-node Lobatto collocation has order 8 (cf. Sec. 4.1, Fig. 4).
    The non-uniform substeps leave a long pre-asymptotic range, so each K is
    measured at step counts where the slope has settled."""
    dim, n, nu, T = 1, 7, 0.5, 1.0
    phi = inputs.sine_mode(n, (1,), 1)
    lam = nu * pins.mu(n, (1,))
    errs = []
    for nt in nts:
        dt = T / nt
        pf = O.Pfasst(dim, n, nu, dt, 1, 5, 0, O.policy(smoother=O.RBGS, **EXACT))
        u = phi.copy()
        for _ in range(nt):
            pf.set_initial(u)
            for _ in range(K):
                pf.iterate()
            u = pf.field(O.UF, 0, 4)
        errs.append(np.max(np.abs(u - np.exp(lam * T) * phi)))
    slope = np.log2(errs[0] / errs[1])
    assert abs(slope - order) < 0.35, (errs, slope)


def test_fas_fixed_point():
    """Sec. 2.3: with the FAS term the coarse level reproduces the restricted
    fine collocation solution, so the coarse correction is zero and
    interpolation leaves the fine state unchanged."""
    dim, n, nu, dt, P = 1, 15, 1.0, 0.02, 2
    u0 = inputs.heat_1d(n)[0]
    pf = O.Pfasst(dim, n, nu, dt, P, 5, 3, O.policy(smoother=O.RBGS, **EXACT))
    pf.spread(u0)
    Us, _ = colloc_state(pf, dim, n, nu, dt, u0, P)
    for p in range(P):
        pf.fas_restrict(p)
    for p in range(P):
        if p > 0:
            pf.set_field(O.UC, p, 0, pf.field(O.UC, p - 1, 2))
        pf.sweep(1, p)
    for p in range(P):
        for mc in range(3):
            assert pins.rel_err(pf.field(O.UC, p, mc), pf.field(O.UCOLD, p, mc)) <= 1e-13
        pf.interpolate(p)
        for m in range(5):
            assert pins.rel_err(pf.field(O.UF, p, m), Us[p][m]) <= 1e-13
    blk, _ = pf.residual()
    assert blk <= 1e-13


@pytest.mark.parametrize("dim,n,P,cyc", [(1, 31, 4, 1), (1, 15, 3, 0), (3, 7, 3, 1)])
def test_pfasst_converges_to_composite_collocation(dim, n, P, cyc):
    """The IPFASST fixed point is the composite collocation solution of eq.
    bigPmatk_2 over the slices (dense solve), with exact or inexact solves."""
    nu, dt = 1.0, 0.01 if dim == 1 else 2e-3
    u0 = inputs.heat_1d(n)[0] if dim == 1 else inputs.random_fourier(n, 3, n_modes=4, kmax=3)[0]
    pol = O.policy(smoother=O.RBGS, cycles=cyc, tol=1e-14, stall=0.999, max_cycles=100)
    pf = O.Pfasst(dim, n, nu, dt, P, 5, 3, pol)
    pf.set_initial(u0)
    for _ in range(150):
        if pf.iterate() <= 1e-13:
            break
    A = nu * pins.lap_dense(dim, n)
    Us = pins.collocation_block(A, pins.q_vandermonde(pins.lobatto5()), dt, u0.ravel(), P)
    for p in range(P):
        for m in range(5):
            assert pins.rel_err(pf.field(O.UF, p, m).ravel(), Us[p][m]) <= 1e-11


def test_heat1d_127_end_values_match_pade_closed_form():
    """The 1D case (N=127, P=4, dt=0.01, 5/3 Lobatto, Jacobi 2/3 V(2,2), one
    V-cycle per solve) iterated to convergence: each slice's end value is
    sum_j a_j R44(dt nu mu_j)^(p+1) phi_j, R44 the (4,4) Pade approximant
    (Lobatto IIIA, eq. BT)."""
    g = pins.golden("lobatto_iiia.json")
    n, nu, dt, P = 127, 1.0, 0.01, 4
    u0, modes = inputs.heat_1d(n)
    pf = O.Pfasst(1, n, nu, dt, P, 5, 3, O.policy(smoother=O.JACOBI, omega=2 / 3, cycles=1))
    pf.set_initial(u0)
    it = 0
    while pf.iterate() > 1e-12 and it < 200:
        it += 1
    for p in range(P):
        want = sum(a * pins.pade(dt * nu * pins.mu(n, k), g["pade44_num"]) ** (p + 1)
                   * inputs.sine_mode(n, k, 1) for a, k in zip(modes.amp, modes.k))
        assert pins.rel_err(pf.field(O.UF, p, 4), want) <= 1e-11


def test_1d_decay_matches_paper_value():
    """Sec. 4.1: k = L = nu = T = 1 decays to about 5e-5 at T = 1."""
    pv = pins.golden("paper_values.json")
    n, nu, T, nt = 127, 1.0, 1.0, 10
    u = inputs.sine_mode(n, (1,), 1)
    pf = O.Pfasst(1, n, nu, T / nt, 1, 5, 0, O.policy(smoother=O.JACOBI, omega=2 / 3, **EXACT))
    for _ in range(nt):
        pf.set_initial(u)
        for _ in range(30):
            if pf.iterate() <= 1e-13:
                break
        u = pf.field(O.UF, 0, 4)
    mid = u[n // 2]      # x = 1/2
    assert abs(mid - pv["decay_T1_approx"]) <= pv["decay_T1_rel_tol"] * pv["decay_T1_approx"] + 2e-6
    assert abs(mid - np.exp(-np.pi ** 2)) <= 1e-7


def test_predictor_sweep_counts():
    """Sec. 2.4 predictor: slice p does p+1 coarse sweeps (2 solves each)."""
    n, P = 15, 4
    pf = O.Pfasst(1, n, 1.0, 0.01, P, 5, 3, O.policy(smoother=O.JACOBI, omega=2 / 3, cycles=1))
    pf.set_initial(inputs.heat_1d(n)[0])
    assert pf.vcycles(1) == 2 * sum(p + 1 for p in range(P))
    assert pf.vcycles(0) == 0
    pf.iterate()
    assert pf.vcycles(0) == 4 * P and pf.vcycles(1) == 2 * sum(p + 1 for p in range(P)) + 2 * P


def test_single_slice_pfasst_is_mlsdc():
    """P = 1: no initial-value exchange; the iteration is MLSDC (Sec. 2.3)
    and converges to the single-slice collocation solution."""
    n, nu, dt = 31, 1.0, 0.02
    u0 = inputs.heat_1d(n)[0]
    pf = O.Pfasst(1, n, nu, dt, 1, 5, 3, O.policy(smoother=O.RBGS, **EXACT))
    pf.set_initial(u0)
    for _ in range(80):
        if pf.iterate() <= 1e-13:
            break
    A = nu * pins.lap_dense(1, n)
    U = pins.collocation_block(A, pins.q_vandermonde(pins.lobatto5()), dt, u0, 1)[0]
    assert pins.rel_err(pf.field(O.UF, 0, 4), U[4]) <= 1e-12
