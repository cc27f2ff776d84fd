"""Pins for the oracle's uniform node family: nodes m/M on the slice with a
quadrature that leaves out the left end point (the second- and fourth-order
methods of Sec. 3 and of the 3D runs in Sec. 4; M = 1 is backward Euler).

Each pin comes from outside the oracle's construction (Lagrange basis over
nodes 1..M, integrated exactly): hand-derived and textbook rules, exactness
on monomials, Norsett's closed form of a collocation method's stability
function, nilpotency of the stiff limit of the SDC iteration, and end values
of a converged heat run against that closed form.
"""
from math import factorial

import numpy as np
import pytest
from numpy.polynomial import polynomial as Pn

import inputs
import oracle as O
from tests import pins

EXACT = dict(cycles=0, tol=1e-15, stall=0.999, max_cycles=200)


def q_uniform(M):
    return O.qmat(O.uniform_nodes(M + 1), O.UNIFORM)


def test_uniform_nodes_are_exact_fractions():
    for M in (1, 2, 3, 4, 8):
        s = O.uniform_nodes(M + 1)
        assert np.array_equal(s, np.array([m / M for m in range(M + 1)]))


def test_backward_euler_and_midpoint_rules():
    """M = 1: y1 = y0 + dt f(y1) (backward Euler).  M = 2: the interpolant
    through t = 1/2 and t = 1 integrates to (3/4, -1/4) over [0, 1/2] and to
    (1, 0) over [0, 1] (the midpoint rule), derived by hand."""
    Q1, S1, d1 = q_uniform(1)
    assert np.array_equal(Q1, [[0, 0], [0, 1]]) and np.array_equal(d1, [0, 1])
    Q2, S2, d2 = q_uniform(2)
    assert np.allclose(Q2, [[0, 0, 0], [0, 0.75, -0.25], [0, 1, 0]], atol=1e-16, rtol=0)
    assert np.allclose(S2, [[0, 0.75, -0.25], [0, 0.25, 0.25]], atol=1e-16, rtol=0)
    assert np.allclose(d2, [0, 0.5, 0.5], atol=0, rtol=0)


def test_fourth_order_rule_ends_in_milnes_rule():
    """M = 4: over the whole slice the rule through nodes 1/4, 1/2, 3/4, 1 is
    Milne's open Newton-Cotes rule (2, -1, 2)/3 on the three inner nodes."""
    Q, _, d = q_uniform(4)
    assert np.allclose(Q[4], [0, 2 / 3, -1 / 3, 2 / 3, 0], atol=2e-16, rtol=0)
    assert np.allclose(d, [0, 0.25, 0.25, 0.25, 0.25], atol=0, rtol=0)


@pytest.mark.parametrize("M", [1, 2, 3, 4, 6])
def test_uniform_rule_is_exact_through_degree_M_minus_1(M):
    """Column 0 is zero and sum_i q_{m,i} s_i^k = s_m^(k+1)/(k+1) for k < M;
    degree M is not integrated exactly (node 0 takes no part)."""
    s = O.uniform_nodes(M + 1)
    Q, _, _ = q_uniform(M)
    assert np.all(Q[:, 0] == 0) and np.all(Q[0] == 0)
    for k in range(M):
        assert np.allclose(Q @ s ** k, s ** (k + 1) / (k + 1), atol=1e-15, rtol=0), k
    assert not np.allclose(Q @ s ** M, s ** (M + 1) / (M + 1), atol=1e-8, rtol=0)


def norsett(c, z):
    """Stability function of the collocation method with nodes c (Norsett):
    with N(x) = prod (x - c_i) / s!, R(z) = sum_j N^(s-j)(1) z^j /
    sum_j N^(s-j)(0) z^j."""
    s = len(c)
    N = Pn.polyfromroots(c) / factorial(s)
    der = [N]
    for _ in range(s):
        der.append(Pn.polyder(der[-1]))
    num = sum(Pn.polyval(1.0, der[s - j]) * z ** j for j in range(s + 1))
    den = sum(Pn.polyval(0.0, der[s - j]) * z ** j for j in range(s + 1))
    return num / den


def r_collocation(M, z):
    """End value of the converged rule on y' = y/dt * z: Y = 1 + z Q Y."""
    Q, _, _ = q_uniform(M)
    A = Q[1:, 1:]
    return np.linalg.solve(np.eye(M) - z * A, np.ones(M))[-1]


@pytest.mark.parametrize("M", [1, 2, 4])
def test_stability_function_matches_norsett(M):
    c = [m / M for m in range(1, M + 1)]
    for z in (0.3, -0.5, -2.0, -5.0, -20.0, -200.0, -1e4):
        assert abs(r_collocation(M, z) - norsett(c, z)) <= 2e-14 * max(1.0, abs(norsett(c, z))), z
    # second order: (1 + z/4) / (1 - 3z/4 + z^2/4), by hand
    if M == 2:
        for z in (-0.5, -7.0):
            assert abs(r_collocation(2, z) - (1 + z / 4) / (1 - 0.75 * z + z * z / 4)) <= 1e-15


@pytest.mark.parametrize("M,order", [(1, 1), (2, 2), (4, 4)])
def test_stability_function_order(M, order):
    """|R(z) - e^z| = O(z^(order+1)): halving z divides the error by about
    2^(order+1)."""
    e1 = abs(r_collocation(M, 0.04) - np.exp(0.04))
    e2 = abs(r_collocation(M, 0.02) - np.exp(0.02))
    assert abs(np.log2(e1 / e2) - (order + 1)) < 0.15, (e1, e2)


@pytest.mark.parametrize("M", [1, 2, 4])
def test_stiff_limit_of_sdc_iteration_is_nilpotent(M):
    """With backward-Euler substeps, the SDC iteration matrix
    (I - z Q_D)^-1 z (Q - Q_D) tends to I - Q_D^-1 Q as z -> -inf; for these
    rules that limit is nilpotent (its M-th power vanishes), so stiff error
    components are damped to zero (Sec. 3, damping of the uniform rules)."""
    Q, _, d = q_uniform(M)
    A = Q[1:, 1:]
    QD = np.tril(np.ones((M, M))) * d[1:][None, :]
    E = np.eye(M) - np.linalg.solve(QD, A)
    assert np.linalg.norm(np.linalg.matrix_power(E, M)) <= 1e-13
    # not so for the 5-node Lobatto rule: its stiff limit damps by about 0.68
    QL, _, dL = O.qmat(O.lobatto_nodes(5))
    QDL = np.tril(np.ones((4, 4))) * dL[1:][None, :]
    EL = np.eye(4) - np.linalg.solve(QDL, QL[1:, 1:])
    assert max(abs(np.linalg.eigvals(EL))) > 0.5


@pytest.mark.parametrize("nf,nc", [(5, 3), (3, 2)])
def test_heat1d_uniform_end_values_match_norsett(nf, nc):
    """1D heat, N=31, P=4, dt=0.01, uniform nodes (fine M = nf-1, coarse
    M = nc-1), one Jacobi V-cycle per solve, iterated to convergence: each
    slice's end value is sum_k a_k R(dt nu mu_k)^(p+1) phi_k with R from
    Norsett's formula for the fine nodes."""
    n, nu, dt, P = 31, 1.0, 0.01, 4
    u0, modes = inputs.heat_1d(n)
    pf = O.Pfasst(1, n, nu, dt, P, nf, nc, O.policy(smoother=O.JACOBI, omega=2 / 3, cycles=1),
                  node_family=O.UNIFORM)
    pf.set_initial(u0)
    it = 0
    while pf.iterate() > 1e-13 and it < 300:
        it += 1
    M = nf - 1
    c = [m / M for m in range(1, M + 1)]
    for p in range(P):
        want = sum(a * norsett(c, dt * nu * pins.mu(n, k)) ** (p + 1) * inputs.sine_mode(n, k, 1)
                   for a, k in zip(modes.amp, modes.k))
        assert pins.rel_err(pf.field(O.UF, p, M), want) <= 1e-11, p


def test_uniform_nodes_reach_fourth_order_in_time():
    """Converged 4-substep rule over T = 1 on one mode: the global error
    falls by about 2^4 when the step halves."""
    dim, n, nu, T = 1, 7, 0.5, 1.0
    phi = inputs.sine_mode(n, (1,), 1)
    lam = nu * pins.mu(n, (1,))
    errs = []
    for nt in (16, 32):
        pf = O.Pfasst(dim, n, nu, T / nt, 1, 5, 0, O.policy(smoother=O.RBGS, **EXACT), node_family=O.UNIFORM)
        u = phi.copy()
        for _ in range(nt):
            pf.set_initial(u)
            for _ in range(60):
                if pf.iterate() <= 1e-14:
                    break
            u = pf.field(O.UF, 0, 4)
        errs.append(np.max(np.abs(u - np.exp(lam * T) * phi)))
    assert abs(np.log2(errs[0] / errs[1]) - 4) < 0.3, errs
