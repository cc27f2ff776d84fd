"""Pins for the oracle's two options on how F values are formed (the paper
leaves both open; Sec. 4.3's runs use two V-cycles per solve, where they
matter):

  f_solve   F at a node after its implicit-Euler solve is (U - b)/(dt d_m),
            the value the substep implies; equal to nu L U for an exact
            solve.
  f_interp  after the coarse correction the fine F values take the coarse
            F change, interpolated like U's, instead of being re-evaluated.

Neither changes the fixed point (the collocation solution), only the path
to it; the collocation residual re-evaluates F(U) whenever either is set.
The pins: equality with the plain form for exact solves, the residual
against its definition evaluated here from U alone, the interpolated F
change against nu L_2h of the coarse U change (the coarse F of a plain
sweep), converged end values against Norsett's closed form, and the
two-level iteration count against the single-level one (Sec. 4.3: IMLSDC
needs about as many iterations as ISDC).
"""
import numpy as np
import pytest

import inputs
import oracle as O
from tests import pins
from tests.test_oracle_uniform_nodes import norsett

EXACT = dict(cycles=0, tol=1e-14, stall=0.999, max_cycles=100)


def test_exact_solves_make_f_solve_the_plain_form():
    u0 = inputs.random_field((15,) * 3, 77)
    runs = []
    for fs in (0, 1):
        pf = O.Pfasst(3, 15, 1.0, 2e-3, 3, 5, 3, O.policy(**EXACT), f_solve=fs)
        pf.set_initial(u0)
        for _ in range(3):
            pf.iterate()
        runs.append(pf)
    for p in range(3):
        for m in range(5):
            assert pins.rel_err(runs[1].field(O.UF, p, m), runs[0].field(O.UF, p, m)) <= 1e-11
            assert pins.rel_err(runs[1].field(O.FF, p, m), runs[0].field(O.FF, p, m)) <= 1e-9


@pytest.mark.parametrize("fam", [O.LOBATTO, O.UNIFORM])
def test_residual_is_the_collocation_residual_of_U(fam):
    """eq. resid with F(U) = nu L_h U evaluated here from the U fields."""
    n, nu, dt, P = 15, 1.0, 3e-3, 3
    pf = O.Pfasst(3, n, nu, dt, P, 5, 3, O.policy(cycles=1), node_family=fam, f_solve=1, f_interp=1)
    u0 = inputs.random_field((n,) * 3, 5)
    pf.set_initial(u0)
    pf.iterate()
    blk, per = pf.residual()
    Q = O.qmat(O.nodes(5, fam), fam)[0]
    want = []
    for p in range(P):
        a = u0 if p == 0 else pf.field(O.UF, p - 1, 4)
        U = [pf.field(O.UF, p, m) for m in range(5)]
        F = [nu * O.lap(3, u) for u in U]
        r = max(np.max(np.abs(a - U[m] + dt * sum(Q[m, i] * F[i] for i in range(5)))) for m in range(5))
        want.append(r / np.max(np.abs(a)))
        # the stored F is not F(U) mid-iteration
        assert pins.rel_err(pf.field(O.FF, p, 2), F[2]) > 1e-8
    assert np.allclose(per, want, rtol=1e-12, atol=0)
    assert blk == max(per)


def test_interpolated_F_change_is_the_coarse_operator_on_the_U_change():
    """f_interp with plain coarse F (f_solve = 0): the fine F change at
    node m is P_s of sum_mc l_{m,mc} nu L_2h (U_c - U_c^old)[mc]."""
    n, nu, dt = 31, 1.0, 4e-3
    pf = O.Pfasst(3, n, nu, dt, 2, 5, 3, O.policy(cycles=2), f_interp=1)
    pf.spread(inputs.random_field((n,) * 3, 9))
    sf, sc = O.nodes(5), O.nodes(3)
    Lt = O.interp_matrix(sf, sc)
    for p in range(2):
        pf.sweep(0, p)
        pf.fas_restrict(p)
        pf.sweep(1, p)
        before = [pf.field(O.FF, p, m) for m in range(5)]
        dU = [pf.field(O.UC, p, j) - pf.field(O.UCOLD, p, j) for j in range(3)]
        assert max(np.max(np.abs(d)) for d in dU) > 1e-6
        pf.interpolate(p)
        for m in range(5):
            dF = sum(Lt[m, j] * nu * O.lap(3, dU[j]) for j in range(3))
            want = O.prolong_add(3, dF, np.zeros((n,) * 3))
            got = pf.field(O.FF, p, m) - before[m]
            assert np.max(np.abs(got - want)) <= 1e-10 * max(1.0, np.max(np.abs(want))), m


@pytest.mark.parametrize("fs,fi", [(1, 1), (1, 0), (0, 1)])
def test_converged_end_values_are_unchanged(fs, fi):
    """1D heat, N=31, P=4, dt=0.01, uniform 5/3 nodes, two V-cycles per
    solve, iterated to convergence: end values from Norsett's formula."""
    n, nu, dt, P = 31, 1.0, 0.01, 4
    u0, modes = inputs.heat_1d(n)
    pf = O.Pfasst(1, n, nu, dt, P, 5, 3, O.policy(smoother=O.RBGS, cycles=2), interp_order=4,
                  node_family=O.UNIFORM, f_solve=fs, f_interp=fi)
    pf.set_initial(u0)
    it = 0
    while pf.iterate() > 1e-13 and it < 300:
        it += 1
    c = [0.25, 0.5, 0.75, 1.0]
    for p in range(P):
        want = sum(a * norsett(c, dt * nu * pins.mu(n, k)) ** (p + 1) * inputs.sine_mode(n, k, 1)
                   for a, k in zip(modes.amp, modes.k))
        assert pins.rel_err(pf.field(O.UF, p, 4), want) <= 1e-11, p


def iterations(nc, fs, fi, n=31, tol=1e-9):
    pf = O.Pfasst(3, n, 1.0 / 3.0, 1.0 / 128, 1, 3, nc, O.policy(cycles=2), interp_order=4,
                  node_family=O.UNIFORM, f_solve=fs, f_interp=fi)
    pf.set_initial(inputs.sine_mode(n, (1, 1, 1), 3))
    for k in range(1, 60):
        if pf.iterate() <= tol:
            return k
    return 60


def test_two_level_needs_no_more_iterations_than_single_level():
    """Second order in time (uniform 3/2 nodes), 31^3, dt = 1/128, nu = 1/3,
    two V(2,2) cycles per solve: with both options IMLSDC needs at most
    ISDC's iterations; with neither it needs more."""
    isdc = iterations(0, 0, 0)
    both = iterations(2, 1, 1)
    plain = iterations(2, 0, 0)
    assert both <= isdc < plain, (both, isdc, plain)


def test_options_rejected_outside_0_1():
    with pytest.raises(ValueError):
        O.Pfasst(3, 15, 1.0, 1e-3, 2, 5, 3, O.policy(cycles=1), f_solve=2)
    with pytest.raises(ValueError):
        O.Pfasst(3, 15, 1.0, 1e-3, 2, 5, 3, O.policy(cycles=1), f_interp=-1)


def test_absolute_residual_is_relative_times_initial_norm():
    """residual_abs: each slice's residual is the plain max-norm of eq.
    resid, i.e. the relative one times |U0_p|_inf (U0_p from the fields)."""
    n, P = 15, 4
    u0 = inputs.random_fourier(n, 31)[0]
    runs = []
    for ra in (0, 1):
        pf = O.Pfasst(3, n, 1.0, 2e-3, P, 5, 3, O.policy(cycles=1), residual_abs=ra)
        pf.set_initial(u0)
        pf.iterate()
        runs.append(pf)
    _, rel = runs[0].residual()
    blk, ab = runs[1].residual()
    norms = [np.max(np.abs(u0))] + [np.max(np.abs(runs[0].field(O.UF, p - 1, 4))) for p in range(1, P)]
    assert np.allclose(ab, rel * np.array(norms), rtol=1e-13, atol=0)
    assert blk == max(ab) and not np.allclose(ab, rel)
    with pytest.raises(ValueError):
        O.Pfasst(3, 15, 1.0, 1e-3, 2, 5, 3, O.policy(cycles=1), residual_abs=2)
