"""Pins for the oracle's three-level hierarchy (Sec. 4.2's weak-scaling
runs: fine and middle levels with 3 uniform nodes, backward Euler on the
coarsest, coarsening by two in space on every level).

The FAS term below the middle level carries the middle level's own term
through the restriction; if it did not, the fine collocation solution
would not be a fixed point of the iteration.  So the pins are the
converged end values against the fine rule's closed-form stability
function (Norsett for uniform nodes, the Pade (4,4) form for 5 Lobatto
nodes), agreement with the two-level hierarchy's converged state, the
restricted tau against its definition evaluated here from the fields, and
fixed-point preservation from the converged state.
"""
import numpy as np
import pytest

import inputs
import oracle as O
from tests import pins
from tests.test_oracle_uniform_nodes import norsett


def converge(pf, tol=1e-13, cap=300):
    it = 0
    while pf.iterate() > tol and it < cap:
        it += 1
    return it


@pytest.mark.parametrize("fam,nf,nm,nc,fs,io", [(O.UNIFORM, 3, 3, 2, 1, 4), (O.UNIFORM, 3, 3, 2, 0, 2),
                                                (O.LOBATTO, 5, 3, 2, 0, 2), (O.UNIFORM, 5, 3, 2, 1, 4)])
def test_three_levels_converge_to_the_fine_collocation_solution(fam, nf, nm, nc, fs, io):
    """1D heat, N=31, P=4, dt=0.01, two V-cycles per solve: each slice's end
    value is sum_k a_k R(dt nu mu_k)^(p+1) phi_k."""
    n, nu, dt, P = 31, 1.0, 0.01, 4
    u0, modes = inputs.heat_1d(n)
    pf = O.Pfasst(1, n, nu, dt, P, nf, nc, O.policy(smoother=O.RBGS, cycles=2), interp_order=io, node_family=fam,
                  f_solve=fs, f_interp=fs, nodes_middle=nm)
    assert pf.ns == [31, 15, 7] and pf.nn == [nf, nm, nc]
    pf.set_initial(u0)
    assert converge(pf) < 300
    if fam == O.UNIFORM:
        M = nf - 1
        R = lambda z: norsett([m / M for m in range(1, M + 1)], z)
    else:
        g = pins.golden("lobatto_iiia.json")
        R = lambda z: pins.pade(z, g["pade44_num"])
    for p in range(P):
        want = sum(a * R(dt * nu * pins.mu(n, k)) ** (p + 1) * inputs.sine_mode(n, k, 1)
                   for a, k in zip(modes.amp, modes.k))
        assert pins.rel_err(pf.field(O.UF, p, nf - 1), want) <= 1e-11, p


def test_three_levels_reach_the_two_level_state_in_3d():
    n, P = 15, 3
    u0 = inputs.random_fourier(n, 88)[0]
    out = []
    for nm in (0, 3):
        pf = O.Pfasst(3, n, 1.0, 2e-3, P, 5, 2, O.policy(cycles=2), nodes_middle=nm)
        pf.set_initial(u0)
        assert converge(pf, 1e-13, 200) < 200
        out.append([pf.field(O.UF, p, 4) for p in range(P)])
    for p in range(P):
        assert pins.rel_err(out[1][p], out[0][p]) <= 1e-11, p


def test_restricted_tau_carries_the_middle_tau():
    """After a middle-to-coarse restriction: tau_2[mc] = R(dt sum_i
    q1_{cmap(mc),i} F_1[i] + tau_1[cmap(mc)]) - dt sum_j q2_{mc,j} F_2[j],
    with F_2 = nu L_2h U_2 and U_2 = R U_1 evaluated here."""
    n, dt, nu = 31, 3e-3, 1.0
    pf = O.Pfasst(3, n, nu, dt, 2, 5, 2, O.policy(cycles=1), nodes_middle=3)
    pf.set_initial(inputs.random_field((n,) * 3, 4))
    pf.iterate()
    p = 1
    pf.fas_restrict_level(1, p)
    _, Q1 = pf.matrices(1)
    _, Q2 = pf.matrices(2)
    cmap = [0, 2]
    inj = lambda v: v[1::2, 1::2, 1::2]
    F1 = [pf.level_field(1, O.K_F, p, i) for i in range(3)]
    U2 = [inj(pf.level_field(1, O.K_U, p, cmap[j])) for j in range(2)]
    F2 = [nu * O.lap(3, u) for u in U2]
    for mc in range(2):
        mf = cmap[mc]
        want = inj(dt * sum(Q1[mf, i] * F1[i] for i in range(3)) + pf.level_field(1, O.K_TAU, p, mf)) \
            - dt * sum(Q2[mc, j] * F2[j] for j in range(2))
        got = pf.level_field(2, O.K_TAU, p, mc)
        assert np.max(np.abs(got - want)) <= 1e-12 * max(1.0, np.max(np.abs(want))), mc
        assert pins.rel_err(pf.level_field(2, O.K_U, p, mc), U2[mc]) == 0.0


def test_converged_state_is_a_fixed_point():
    n, P = 15, 4
    pf = O.Pfasst(3, n, 1.0, 2e-3, P, 3, 2, O.policy(cycles=2), node_family=O.UNIFORM, nodes_middle=3,
                  f_solve=1, f_interp=1, interp_order=4)
    pf.set_initial(inputs.random_fourier(n, 5)[0])
    converge(pf, 1e-14, 300)
    before = [pf.field(O.UF, p, 2) for p in range(P)]
    assert pf.iterate() <= 1e-13
    for p in range(P):
        assert pins.rel_err(pf.field(O.UF, p, 2), before[p]) <= 1e-13


def test_three_level_parameters_rejected():
    with pytest.raises(ValueError):
        O.Pfasst(3, 15, 1.0, 1e-3, 2, 5, 0, O.policy(cycles=1), nodes_middle=3)   # no coarse level
    with pytest.raises(ValueError):
        O.Pfasst(3, 15, 1.0, 1e-3, 2, 5, 2, O.policy(cycles=1), nodes_middle=4)   # not a subset
    with pytest.raises(ValueError):
        O.Pfasst(3, 5, 1.0, 1e-3, 2, 5, 2, O.policy(cycles=1), nodes_middle=3)    # coarse grid too small
