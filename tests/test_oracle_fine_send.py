"""Pins of the oracle's fine_send = 1 option (Sec. 2.4: the fine level
sends its end value after the sweep): slice p's new initial value at
iteration k+1 is slice p-1's end value right after its fine sweep of
iteration k, before the coarse correction reaches it.

- with one slice, or one level, nothing changes: bitwise equal to the
  default (end value after the iteration);
- iteration 1 starts from the predictor's end values either way: equal;
- iteration 2 composed from the oracle's own pinned steps (sweep, FAS
  restriction, coarse sweep, interpolation) with the node-0 values taken
  after the fine sweeps equals the option;
- the fixed point is the composite collocation solution: the converged end
  values are the (4,4) Pade closed form (Lobatto IIIA).
"""
import numpy as np

import inputs
import oracle as O
from tests import pins


def run(fs, dim=1, n=63, P=4, nc=3, iters=3, dt=0.01):
    orc = O.Pfasst(dim, n, 1.0, dt, P, 5, nc, O.policy(smoother=O.JACOBI, omega=2 / 3, cycles=1), fine_send=fs)
    u0 = inputs.heat_1d(n)[0] if dim == 1 else inputs.random_fourier(n, 31)[0]
    orc.set_initial(u0)
    res = [orc.iterate() for _ in range(iters)]
    return orc, res


def states(orc, P, nn=5):
    return [orc.field(O.UF, p, m) for p in range(P) for m in range(nn)]


def test_one_slice_and_one_level_are_unchanged():
    for kw in (dict(P=1), dict(nc=0)):
        a, ra = run(0, **kw)
        b, rb = run(1, **kw)
        assert ra == rb
        P = kw.get("P", 4)
        for x, y in zip(states(a, P), states(b, P)):
            assert np.array_equal(x, y)


def test_first_iteration_equal_second_differs():
    a, ra = run(0, iters=1)
    b, rb = run(1, iters=1)
    assert ra == rb
    for x, y in zip(states(a, 4), states(b, 4)):
        assert np.array_equal(x, y)
    a.iterate()
    b.iterate()
    d = max(np.max(np.abs(x - y)) for x, y in zip(states(a, 4), states(b, 4)))
    assert d > 1e-10


def test_second_iteration_equals_composition_from_steps():
    dim, n, P, dt, nu = 3, 15, 3, 2e-3, 1.0
    pol = O.policy(cycles=1)
    u0 = inputs.random_fourier(n, 77)[0]
    ref = O.Pfasst(dim, n, nu, dt, P, 5, 3, pol, fine_send=1)
    cmp_ = O.Pfasst(dim, n, nu, dt, P, 5, 3, pol, fine_send=0)
    for o in (ref, cmp_):
        o.set_initial(u0)
    # iteration 1: the same either way; keep the fine end values right after the sweeps
    ref.iterate()
    snap = []
    for p in range(P):
        cmp_.sweep(0, p)
    # cmp_ did only the sweeps of its iteration 1 so far: build the rest by hand
    for p in range(P):
        snap.append(cmp_.field(O.UF, p, 4))
    # (node 0 of iteration 1 was the predictor's end values: nothing to set)
    for p in range(P):
        cmp_.fas_restrict(p)
    ub_c = u0[1::2, 1::2, 1::2]
    for p in range(P):
        uc0 = ub_c if p == 0 else cmp_.field(O.UC, p - 1, 2)
        cmp_.set_field(O.UC, p, 0, uc0)
        cmp_.set_field(O.FC, p, 0, nu * O.lap(dim, uc0))
        cmp_.sweep(1, p)
    for p in range(P):
        cmp_.interpolate(p)
    for x, y in zip(states(ref, P), states(cmp_, P)):
        assert np.array_equal(x, y)
    # iteration 2: node 0 from the kept values, then the same steps
    ref.iterate()
    for p in range(1, P):
        cmp_.set_field(O.UF, p, 0, snap[p - 1])
        cmp_.set_field(O.FF, p, 0, nu * O.lap(dim, snap[p - 1]))
    for p in range(P):
        cmp_.sweep(0, p)
    for p in range(P):
        cmp_.fas_restrict(p)
    for p in range(P):
        uc0 = ub_c if p == 0 else cmp_.field(O.UC, p - 1, 2)
        cmp_.set_field(O.UC, p, 0, uc0)
        cmp_.set_field(O.FC, p, 0, nu * O.lap(dim, uc0))
        cmp_.sweep(1, p)
    for p in range(P):
        cmp_.interpolate(p)
    for x, y in zip(states(ref, P), states(cmp_, P)):
        assert np.array_equal(x, y)


def test_converges_to_the_collocation_closed_form():
    """1D, N = 127, P = 4, dt = 0.01, 5/3 Lobatto, Jacobi 2/3 V(2,2) with
    one V-cycle per solve, iterated to a block residual of 1e-12: each
    slice's end value is sum_j a_j R44(dt nu mu_j)^(p+1) phi_j."""
    g = pins.golden("lobatto_iiia.json")
    n, P, dt, nu = 127, 4, 0.01, 1.0
    u0, modes = inputs.heat_1d(n)
    orc = O.Pfasst(1, n, nu, dt, P, 5, 3, O.policy(smoother=O.JACOBI, omega=2 / 3, cycles=1), fine_send=1)
    orc.set_initial(u0)
    it = 0
    while orc.iterate() > 1e-12 and it < 200:
        it += 1
    assert it < 200
    for p in range(P):
        want = sum(a * pins.pade(dt * nu * pins.mu(n, k), g["pade44_num"]) ** (p + 1) * inputs.sine_mode(n, k, 1)
                   for a, k in zip(modes.amp, modes.k))
        assert pins.rel_err(orc.field(O.UF, p, 4), want) <= 1e-11, p
