"""Parity of the fourth-order fine level and the cubic PFASST interpolation
(the paper's fourth-order runs, Sec. 4.3) with the FP64 oracle, through the
C-ABI.  Bars as in test_gpu_parity: U-type arrays within 1e-12 relative;
F within that bar times |nu L4|_inf |U| / |F| (L4's row sum is 64/12 per
axis over h^2); tau by the propagated bound of tau_bar.
"""
import numpy as np
import pytest

import inputs
import oracle as O
from tests import pins
from tests.test_gpu_parity import TOL, compare_state, make, say, smoother_args

pytestmark = pytest.mark.gpu
L4NORM = 64.0 / 12.0


@pytest.fixture(scope="module")
def pf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible ROCm device"
    from paper_1407_6486_amd import pfmg
    return pfmg


@pytest.mark.parametrize("dim,n,sm,cycles", [(3, 15, "rb", 1), (3, 31, "rb", 2), (3, 31, "jac", 1), (3, 63, "rb", 1),
                                             (3, 7, "rb", 1), (1, 63, "jac", 2), (1, 3, "rb", 1)])
def test_vcycle4_matches_oracle(pf, dim, n, sm, cycles):
    say(f"vcycle4 dim={dim} n={n} smoother={sm} cycles={cycles}")
    psm, osm, om = smoother_args(pf, sm)
    c = make(pf, dim=dim, n=n, n_slices=1, nodes_coarse=0, smoother=psm, omega=om, stencil_order=4)
    alpha = 3.0 / (n + 1) ** 2
    b = inputs.random_field((n,) * dim, 500 + n)
    u0 = inputs.random_field((n,) * dim, 600 + n)
    u_gpu, st, rr, nc = c.vcycle(alpha, b, u0, cycles)
    assert st == pf.OK and nc == cycles
    u_or = u0.copy()
    for _ in range(cycles):
        u_or = O.vcycle4(dim, alpha, b, u_or, osm, om)
    assert pins.rel_err(u_gpu.cpu().numpy(), u_or) <= TOL
    r_or = np.max(np.abs(O.resid4(dim, alpha, b, u_or))) / np.max(np.abs(b))
    assert abs(rr - r_or) <= 1e-9 * r_or + 1e-15


@pytest.mark.parametrize("dim,n,sm", [(3, 31, "rb"), (1, 63, "jac")])
def test_full_solve4_matches_oracle(pf, dim, n, sm):
    say(f"full solve4 dim={dim} n={n} smoother={sm}")
    psm, osm, om = smoother_args(pf, sm)
    c = make(pf, dim=dim, n=n, n_slices=1, nodes_coarse=0, smoother=psm, omega=om, stencil_order=4,
             mg_tol=1e-12, mg_stall=0.75, mg_max_cycles=50)
    alpha = 5.0 / (n + 1) ** 2
    b = inputs.random_field((n,) * dim, 700 + n)
    u_gpu, st, rr, nc = c.vcycle(alpha, b, np.zeros_like(b), 0)
    u_or, nc_or, rr_or = O.mg_solve4(dim, alpha, b, np.zeros_like(b), O.policy(smoother=osm, omega=om, cycles=0))
    assert nc == nc_or and st in (pf.OK, pf.STALLED)
    assert pins.rel_err(u_gpu.cpu().numpy(), u_or) <= TOL


@pytest.mark.parametrize("n,P,fam,so,io,cycles", [(31, 4, 1, 4, 4, 2), (31, 3, 0, 4, 4, 1), (31, 4, 1, 2, 4, 2),
                                                  (15, 8, 1, 4, 4, 2), (63, 2, 0, 4, 2, 1)])
def test_pfasst4_matches_oracle(pf, n, P, fam, so, io, cycles):
    """IPFASST with the fourth-order fine level and/or cubic spatial
    interpolation: predictor and three iterations (P = 8: pipelined
    groups)."""
    say(f"PFASST stencil {so} interp {io} family {fam} n={n} P={P} cycles={cycles}")
    nu, dt = 1.0 / 3.0, 1.0 / 24
    c = make(pf, dim=3, n=n, n_slices=P, nu=nu, dt=dt, node_family=fam, stencil_order=so, interp_order=io,
             vcycles_per_solve=cycles)
    orc = O.Pfasst(3, n, nu, dt, P, 5, 3, O.policy(cycles=cycles), interp_order=io, node_family=fam,
                   stencil_order=so)
    u0 = inputs.sine_mode(n, (1, 1, 1), 3) + 0.1 * inputs.sine_mode(n, (3, 2, 5), 3)
    c.set_initial(u0)
    orc.set_initial(u0)
    ln = L4NORM if so == 4 else 4.0
    compare_state(c, orc, P, lnorm_f=ln)
    for k in range(3):
        r_gpu = c.pfasst_iter()
        r_or = orc.iterate()
        assert abs(r_gpu - r_or) <= 1e-9 * r_or, (k, r_gpu, r_or)
        compare_state(c, orc, P, lnorm_f=ln)
    assert c.vcycle_count(0) == orc.vcycles(0) and c.vcycle_count(1) == orc.vcycles(1)


@pytest.mark.parametrize("fi", [0, 1])
def test_cubic_interpolation_255_matches_oracle(pf, fi):
    """The widest cubic-interpolation launch (fine 255^3, 256-lane rows):
    one slice, uniform 3/2 nodes, so that the predictor's interpolation
    moves U (and, with f_interp, F in the same launch) of every fine node;
    every field after the predictor and one iteration."""
    from tests.test_gpu_f_options import lnorm_eff
    say(f"cubic interpolation at 255^3, f_interp {fi}")
    n, P, nu, dt = 255, 1, 1.0 / 3.0, 1.0 / 64
    c = make(pf, dim=3, n=n, n_slices=P, nu=nu, dt=dt, nodes_fine=3, nodes_coarse=2, node_family=pf.NODES_UNIFORM,
             interp_order=4, f_solve=fi, f_interp=fi, vcycles_per_solve=1)
    orc = O.Pfasst(3, n, nu, dt, P, 3, 2, O.policy(cycles=1), interp_order=4, node_family=O.UNIFORM, f_solve=fi,
                   f_interp=fi)
    u0 = inputs.sine_mode(n, (1, 1, 1), 3) + 0.1 * inputs.sine_mode(n, (7, 3, 11), 3)
    c.set_initial(u0)
    orc.set_initial(u0)
    ln = lnorm_eff(orc, 2)
    compare_state(c, orc, P, lnorm_f=ln)
    r_gpu, r_or = c.pfasst_iter(), orc.iterate()
    assert abs(r_gpu - r_or) <= 1e-9 * r_or + 1e-15, (r_gpu, r_or)
    compare_state(c, orc, P, lnorm_f=ln)
