"""Parity of the two F options with the FP64 oracle through the C-ABI:
f_solve (F at a node from its implicit solve, (U - b)/(dt d_m)) and
f_interp (the coarse F change interpolated onto the fine F values instead
of re-evaluating F), alone and together, with Lobatto and uniform nodes,
both stencil orders, d-linear and cubic interpolation, pipelined slice
groups, full solves and the mixed-precision solve.

Bars as in test_gpu_parity, with F's amplification of a U difference
taken as the larger of |nu L_h|_inf and 1/(dt d_min): F from a solve
divides U - b by dt d_m."""
import os

import numpy as np
import pytest

import inputs
import oracle as O
from tests import pins
from tests.test_gpu_parity import TOL, compare_state, make, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible ROCm device"
    from paper_1407_6486_amd import pfmg
    return pfmg


def lnorm_eff(orc, so):
    """Amplification factor of a U difference into F, in units of
    dim nu (n+1)^2 (the form f_tol and tau_bar take it in)."""
    ln = 64.0 / 12.0 if so == 4 else 4.0
    s, _ = orc.matrices(0)
    dmin = float(np.min(np.diff(s)))
    return max(ln, 1.0 / (orc.prm.dt * dmin * orc.dim * orc.prm.nu * (orc.n + 1) ** 2))


#         dim  n   P  family          nf nc fs fi interp stencil cycles
CASES = [(3, 31, 4, O.UNIFORM, 3, 2, 1, 1, 4, 2, 2),
         (3, 31, 3, O.LOBATTO, 5, 3, 1, 0, 2, 2, 1),
         (3, 31, 8, O.LOBATTO, 5, 3, 0, 1, 2, 2, 1),
         (3, 31, 4, O.UNIFORM, 5, 3, 1, 1, 4, 4, 2),
         (3, 15, 16, O.LOBATTO, 5, 3, 1, 1, 2, 2, 2),
         (1, 63, 4, O.UNIFORM, 5, 3, 1, 1, 4, 2, 2),
         (3, 15, 3, O.LOBATTO, 5, 3, 1, 1, 2, 2, 0),
         (3, 31, 1, O.UNIFORM, 3, 0, 1, 0, 2, 2, 2)]


@pytest.mark.parametrize("dim,n,P,fam,nf,nc,fs,fi,io,so,cycles", CASES)
def test_pfasst_f_options_match_oracle(pf, dim, n, P, fam, nf, nc, fs, fi, io, so, cycles):
    say(f"F options fs={fs} fi={fi}: dim={dim} n={n} P={P} family={fam} nodes {nf}/{nc} interp {io} "
        f"stencil {so} cycles {cycles}")
    nu, dt = (1.0 / 3.0, 1.0 / 24) if fam == O.UNIFORM else (1.0, 1e-3)
    kw = dict(vcycles_per_solve=cycles)
    pol = O.policy(cycles=cycles)
    if cycles == 0:
        kw.update(mg_tol=1e-12, mg_stall=0.75, mg_max_cycles=50)
        pol = O.policy(cycles=0, tol=1e-12, stall=0.75, max_cycles=50)
    c = make(pf, dim=dim, n=n, n_slices=P, nu=nu, dt=dt, nodes_fine=nf, nodes_coarse=nc, node_family=fam,
             interp_order=io, stencil_order=so, f_solve=fs, f_interp=fi, **kw)
    orc = O.Pfasst(dim, n, nu, dt, P, nf, nc, pol, interp_order=io, node_family=fam, stencil_order=so,
                   f_solve=fs, f_interp=fi)
    if dim == 3:
        u0 = inputs.sine_mode(n, (1, 1, 1), 3) + 0.1 * inputs.random_fourier(n, 77)[0]
    else:
        u0, _ = inputs.heat_1d(n)
    c.set_initial(u0)
    orc.set_initial(u0)
    ln = lnorm_eff(orc, so)
    two = nc > 0
    compare_state(c, orc, P, two_levels=two, lnorm_f=ln)
    for k in range(3):
        r_gpu = c.pfasst_iter()
        r_or = orc.iterate()
        assert abs(r_gpu - r_or) <= 1e-9 * r_or, (k, r_gpu, r_or)
        np.testing.assert_allclose(c.residual(), orc.residual()[1], rtol=1e-9)
        compare_state(c, orc, P, two_levels=two, lnorm_f=ln)
    assert c.vcycle_count(0) == orc.vcycles(0)
    if two:
        assert c.vcycle_count(1) == orc.vcycles(1)


def test_f_options_mixed_precision_track_oracle_mixed(pf):
    n, P = 31, 4
    say(f"F options with the mixed-precision solve n={n} P={P}")
    c = pf.Context(pf.pfmg_default_params(dim=3, n=n, n_slices=P, precision=pf.MIXED, f_solve=1, f_interp=1))
    orc = O.Pfasst(3, n, 1.0, 1e-3, P, 5, 3, O.policy(cycles=1, mixed=1), f_solve=1, f_interp=1)
    u0, _ = inputs.random_fourier(n, 1407)
    c.set_initial(u0)
    orc.set_initial(u0)
    for k in range(2):
        r_gpu, r_or = c.pfasst_iter(), orc.iterate()
        assert abs(r_gpu - r_or) <= 1e-3 * r_or, (k, r_gpu, r_or)
        for p in range(P):
            assert pins.rel_err(c.get(O.UF, p, 4), orc.field(O.UF, p, 4)) <= 1e-5, (k, p)


@pytest.mark.parametrize("n,P,nf,nc,fam", [(31, 4, 5, 3, O.LOBATTO), (31, 8, 3, 2, O.UNIFORM)])
def test_f_options_fused_launches_match_separate(pf, n, P, nf, nc, fam):
    """With both options the fused sweep start (node 0's F evaluated from
    the sent value) gives the separate launches' state."""
    say(f"F options, fused vs separate sweep launches n={n} P={P} nodes {nf}/{nc}")
    u0, _ = inputs.random_fourier(n, 616)
    states = {}
    for fused in ("1", "0"):
        os.environ["PFMG_FUSED_SDC"] = fused
        try:
            c = make(pf, n=n, n_slices=P, nodes_fine=nf, nodes_coarse=nc, node_family=fam, dt=2e-3,
                     f_solve=1, f_interp=1, vcycles_per_solve=2)
        finally:
            del os.environ["PFMG_FUSED_SDC"]
        c.set_initial(u0)
        res = [c.pfasst_iter() for _ in range(3)]
        states[fused] = (res, [c.get(O.UF, p, nf - 1) for p in range(P)], [c.get(O.FC, p, 0) for p in range(P)])
        c.close()
    (r1, f1, g1), (r0, f0, g0) = states["1"], states["0"]
    assert all(abs(a - b) <= 1e-13 * a for a, b in zip(r1, r0)), (r1, r0)
    for p in range(P):
        assert pins.rel_err(f1[p], f0[p]) <= 1e-14, p
        assert pins.rel_err(g1[p], g0[p]) <= 1e-13, p


def test_table1_second_order_two_level_converges_like_single_level(pf):
    """Sec. 4.3's observation on the GPU path: uniform 3/2 nodes, 63^3,
    nu = 1/3, dt = 1/128, two V(2,2) cycles per solve, cubic interpolation,
    relative residual 1e-9: with both options IMLSDC needs at most one
    iteration more than ISDC."""
    n = 63
    u0 = inputs.sine_mode(n, (1, 1, 1), 3)
    its = {}
    for nc, fs, fi in ((0, 0, 0), (2, 1, 1)):
        c = make(pf, n=n, n_slices=1, nu=1.0 / 3.0, dt=1.0 / 128, nodes_fine=3, nodes_coarse=nc,
                 node_family=pf.NODES_UNIFORM, interp_order=4, vcycles_per_solve=2, f_solve=fs, f_interp=fi)
        c.set_initial(u0)
        k = 0
        while k < 40:
            k += 1
            if c.pfasst_iter() <= 1e-9:
                break
        its[nc] = k
        c.close()
    say(f"ISDC {its[0]} iterations, IMLSDC with both options {its[2]}")
    assert its[2] <= its[0] + 1, its


def test_absolute_residual_matches_oracle(pf):
    """residual_abs = 1: per-slice and block residuals without the
    normalisation, and run_block stopping on the absolute bound."""
    n, P = 31, 4
    say(f"absolute residual n={n} P={P}")
    u0, _ = inputs.random_fourier(n, 1409)
    c = make(pf, n=n, n_slices=P, residual_abs=1, f_solve=1, f_interp=1, pfasst_tol=1e-7, pfasst_max_iter=60)
    orc = O.Pfasst(3, n, 1.0, 1e-3, P, 5, 3, O.policy(cycles=1), f_solve=1, f_interp=1, residual_abs=1)
    c.set_initial(u0)
    orc.set_initial(u0)
    for k in range(2):
        r_gpu, r_or = c.pfasst_iter(), orc.iterate()
        assert abs(r_gpu - r_or) <= 1e-9 * r_or, (k, r_gpu, r_or)
        np.testing.assert_allclose(c.residual(), orc.residual()[1], rtol=1e-9)
    st, it, res = c.run_block(u0)
    assert st == pf.OK and res <= 1e-7
    orc.set_initial(u0)
    k = 0
    while k < 60:
        k += 1
        if orc.iterate() <= 1e-7:
            break
    assert it == k, (it, k)


def resid_bar(c, orc, P, lnorm):
    """Absolute bar for the (absolute) collocation residual
    u0 - U[m] + dt sum_i q_{m,i} nu L_h U[i]: both sides evaluate it from
    their own U, so the max-norm difference du of U (measured, at least 4
    ulps of U) reaches it amplified by 2 + dt max_m sum_i |q_{m,i}| |nu L_h|;
    four times that, plus a few ulps of the summed terms."""
    eps = np.finfo(np.float64).eps
    du = umax = 0.0
    for p in range(P):
        for m in range(orc.nn[0]):
            u_or = orc.field(O.UF, p, m)
            du = max(du, float(np.max(np.abs(c.get(O.UF, p, m) - u_or))))
            umax = max(umax, float(np.max(np.abs(u_or))))
    du = max(du, 4 * eps * umax)
    _, Q = orc.matrices(0)
    Lh = lnorm * orc.dim * orc.prm.nu * (orc.n + 1) ** 2
    amp = 2.0 + orc.prm.dt * np.abs(Q).sum(axis=1).max() * Lh
    return 4 * du * amp + 16 * eps * umax * amp


def test_table1_127_second_order_matches_oracle(pf):
    """The Table 1 form's launch configuration at its full size: 127^3,
    uniform 3/2 nodes, nu = 1/3, dt = 1/128, two V-cycles per solve, cubic
    interpolation, both F options, absolute residual; two slices, the
    predictor and two iterations."""
    n, P = 127, 2
    say(f"Table 1 configuration at n={n}, P={P}: predictor + 2 iterations")
    nu, dt = 1.0 / 3.0, 1.0 / 128
    c = make(pf, n=n, n_slices=P, nu=nu, dt=dt, nodes_fine=3, nodes_coarse=2, node_family=pf.NODES_UNIFORM,
             interp_order=4, vcycles_per_solve=2, f_solve=1, f_interp=1, residual_abs=1)
    orc = O.Pfasst(3, n, nu, dt, P, 3, 2, O.policy(cycles=2), interp_order=4, node_family=O.UNIFORM,
                   f_solve=1, f_interp=1, residual_abs=1)
    u0 = inputs.sine_mode(n, (1, 1, 1), 3)
    c.set_initial(u0)
    orc.set_initial(u0)
    ln = lnorm_eff(orc, 2)
    compare_state(c, orc, P, lnorm_f=ln)
    for k in range(2):
        r_gpu, r_or = c.pfasst_iter(), orc.iterate()
        bar = resid_bar(c, orc, P, ln)
        assert abs(r_gpu - r_or) <= bar, (k, r_gpu, r_or, bar)
        np.testing.assert_allclose(c.residual(), orc.residual()[1], rtol=0, atol=bar)
        compare_state(c, orc, P, lnorm_f=ln)
