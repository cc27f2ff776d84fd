"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Bar: FP64 results within 1e-12 relative (max-norm of the difference over
the max-norm of the oracle's array) of the oracle on the same seeded
inputs.  Sizes span several 64x4 tiles and ragged tails (n = 31, 63, 95,
127), the degenerate grids (n = 1, 3, 5: coarsest solves with n in {1, 2}),
one and several slices, both smoothers, fixed and full solves.
"""
import sys

import numpy as np
import pytest

import inputs
import oracle as O
from tests import pins

pytestmark = pytest.mark.gpu
TOL = 1e-12


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible ROCm device"
    from paper_1407_6486_amd import pfmg
    return pfmg


def make(pf, **kw):
    return pf.Context(pf.pfmg_default_params(**kw))


def smoother_args(pf, sm):
    return (pf.SMOOTH_JACOBI, O.JACOBI, 2.0 / 3.0) if sm == "jac" else (pf.SMOOTH_RBGS, O.RBGS, 1.0)


# ---------------------------------------------------------------- V-cycles
@pytest.mark.parametrize("dim,n,sm,cycles", [
    (1, 127, "jac", 1), (1, 95, "jac", 2), (1, 5, "rb", 1), (1, 1, "jac", 1),
    (3, 1, "rb", 1), (3, 3, "rb", 1), (3, 5, "jac", 2), (3, 15, "rb", 1), (3, 31, "rb", 2),
    (3, 63, "jac", 1), (3, 95, "rb", 1), (3, 127, "rb", 1), (3, 127, "jac", 1)])
def test_vcycle_matches_oracle(pf, dim, n, sm, cycles):
    say(f"vcycle dim={dim} n={n} smoother={sm} cycles={cycles}")
    psm, osm, om = smoother_args(pf, sm)
    c = make(pf, dim=dim, n=n, n_slices=1, nodes_coarse=0, smoother=psm, omega=om)
    alpha = 3.0 / (n + 1) ** 2
    b = inputs.random_field((n,) * dim, 100 + n)
    u0 = inputs.random_field((n,) * dim, 200 + n)
    u_gpu, st, rr, nc = c.vcycle(alpha, b, u0, cycles)
    assert st == pf.OK and nc == cycles
    u_or = u0.copy()
    for _ in range(cycles):
        u_or = O.vcycle(dim, alpha, b, u_or, osm, om)
    assert pins.rel_err(u_gpu.cpu().numpy(), u_or) <= TOL
    r_or = np.max(np.abs(O.resid(dim, alpha, b, u_or))) / np.max(np.abs(b))
    assert abs(rr - r_or) <= 1e-10 * r_or + 1e-15


# Rows per workgroup that select each compiled one-pass sweep: row lanes
# (n rounded up to 64) -> ty values; rows per thread = ceil((ty + 2) /
# (threads / lanes)) gives 1, 2, 3, 5, 6 (64 lanes), 2, 3, 5, 6 (128) and 3,
# 4, 6 (256) with 256 threads, 1, 2, 3 / 2, 3 / 3 with 512 (a row count
# below a compiled one runs the next one up).
# (8 at 128 lanes and 8, 16 at 64 lanes with 512 threads, 2 at 64 lanes
# with 256: the shapes with compile-time row counts)
SWEEP_TY = {256: {64: [2, 4, 8, 14, 22], 128: [2, 4, 8, 10], 256: [1, 2, 4]},
            512: {64: [6, 8, 14, 16, 22], 128: [2, 6, 8, 10], 256: [4]}}
SWEEP_ZC = [5, 7, 3, 16, 9, 64, 2, 31]


def sweep_cases():
    for nt, by_lanes in SWEEP_TY.items():
        for top in (63, 127, 255):
            for i in range(len(by_lanes[(top + 63) // 64 * 64])):
                yield nt, top, i


@pytest.mark.parametrize("nt,n,i", list(sweep_cases()))
def test_vcycle_every_sweep_shape_matches_oracle(pf, nt, n, i):
    """Each level's one-pass sweep pinned to a shape (ragged row tiles and
    z-chunks; the top level from a given guess, the coarser ones from zero)."""
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    levels, m = [], n
    while m >= 31:
        levels.append(m)
        m = (m - 1) // 2
    pins_set = {}
    for d, lv in enumerate(levels):
        tys = SWEEP_TY[nt][(lv + 63) // 64 * 64]
        pins_set[f"{arch}/rbgs/f64/{lv}x1"] = (2 if nt == 512 else 1, tys[(i + d) % len(tys)],
                                                SWEEP_ZC[(i + 2 * d + lv) % len(SWEEP_ZC)])
    say(f"vcycle sweep shapes nt={nt} n={n} pins={pins_set}")
    try:
        for key, (f, ty, zc) in pins_set.items():
            pf.pfmg_tune_set(key, f, ty, zc)
        c = make(pf, dim=3, n=n, n_slices=1, nodes_coarse=0, smoother=pf.SMOOTH_RBGS, omega=1.0)
        alpha = 3.0 / (n + 1) ** 2
        b = inputs.random_field((n,) * 3, 300 + n + i)
        u0 = inputs.random_field((n,) * 3, 400 + n + i)
        c.timing_enable(f"rbgs@{n}")
        u_gpu, st, rr, nc = c.vcycle(alpha, b, u0, 1)
        launches, _, nbytes = c.timing_read()
        c.timing_enable(None, False)
    finally:
        for key in pins_set:
            pf.pfmg_tune_set(key, -1)
    assert st == pf.OK and nc == 1
    # the one-pass kernel ran on the top level: 24 bytes a point a launch
    assert launches > 0 and nbytes == launches * 24 * n ** 3
    u_or = O.vcycle(3, alpha, b, u0.copy(), O.RBGS, 1.0)
    assert pins.rel_err(u_gpu.cpu().numpy(), u_or) <= TOL


def test_one_and_two_barrier_sweeps_agree(pf, monkeypatch):
    """The 127^3 sweep shape (128 lanes, 8 rows, 512 threads) with one
    barrier per z-step and with two: the same operations in the same order,
    so the V-cycles agree bitwise, and both match the oracle."""
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    n = 127
    key = f"{arch}/rbgs/f64/{n}x1"
    alpha = 3.0 / (n + 1) ** 2
    b = inputs.random_field((n,) * 3, 901)
    u0 = inputs.random_field((n,) * 3, 902)
    out = {}
    try:
        pf.pfmg_tune_set(key, 2, 8, 11)
        for flag in ("1", "0"):
            say(f"127^3 sweep, PFMG_SWEEP_1B={flag}")
            monkeypatch.setenv("PFMG_SWEEP_1B", flag)
            c = make(pf, dim=3, n=n, n_slices=1, nodes_coarse=0, smoother=pf.SMOOTH_RBGS, omega=1.0)
            u_gpu, st, rr, nc = c.vcycle(alpha, b, u0, 1)
            assert st == pf.OK and nc == 1
            out[flag] = u_gpu.cpu().numpy()
    finally:
        pf.pfmg_tune_set(key, -1)
    assert np.array_equal(out["1"], out["0"])
    u_or = O.vcycle(3, alpha, b, u0.copy(), O.RBGS, 1.0)
    assert pins.rel_err(out["1"], u_or) <= TOL


@pytest.mark.parametrize("dim,n,sm", [(3, 31, "rb"), (1, 63, "jac")])
def test_full_solve_matches_oracle(pf, dim, n, sm):
    say(f"full solve dim={dim} n={n} smoother={sm}")
    psm, osm, om = smoother_args(pf, sm)
    c = make(pf, dim=dim, n=n, n_slices=1, nodes_coarse=0, smoother=psm, omega=om,
             mg_tol=1e-12, mg_stall=0.75, mg_max_cycles=50)
    alpha = 5.0 / (n + 1) ** 2
    b = inputs.random_field((n,) * dim, 300 + n)
    u0 = np.zeros_like(b)
    u_gpu, st, rr, nc = c.vcycle(alpha, b, u0, 0)
    u_or, nc_or, rr_or = O.mg_solve(dim, alpha, b, u0, O.policy(smoother=osm, omega=om, cycles=0))
    assert nc == nc_or and st in (pf.OK, pf.STALLED)
    assert pins.rel_err(u_gpu.cpu().numpy(), u_or) <= TOL
    assert rr <= 1e-12 or st == pf.STALLED


def test_mixed_precision_refinement_converges(pf):
    """FP32 V-cycles inside FP64 refinement reach the FP64 solution; one
    refinement step agrees with the oracle's FP32 step to FP32 rounding."""
    dim, n = 3, 31
    say("mixed vcycle n=31")
    c = make(pf, dim=dim, n=n, n_slices=1, nodes_coarse=0, precision=pf.MIXED)
    alpha = 3.0 / (n + 1) ** 2
    b = inputs.random_field((n,) * dim, 7)
    u0 = np.zeros_like(b)
    u1, _, _, _ = c.vcycle(alpha, b, u0, 1)
    o1, _, _ = O.mg_solve(dim, alpha, b, u0, O.policy(cycles=1, mixed=1))
    assert pins.rel_err(u1.cpu().numpy(), o1) <= 2e-6
    u8, _, rr, _ = c.vcycle(alpha, b, u0, 10)
    exact, _, _ = O.mg_solve(dim, alpha, b, u0, O.policy(cycles=0, tol=1e-14, stall=0.999, max_cycles=80))
    assert rr <= 1e-13
    assert pins.rel_err(u8.cpu().numpy(), exact) <= 1e-12


# -------------------------------------------------------------- SDC sweep
def random_state(c, orc, dim, n, nc, P, nnf, nnc, seed):
    rng = np.random.default_rng(seed)
    for p in range(P):
        for m in range(nnf):
            for f_or, f_pf in ((O.UF, 0), (O.FF, 1)):
                v = rng.standard_normal((n,) * dim)
                c.set(f_pf, p, m, v)
                orc.set_field(f_or, p, m, v)
        for m in range(nnc):
            for f_or, f_pf in ((O.UC, 2), (O.FC, 3), (O.TAU, 4)):
                v = rng.standard_normal((nc,) * dim) * (1e-3 if f_or == O.TAU else 1.0)
                c.set(f_pf, p, m, v)
                orc.set_field(f_or, p, m, v)


@pytest.mark.parametrize("dim,n,P,level,sm", [(3, 31, 3, 0, "rb"), (3, 31, 3, 1, "rb"),
                                              (1, 63, 4, 0, "jac"), (3, 63, 2, 0, "jac")])
def test_sdc_sweep_matches_oracle(pf, dim, n, P, level, sm):
    say(f"sweep dim={dim} n={n} P={P} level={level}")
    psm, osm, om = smoother_args(pf, sm)
    nu, dt = 1.0, 2e-3
    c = make(pf, dim=dim, n=n, n_slices=P, smoother=psm, omega=om, nu=nu, dt=dt, vcycles_per_solve=1)
    orc = O.Pfasst(dim, n, nu, dt, P, 5, 3, O.policy(smoother=osm, omega=om, cycles=1))
    nc = (n + 1) // 2 - 1
    random_state(c, orc, dim, n, nc, P, 5, 3, 11)
    c.sdc_sweep(level, 0, P)
    for p in range(P):
        orc.sweep(level, p)
    fu, ff, nn = (O.UF, O.FF, 5) if level == 0 else (O.UC, O.FC, 3)
    for p in range(P):
        for m in range(nn):
            u_or, f_or = orc.field(fu, p, m), orc.field(ff, p, m)
            ng = n if level == 0 else nc
            assert pins.rel_err(c.get(fu, p, m), u_or) <= TOL, (p, m)
            assert pins.rel_err(c.get(ff, p, m), f_or) <= f_tol(u_or, f_or, ng, dim, nu), (p, m)


# ----------------------------------------------------------------- PFASST
def f_tol(u, f, n, dim, nu=1.0, tol=TOL, lnorm=4.0):
    """F = nu L_h U is recomputed from U on both sides, so a difference dU
    of U (bounded by tol |U|) reaches F amplified by |nu L_h|_inf =
    lnorm dim nu (n+1)^2 (lnorm 4 for the second-order stencil, 64/12 for
    the fourth-order one): the bar for F is tol * max(1, |nu L_h| |U| / |F|)."""
    amp = lnorm * dim * nu * (n + 1) ** 2 * np.max(np.abs(u)) / max(np.max(np.abs(f)), 1e-300)
    return tol * max(1.0, amp)


def u_close(a, b, tol=TOL, floor=0.0) -> bool:
    """U-type parity: max|a - b| <= max(tol |b|, floor).  `floor` is an
    absolute bound (u_floor) for slices whose solution has decayed far below
    the block's initial value; 0 keeps the plain relative bar."""
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b)))) <= max(tol * float(np.max(np.abs(b))), floor)


def u_floor(u_block, ulps=64.0) -> float:
    """Absolute U bar floor: a few dozen ulps of the block's initial value.
    In the predictor, a late slice's U is the spread value u_block plus an
    interpolated coarse correction of almost the same size and opposite
    sign; what is left is the decayed solution.  Each side rounds the
    correction's weighted sums (Lagrange weights in time, cubic or linear
    weights in space, on each level it passes) in its own order, a few ulps
    of the correction per sum, and the cancellation keeps those ulps of
    u_block in the small result.  Two levels of time-then-space sums of 2-3
    and 4 terms with weights summing to at most 1.625 per axis give about
    20 ulps of u_block; the floor is three times that."""
    return ulps * np.finfo(np.float64).eps * float(np.max(np.abs(u_block)))


def level_lnorm(orc, lev, lnorm=4.0):
    """Amplification of a U difference into F on level lev, in units of
    dim nu (n_lev+1)^2: the stencil's |L| (second order below the fine
    level), or 1/(dt d_min) when F is (U - b)/(dt d_m) (f_solve)."""
    if not orc.prm.f_solve:
        return lnorm
    s, _ = orc.matrices(lev)
    dmin = float(np.min(np.diff(s)))
    return max(lnorm, 1.0 / (orc.prm.dt * dmin * orc.dim * orc.prm.nu * (orc.ns[lev] + 1) ** 2))


def tau_bar_level(orc, lev, p, mc, cmap, du_f, du_c, dtau_f=0.0, lnorm_f=4.0, lnorm_c=4.0):
    """Absolute bar for the FAS term of level lev (>= 1),
    tau[mc] = R(dt sum_i Q_f[cmap mc, i] F_f[i] + tau_f[cmap mc]) - dt sum_j Q_c[mc, j] F_c[j]
    (tau_f = 0 when the finer level is the fine one): a difference of two
    nearly equal sums.  Both sides compute F from their own U, so the
    max-norm differences du_f, du_c of U (measured, and at least 4 ulps of
    U: two implementations agree on U only to rounding) reach F amplified
    by |nu L_h|_inf; each sum adds rounding of a few ulps of its terms; the
    finer level's own term enters as its measured difference dtau_f.  The
    bar is four times that propagated bound."""
    dt, nu, dim = orc.prm.dt, orc.prm.nu, orc.dim
    lf = lev - 1
    _, Qf = orc.matrices(lf)
    _, Qc = orc.matrices(lev)
    fld = lambda l, k, q, m: orc.level_field(l, k, q, m)
    ff = max(np.max(np.abs(fld(lf, O.K_F, p, i))) for i in range(orc.nn[lf]))
    fc = max(np.max(np.abs(fld(lev, O.K_F, p, j))) for j in range(orc.nn[lev]))
    eps = np.finfo(np.float64).eps
    uf = max(np.max(np.abs(fld(lf, O.K_U, p, i))) for i in range(orc.nn[lf]))
    uc = max(np.max(np.abs(fld(lev, O.K_U, p, j))) for j in range(orc.nn[lev]))
    du_f = max(du_f, 4 * eps * uf)
    du_c = max(du_c, 4 * eps * uc)
    bf = lnorm_f * dim * nu * (orc.ns[lf] + 1) ** 2 * du_f + 16 * eps * ff
    bc = lnorm_c * dim * nu * (orc.ns[lev] + 1) ** 2 * du_c + 16 * eps * fc
    tf = 0.0
    if lf > 0:
        tf = float(np.max(np.abs(fld(lf, O.K_TAU, p, cmap[mc])))) * 16 * eps + dtau_f
    return 4 * (dt * (np.abs(Qf[cmap[mc]]).sum() * bf + np.abs(Qc[mc]).sum() * bc) + tf)


def tau_bar(orc, p, mc, cmap, du_f, du_c, lnorm_f=4.0):
    """tau_bar_level for the level below the fine one."""
    return tau_bar_level(orc, 1, p, mc, cmap, du_f, du_c, 0.0, lnorm_f, 4.0)


def node_map(orc, lev):
    """Level lev's nodes -> the coinciding nodes of level lev - 1."""
    sf, _ = orc.matrices(lev - 1)
    sc, _ = orc.matrices(lev)
    return [int(np.argmin(np.abs(sf - x))) for x in sc]


FIELD_IDS = {1: (O.UC, O.FC, O.TAU)}


def compare_levels(c, orc, P, ids, tol=TOL, lnorm_f=4.0, floor=0.0):
    """Every level below the fine one: U (tol, or the floor), F (f_tol with
    the level's own amplification) and tau (tau_bar_level, carrying the
    finer level's measured tau difference down)."""
    for p in range(P):
        du_up = 0.0
        for m in range(orc.nn[0]):
            du_up = max(du_up, float(np.max(np.abs(c.get(O.UF, p, m) - orc.field(O.UF, p, m)))))
        dtau_up = [0.0] * orc.nn[0]
        ln_up = lnorm_f
        for lev in range(1, len(orc.nn)):
            fu, ff, ft = ids[lev]
            du = 0.0
            ln = level_lnorm(orc, lev)
            for m in range(orc.nn[lev]):
                u_or, u_g = orc.level_field(lev, O.K_U, p, m), c.get(fu, p, m)
                du = max(du, float(np.max(np.abs(u_g - u_or))))
                assert u_close(u_g, u_or, tol, floor), (f"U_{lev}", p, m)
                f_or = orc.level_field(lev, O.K_F, p, m)
                assert pins.rel_err(c.get(ff, p, m), f_or) <= f_tol(u_or, f_or, orc.ns[lev], orc.dim, orc.prm.nu,
                                                                     tol, ln), (f"F_{lev}", p, m)
            cmap = node_map(orc, lev)
            dtau = []
            for m in range(orc.nn[lev]):
                t_or = orc.level_field(lev, O.K_TAU, p, m)
                d = float(np.max(np.abs(c.get(ft, p, m) - t_or)))
                dtau.append(d)
                if np.max(np.abs(t_or)) > 0:
                    bar = tau_bar_level(orc, lev, p, m, cmap, du_up, du, dtau_up[cmap[m]], ln_up, ln)
                    assert d <= bar, (f"tau_{lev}", p, m, d, bar)
            du_up, dtau_up, ln_up = du, dtau, ln


def compare_state(c, orc, P, two_levels=True, tol=TOL, lnorm_f=4.0, floor=0.0, ids=None):
    """The fine level's U (tol, or the floor) and F (f_tol), then every
    coarser level through compare_levels."""
    for p in range(P):
        for m in range(orc.nn[0]):
            u_or, f_or = orc.field(O.UF, p, m), orc.field(O.FF, p, m)
            assert u_close(c.get(O.UF, p, m), u_or, tol, floor), ("U_f", p, m)
            assert pins.rel_err(c.get(O.FF, p, m), f_or) <= f_tol(u_or, f_or, orc.n, orc.dim, orc.prm.nu, tol,
                                                                    lnorm_f), ("F_f", p, m)
    if two_levels:
        compare_levels(c, orc, P, ids or FIELD_IDS, tol, lnorm_f, floor)


def test_heat1d_127_predictor_and_five_iterations_match_oracle(pf):
    """1D heat, N=127, P=4, dt=0.01, 5/3 Lobatto, coarse N=63, weighted
    Jacobi 2/3 V(2,2), one V-cycle per solve, predictor + 5 iterations."""
    say("1D heat n=127, 4 slices: predictor + 5 iterations")
    n, P, nu, dt = 127, 4, 1.0, 0.01
    c = make(pf, dim=1, n=n, n_slices=P, nu=nu, dt=dt, smoother=pf.SMOOTH_JACOBI, omega=2 / 3)
    orc = O.Pfasst(1, n, nu, dt, P, 5, 3, O.policy(smoother=O.JACOBI, omega=2 / 3, cycles=1))
    u0, _ = inputs.heat_1d(n)
    c.set_initial(u0)
    orc.set_initial(u0)
    compare_state(c, orc, P)
    for k in range(5):
        r_gpu = c.pfasst_iter()
        r_or = orc.iterate()
        assert abs(r_gpu - r_or) <= 1e-10 * r_or, (k, r_gpu, r_or)
        np.testing.assert_allclose(c.residual(), orc.residual()[1], rtol=1e-10)
        compare_state(c, orc, P)


@pytest.mark.parametrize("n,P,sm,cycles", [(31, 4, "rb", 1), (15, 16, "rb", 2), (63, 2, "jac", 1), (3, 2, "rb", 1),
                                           (15, 3, "rb", 0), (127, 2, "jac", 1)])
def test_pfasst_3d_matches_oracle(pf, n, P, sm, cycles):
    say(f"PFASST 3D n={n} P={P} smoother={sm} cycles={cycles}")
    psm, osm, om = smoother_args(pf, sm)
    nu, dt = 1.0, 1e-3
    c = make(pf, dim=3, n=n, n_slices=P, nu=nu, dt=dt, smoother=psm, omega=om, vcycles_per_solve=cycles)
    orc = O.Pfasst(3, n, nu, dt, P, 5, 3, O.policy(smoother=osm, omega=om, cycles=cycles))
    u0, _ = inputs.random_fourier(n, 1407) if n >= 7 else (inputs.random_field((n,) * 3, 5), None)
    c.set_initial(u0)
    orc.set_initial(u0)
    compare_state(c, orc, P)
    for k in range(3):
        r_gpu = c.pfasst_iter()
        r_or = orc.iterate()
        assert abs(r_gpu - r_or) <= 1e-9 * r_or, (k, r_gpu, r_or)
        compare_state(c, orc, P)
    assert c.vcycle_count(0) == orc.vcycles(0) and c.vcycle_count(1) == orc.vcycles(1)


@pytest.mark.parametrize("nf,nc,n,P,level", [(5, 3, 31, 3, 0), (5, 3, 31, 3, 1), (3, 2, 31, 2, 0),
                                              (3, 2, 31, 2, 1), (5, 2, 15, 2, 1)])
def test_uniform_nodes_sdc_sweep_matches_oracle(pf, nf, nc, n, P, level):
    """The paper's uniform nodes (quadrature without the left end point):
    one sweep on either level, from random node values."""
    say(f"uniform-node sweep {nf}/{nc} n={n} P={P} level={level}")
    nu, dt = 1.0, 2e-3
    c = make(pf, dim=3, n=n, n_slices=P, nu=nu, dt=dt, nodes_fine=nf, nodes_coarse=nc,
             node_family=pf.NODES_UNIFORM, vcycles_per_solve=1)
    orc = O.Pfasst(3, n, nu, dt, P, nf, nc, O.policy(cycles=1), node_family=O.UNIFORM)
    ncg = (n + 1) // 2 - 1
    random_state(c, orc, 3, n, ncg, P, nf, nc, 17)
    c.sdc_sweep(level, 0, P)
    for p in range(P):
        orc.sweep(level, p)
    fu, ff, nn, ng = (O.UF, O.FF, nf, n) if level == 0 else (O.UC, O.FC, nc, ncg)
    for p in range(P):
        for m in range(nn):
            u_or, f_or = orc.field(fu, p, m), orc.field(ff, p, m)
            assert pins.rel_err(c.get(fu, p, m), u_or) <= TOL, (p, m)
            assert pins.rel_err(c.get(ff, p, m), f_or) <= f_tol(u_or, f_or, ng, 3, nu), (p, m)


@pytest.mark.parametrize("nf,nc,n,P,cycles", [(5, 3, 31, 4, 1), (3, 2, 31, 3, 1), (5, 3, 63, 8, 2), (3, 2, 15, 8, 2)])
def test_uniform_nodes_pfasst_matches_oracle(pf, nf, nc, n, P, cycles):
    """IPFASST with the paper's uniform nodes (fourth order over second, or
    second order over backward Euler): predictor and three iterations; P = 8
    runs the pipelined slice groups."""
    say(f"uniform-node PFASST {nf}/{nc} n={n} P={P} cycles={cycles}")
    nu, dt = 1.0 / 3.0, 1.0 / 24
    c = make(pf, dim=3, n=n, n_slices=P, nu=nu, dt=dt, nodes_fine=nf, nodes_coarse=nc,
             node_family=pf.NODES_UNIFORM, vcycles_per_solve=cycles)
    orc = O.Pfasst(3, n, nu, dt, P, nf, nc, O.policy(cycles=cycles), node_family=O.UNIFORM)
    u0 = inputs.sine_mode(n, (1, 1, 1), 3)
    c.set_initial(u0)
    orc.set_initial(u0)
    compare_state(c, orc, P)
    for k in range(3):
        r_gpu = c.pfasst_iter()
        r_or = orc.iterate()
        assert abs(r_gpu - r_or) <= 1e-9 * r_or, (k, r_gpu, r_or)
        compare_state(c, orc, P)
    assert c.vcycle_count(0) == orc.vcycles(0) and c.vcycle_count(1) == orc.vcycles(1)


def test_single_level_isdc_matches_oracle(pf):
    say("ISDC single level")
    n, P = 31, 1
    c = make(pf, dim=3, n=n, n_slices=P, nodes_coarse=0, dt=2e-3)
    orc = O.Pfasst(3, n, 1.0, 2e-3, P, 5, 0, O.policy(cycles=1))
    u0, _ = inputs.random_fourier(n, 3)
    c.set_initial(u0)
    orc.set_initial(u0)
    for _ in range(4):
        assert abs(c.pfasst_iter() - orc.iterate()) <= 1e-9 * orc.residual()[0]
    compare_state(c, orc, P, two_levels=False)


def test_heat1d_127_converges_to_pade_closed_form(pf):
    say("1D heat n=127, 4 slices: to convergence")
    g = pins.golden("lobatto_iiia.json")
    n, P, nu, dt = 127, 4, 1.0, 0.01
    c = make(pf, dim=1, n=n, n_slices=P, nu=nu, dt=dt, smoother=pf.SMOOTH_JACOBI, omega=2 / 3,
             pfasst_tol=1e-12, pfasst_max_iter=300)
    u0, modes = inputs.heat_1d(n)
    st, iters, res = c.run_block(u0)
    assert st == pf.OK and res <= 1e-12
    for p in range(P):
        want = sum(a * pins.pade(dt * nu * pins.mu(n, k), g["pade44_num"]) ** (p + 1)
                   * inputs.sine_mode(n, k, 1) for a, k in zip(modes.amp, modes.k))
        assert pins.rel_err(c.get(O.UF, p, 4), want) <= 1e-11


def test_heat3d_127x16_predictor_and_two_iterations_match_oracle(pf):
    """127^3, 16 slices, dt = 1e-3, RB-GS V(2,2), one V-cycle per solve, in
    the grouped, pipelined launch configuration the benchmark times: every
    slice and node of U and F on both levels and of tau, after the
    predictor and after each of two iterations."""
    say("127^3 x 16 slices: predictor + 2 iterations, every field")
    n, P = 127, 16
    c = make(pf, dim=3, n=n, n_slices=P)
    orc = O.Pfasst(3, n, 1.0, 1e-3, P, 5, 3, O.policy(cycles=1))
    u0, _ = inputs.random_fourier(n, 1407)
    c.set_initial(u0)
    orc.set_initial(u0)
    compare_state(c, orc, P)
    for k in range(2):
        r_gpu, r_or = c.pfasst_iter(), orc.iterate()
        say(f"  iteration {k + 1}: residual {r_gpu:.6e} (oracle {r_or:.6e})")
        assert abs(r_gpu - r_or) <= 1e-9 * r_or
        np.testing.assert_allclose(c.residual(), orc.residual()[1], rtol=1e-9)
        compare_state(c, orc, P)
    assert c.vcycle_count(0) == orc.vcycles(0) and c.vcycle_count(1) == orc.vcycles(1)


def test_heat3d_127x16_converges_to_collocation_closed_form(pf):
    """At convergence every slice's end value is sum_j a_j R44(z_j)^(p+1) phi_j
    (Lobatto IIIA), a property that holds at any size."""
    say("127^3 x 16 slices: to 1e-10")
    g = pins.golden("lobatto_iiia.json")
    n, P, nu, dt = 127, 16, 1.0, 1e-3
    c = make(pf, dim=3, n=n, n_slices=P)
    u0, modes = inputs.random_fourier(n, 1407)
    st, iters, res = c.run_block(u0)
    say(f"  iterations {iters} residual {res:.3e}")
    assert st == pf.OK and res <= 1e-10
    for p in (0, 7, 15):
        want = np.zeros((n,) * 3)
        for a, k in zip(modes.amp, modes.k):
            want += a * pins.pade(dt * nu * pins.mu(n, k), g["pade44_num"]) ** (p + 1) * inputs.sine_mode(n, k, 3)
        assert pins.rel_err(c.get(O.UF, p, 4), want) <= 1e-9, p


def test_nan_input_reports_err_nan(pf):
    say("NaN input")
    n = 15
    c = make(pf, dim=3, n=n, n_slices=2)
    u0 = inputs.random_field((n,) * 3, 1)
    u0[3, 4, 5] = np.nan
    with pytest.raises(pf.PfmgError) as ei:
        c.set_initial(u0)
        c.pfasst_iter()
    assert ei.value.status == pf.ERR_NAN


@pytest.mark.parametrize("n,P,nf,nc,fam", [(31, 4, 5, 3, 0), (63, 3, 3, 2, 1), (15, 8, 5, 3, 0)])
def test_fused_sweep_launches_match_separate(pf, n, P, nf, nc, fam):
    """The fused sweep kernels (node-0 copies + integrals + first right-hand
    side; F + next right-hand side) give the separate launches' state."""
    import os

    say(f"fused vs separate sweep launches n={n} P={P} nodes {nf}/{nc} family {fam}")
    u0, _ = inputs.random_fourier(n, 515) if n >= 7 else (inputs.random_field((n,) * 3, 5), None)
    states = {}
    for fused in ("1", "0"):
        os.environ["PFMG_FUSED_SDC"] = fused
        try:
            c = make(pf, n=n, n_slices=P, nodes_fine=nf, nodes_coarse=nc, node_family=fam, dt=2e-3)
        finally:
            del os.environ["PFMG_FUSED_SDC"]
        c.set_initial(u0)
        res = [c.pfasst_iter() for _ in range(3)]
        states[fused] = (res, [c.get(O.UF, p, nf - 1) for p in range(P)], [c.get(O.UC, p, nc - 1) for p in range(P)],
                         [c.get(O.FC, p, 1) for p in range(P)])
        c.close()
    (r1, f1, c1, g1), (r0, f0, c0, g0) = states["1"], states["0"]
    assert all(abs(a - b) <= 1e-13 * a for a, b in zip(r1, r0)), (r1, r0)
    for p in range(P):
        assert pins.rel_err(f1[p], f0[p]) <= 1e-14 and pins.rel_err(c1[p], c0[p]) <= 1e-14, p
        assert pins.rel_err(g1[p], g0[p]) <= 1e-13, p


@pytest.mark.parametrize("n,groups,streams,late,one", [(31, 2, 2, 1, 0), (31, 4, 2, 1, 0), (31, 5, 2, 1, 0),
                                                       (31, 4, 1, 1, 0), (63, 4, 2, 1, 0), (31, 3, 1, 0, 0),
                                                       (63, 4, 1, 0, 0), (63, 4, 1, 1, 1)])
def test_pipelined_iteration_matches_sequential(pf, n, groups, streams, late, one):
    """Slice groups whose fine sweeps overlap the coarse chain of earlier
    groups (second stream), and each other (fine sweeps alternating over
    two streams), give the sequential schedule's results, with the early
    groups' interpolation and residual on the main stream under the last
    chain (late = 1) or behind each group's chain (late = 0); one = 1 puts
    the chain on the main stream (the benchmark's timing context)."""
    import os

    P = 8
    say(f"pipelined iteration, {groups} groups, {streams} fine stream(s), late interpolation {late}, "
        f"one stream {one}, n={n}, P={P}")
    u0, _ = inputs.random_fourier(n, 4242)
    states = {}
    for g in (1, groups):
        os.environ["PFMG_GROUPS"] = str(g)
        os.environ["PFMG_FINE_STREAMS"] = str(streams)
        os.environ["PFMG_LATE_INTERP"] = str(late)
        os.environ["PFMG_ONE_STREAM"] = str(one)
        try:
            c = make(pf, n=n, n_slices=P)
        finally:
            del os.environ["PFMG_GROUPS"]
            del os.environ["PFMG_FINE_STREAMS"]
            del os.environ["PFMG_LATE_INTERP"]
            del os.environ["PFMG_ONE_STREAM"]
        c.set_initial(u0)
        res = [c.pfasst_iter() for _ in range(4)]
        states[g] = (res, [c.get(O.UF, p, 4) for p in range(P)], [c.get(O.UC, p, 2) for p in range(P)])
        c.close()
    (r1, f1, c1), (rg, fg, cg) = states[1], states[groups]
    assert all(abs(a - b) <= 1e-12 * a for a, b in zip(r1, rg)), (r1, rg)
    for p in range(P):
        assert pins.rel_err(fg[p], f1[p]) <= 1e-13 and pins.rel_err(cg[p], c1[p]) <= 1e-13, p
