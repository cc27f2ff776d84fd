"""pfmg_vcycle_noalloc (the solve for callers that cannot allocate device
memory) against pfmg_vcycle, the context entry point it shares its
kernels with: the same solve on the same seeded inputs within 1e-12
relative, through the C-ABI, on consecutive calls of decreasing size (the
static scratch keeps the previous call's contents), plus the size limit
and the stream-ordered form."""
import numpy as np
import pytest

import inputs
import oracle as O
from tests import pins

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def pf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible ROCm device"
    from paper_1407_6486_amd import pfmg
    return pfmg


def say(msg):
    print(msg, flush=True)


def both(pf, torch, dim, n, cycles, seed, **kw):
    """(u from the context call, u from the no-allocation call, the
    statuses, relres and cycle counts of both)."""
    prm = pf.pfmg_default_params(dim=dim, n=n, n_slices=1, nodes_coarse=0, **kw)
    alpha = 3.0 / (n + 1) ** 2
    b = inputs.random_field((n,) * dim, seed)
    u0 = inputs.random_field((n,) * dim, seed + 1)
    c = pf.Context(prm)
    u_ctx, st_c, rr_c, nc_c = c.vcycle(alpha, b, u0, cycles)
    c.close()
    bd = torch.from_numpy(b).to("cuda")
    ud = torch.from_numpy(u0).to("cuda")
    st_n, rr_n, nc_n = pf.pfmg_vcycle_noalloc(prm, alpha, bd.data_ptr(), ud.data_ptr(), cycles,
                                              torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return u_ctx.cpu().numpy(), ud.cpu().numpy(), (st_c, rr_c, nc_c), (st_n, rr_n, nc_n), b, u0, alpha


def test_noalloc_matches_context_solve_on_consecutive_calls(pf):
    import torch
    # 127^3 two cycles, then the smaller 63^3 and 31^3 grids on the same
    # scratch, then 1D; the last is a full solve to mg_tol
    for dim, n, cycles, seed in [(3, 127, 2, 700), (3, 63, 1, 710), (3, 31, 0, 720), (1, 255, 3, 730)]:
        say(f"no-allocation solve dim={dim} n={n} cycles={cycles}")
        u_c, u_n, (st_c, rr_c, nc_c), (st_n, rr_n, nc_n), b, u0, alpha = both(pf, torch, dim, n, cycles, seed)
        assert st_n == st_c == pf.OK, (st_c, st_n)
        assert nc_n == nc_c and (cycles == 0 or nc_n == cycles), (nc_c, nc_n)
        assert pins.rel_err(u_n, u_c) <= TOL, (dim, n)
        assert abs(rr_n - rr_c) <= 1e-9 * rr_c + 1e-15, (rr_c, rr_n)
        if n <= 63 and cycles > 0:
            u_or = u0.copy()
            for _ in range(cycles):
                u_or = O.vcycle(dim, alpha, b, u_or)
            assert pins.rel_err(u_n, u_or) <= TOL


def test_noalloc_mixed_and_jacobi_match_context_solve(pf):
    import torch
    for kw, n, seed in [(dict(precision=pf.MIXED), 63, 740), (dict(smoother=pf.SMOOTH_JACOBI, omega=2 / 3), 31, 750)]:
        say(f"no-allocation solve n={n} {kw}")
        u_c, u_n, (st_c, _, nc_c), (st_n, _, nc_n), *_ = both(pf, torch, 3, n, 2, seed, **kw)
        assert st_n == st_c == pf.OK and nc_n == nc_c == 2
        assert pins.rel_err(u_n, u_c) <= TOL


def test_noalloc_stream_ordered_without_relres(pf):
    """n_cycles > 0 without relres_out: kernels only, on the caller's stream."""
    import torch
    n, cycles = 63, 2
    prm = pf.pfmg_default_params(dim=3, n=n, n_slices=1, nodes_coarse=0)
    alpha = 3.0 / (n + 1) ** 2
    b = inputs.random_field((n,) * 3, 760)
    u0 = inputs.random_field((n,) * 3, 761)
    c = pf.Context(prm)
    u_ctx, _, _, _ = c.vcycle(alpha, b, u0, cycles)
    c.close()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        bd = torch.from_numpy(b).to("cuda")
        ud = torch.from_numpy(u0).to("cuda")
        st, rr, nc = pf.pfmg_vcycle_noalloc(prm, alpha, bd.data_ptr(), ud.data_ptr(), cycles, s.cuda_stream,
                                            want_relres=False)
    s.synchronize()
    assert st == pf.OK and rr is None and nc == cycles
    assert pins.rel_err(ud.cpu().numpy(), u_ctx.cpu().numpy()) <= TOL


def test_noalloc_rejects_grids_beyond_the_scratch(pf):
    import torch
    n = 255
    prm = pf.pfmg_default_params(dim=3, n=n, n_slices=1, nodes_coarse=0)
    bd = torch.zeros((n,) * 3, dtype=torch.float64, device="cuda")
    ud = torch.zeros_like(bd)
    with pytest.raises(pf.PfmgError) as ei:
        pf.pfmg_vcycle_noalloc(prm, 1e-4, bd.data_ptr(), ud.data_ptr(), 1, 0)
    assert ei.value.status == pf.ERR_WORKSPACE and "scratch" in str(ei.value)
    # the mixed form's FP32 hierarchy does not fit at 127^3
    prm = pf.pfmg_default_params(dim=3, n=127, n_slices=1, nodes_coarse=0, precision=pf.MIXED)
    b1 = torch.zeros((127,) * 3, dtype=torch.float64, device="cuda")
    with pytest.raises(pf.PfmgError) as ei:
        pf.pfmg_vcycle_noalloc(prm, 1e-4, b1.data_ptr(), b1.data_ptr(), 1, 0)
    assert ei.value.status == pf.ERR_WORKSPACE
