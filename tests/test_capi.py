"""The C-ABI library loads, exports every entry point include/pfmg.h
declares, and validates parameters on the host (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pfmg.h")
LIB = os.path.join(ROOT, "paper_1407_6486_amd", "libpfmg.so")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pfmg_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def pf():
    if not os.path.exists(LIB):
        pytest.fail("libpfmg.so is not built (run __graft_entry__.build())")
    from paper_1407_6486_amd import pfmg
    return pfmg


def test_library_exports_every_declared_symbol(pf):
    lib = C.CDLL(LIB)
    names = declared_symbols()
    assert len(names) >= 16
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(pf.EXPORTED)


def test_params_struct_matches_header_layout(pf):
    # field order in the header
    src = open(HEADER).read()
    body = src[src.index("typedef struct pfmg_params {"):src.index("} pfmg_params;")]
    fields = re.findall(r"\b(?:int32_t|double)\s+(\w+);", body)
    assert fields == [f for f, _ in pf.Params._fields_]


def test_default_params_and_workspace_size(pf):
    p = pf.pfmg_default_params()
    assert (p.dim, p.n, p.n_slices, p.nodes_fine, p.nodes_coarse) == (3, 127, 16, 5, 3)
    nb = pf.pfmg_workspace_bytes(p)
    # fine U and F stacks alone: 2 * 16 * 5 slots of (128*129*129+1) doubles
    assert nb > 2 * 16 * 5 * 128 * 129 * 129 * 8
    assert nb < 8e9


@pytest.mark.parametrize("field,value", [("n", 64), ("n", 9), ("dim", 2), ("nu", -1.0), ("dt", 0.0),
                                         ("n_slices", 0), ("nodes_fine", 1), ("nodes_coarse", 4),
                                         ("omega", 2.5), ("smoother", 7), ("precision", 3),
                                         ("vcycles_per_solve", -1), ("fine_send", 2)])
def test_invalid_parameters_rejected(pf, field, value):
    p = pf.pfmg_default_params(**{field: value})
    with pytest.raises(pf.PfmgError) as ei:
        pf.pfmg_workspace_bytes(p)
    assert ei.value.status == pf.ERR_ARG
    assert pf.pfmg_last_error()


def test_small_workspace_rejected_without_touching_the_gpu(pf):
    p = pf.pfmg_default_params(n=15, n_slices=2)
    with pytest.raises(pf.PfmgError) as ei:
        pf.pfmg_create(p, 0, 0, None)
    assert ei.value.status == pf.ERR_WORKSPACE


def test_node_families_on_the_host(pf):
    """Uniform nodes: 5/3 and 3/2 (coarse nodes a subset of the fine ones)
    and 5/2 are accepted; 5/4 (0, 1/3, 2/3, 1) is not a subset; an unknown
    family is rejected."""
    U = pf.NODES_UNIFORM
    for nf, nc in ((5, 3), (3, 2), (5, 2), (5, 0), (2, 0)):
        assert pf.pfmg_workspace_bytes(pf.pfmg_default_params(n=31, nodes_fine=nf, nodes_coarse=nc,
                                                              node_family=U)) > 0
    for kw in ({"nodes_fine": 5, "nodes_coarse": 4, "node_family": U},
               {"nodes_fine": 4, "nodes_coarse": 3, "node_family": U},
               {"node_family": 2}):
        with pytest.raises(pf.PfmgError) as ei:
            pf.pfmg_workspace_bytes(pf.pfmg_default_params(n=31, **kw))
        assert ei.value.status == pf.ERR_ARG


def test_stencil_and_interpolation_orders_on_the_host(pf):
    for kw in ({"stencil_order": 4}, {"interp_order": 4}, {"stencil_order": 4, "interp_order": 4, "n": 31},
               {"stencil_order": 4, "nodes_coarse": 0, "n": 3, "dim": 1}):
        assert pf.pfmg_workspace_bytes(pf.pfmg_default_params(**kw)) > 0, kw
    for kw in ({"stencil_order": 3}, {"interp_order": 1}, {"stencil_order": 4, "precision": pf.MIXED},
               {"stencil_order": 4, "guess": pf.GUESS_LEARNED, "vcycles_per_solve": 0},
               {"interp_order": 4, "n": 5}):
        with pytest.raises(pf.PfmgError) as ei:
            pf.pfmg_workspace_bytes(pf.pfmg_default_params(**kw))
        assert ei.value.status == pf.ERR_ARG, kw
    with pytest.raises(pf.PfmgError) as ei:
        pf.pfmg_batch_workspace_bytes([pf.pfmg_default_params(n=31, stencil_order=4)])
    assert ei.value.status == pf.ERR_ARG
    # the fourth-order smoother and residual need an out-of-place buffer on
    # the finest grid, which red-black smoothing of a small grid otherwise
    # does not reserve: one more field per slice
    for n, dim in ((15, 3), (7, 3), (63, 1)):
        kw = dict(n=n, dim=dim, n_slices=3, nodes_coarse=0)
        extra = pf.pfmg_workspace_bytes(pf.pfmg_default_params(stencil_order=4, **kw)) - \
            pf.pfmg_workspace_bytes(pf.pfmg_default_params(**kw))
        elems = (n + 1) * (n + 2) ** 2 + 1 if dim == 3 else n + 2
        assert extra >= 3 * elems * 8, (n, dim, extra)


def test_f_options_on_the_host(pf):
    """f_solve / f_interp / residual_abs: 0 or 1, single contexts only; the workspace grows
    by the F(U) fields of the residual (P nn fine fields) and, with f_interp,
    the coarse F at restriction (P nn_c coarse fields)."""
    kw = dict(n=31, n_slices=3)
    base = pf.pfmg_workspace_bytes(pf.pfmg_default_params(**kw))
    fs = pf.pfmg_workspace_bytes(pf.pfmg_default_params(f_solve=1, **kw))
    both = pf.pfmg_workspace_bytes(pf.pfmg_default_params(f_solve=1, f_interp=1, **kw))
    fine, coarse = 32 * 33 ** 2 + 1, 16 * 17 ** 2 + 1
    assert fs - base >= 3 * 5 * fine * 8
    assert both - fs >= 3 * 3 * coarse * 8
    for bad in ({"f_solve": 2}, {"f_interp": -1}, {"residual_abs": 3}):
        with pytest.raises(pf.PfmgError) as ei:
            pf.pfmg_workspace_bytes(pf.pfmg_default_params(**bad))
        assert ei.value.status == pf.ERR_ARG
    for kw in ({"f_interp": 1}, {"residual_abs": 1}):
        with pytest.raises(pf.PfmgError) as ei:
            pf.pfmg_batch_workspace_bytes([pf.pfmg_default_params(n=31, **kw)])
        assert ei.value.status == pf.ERR_ARG


def test_three_levels_on_the_host(pf):
    """nodes_middle: a third level's state, FAS terms and multigrid grow the
    workspace; subsets, grid sizes and the batch are checked."""
    kw = dict(n=31, n_slices=3, nodes_fine=5, nodes_coarse=2)
    # the same fine and 15^3 level (3 nodes) as a two-level context, plus a
    # 7^3 level: U, F, tau and U^old of its 2 nodes per slice at least
    two = pf.pfmg_workspace_bytes(pf.pfmg_default_params(**{**kw, "nodes_coarse": 3}))
    three = pf.pfmg_workspace_bytes(pf.pfmg_default_params(nodes_middle=3, **kw))
    assert three - two >= 4 * 3 * 2 * (8 * 9 ** 2) * 8, (three, two)
    for bad in ({"nodes_middle": 3, "nodes_coarse": 0}, {"nodes_middle": 4},            # 4 Lobatto nodes: no subset
                {"nodes_middle": 3, "n": 5}, {"nodes_middle": 3, "nodes_coarse": 4},
                {"nodes_middle": 3, "n": 7, "interp_order": 4}):
        with pytest.raises(pf.PfmgError) as ei:
            pf.pfmg_workspace_bytes(pf.pfmg_default_params(**{**kw, **bad}))
        assert ei.value.status == pf.ERR_ARG, bad
    assert pf.pfmg_workspace_bytes(pf.pfmg_default_params(**{**kw, "nodes_middle": 3, "n": 7})) > 0
    with pytest.raises(pf.PfmgError) as ei:
        pf.pfmg_batch_workspace_bytes([pf.pfmg_default_params(nodes_middle=3, **kw)])
    assert ei.value.status == pf.ERR_ARG


def test_valid_degenerate_sizes_accepted(pf):
    for n, nc in ((1, 0), (3, 3), (5, 0), (95, 3)):
        p = pf.pfmg_default_params(n=n, nodes_coarse=nc, n_slices=1)
        assert pf.pfmg_workspace_bytes(p) > 0


def test_batch_workspace_and_validation_on_the_host(pf):
    sizes = (31, 63, 95, 127)
    ps = [pf.pfmg_default_params(n=n, n_slices=4, nu=1.0 + q, dt=1e-3 * (q + 1)) for q, n in enumerate(sizes)]
    singles = sum(pf.pfmg_workspace_bytes(p) for p in ps)
    batch = pf.pfmg_batch_workspace_bytes(ps)
    # the batch holds every problem's state; no more than the four contexts
    # plus tables and alignment
    assert 0.8 * singles < batch < 1.1 * singles
    with pytest.raises(pf.PfmgError) as ei:
        pf.pfmg_batch_create(ps, 0, 0, None)
    assert ei.value.status == pf.ERR_WORKSPACE
    bad = [pf.pfmg_default_params(n=31), pf.pfmg_default_params(n=63, nu_pre=1)]
    with pytest.raises(pf.PfmgError) as ei:
        pf.pfmg_batch_workspace_bytes(bad)
    assert ei.value.status == pf.ERR_ARG and "differs from problem 0" in pf.pfmg_last_error()
    for kw in ({"vcycles_per_solve": 0}, {"n_slices": 65}, {"n": 30}):
        with pytest.raises(pf.PfmgError):
            pf.pfmg_batch_workspace_bytes([pf.pfmg_default_params(**kw)])
    assert pf.pfmg_tune_count() >= 0
    assert pf.pfmg_tune_lookup("gfx950/rbgs/f64/0x0") == ""


def test_tune_pins_are_checked_on_the_host(pf):
    key = "testarch/rbgs/f64/127x4+63x8"
    pf.pfmg_tune_set(key, 0)
    assert pf.pfmg_tune_lookup(key) == "0 0 0 0"
    # 127 rows need 128 lanes: 2 rows a pass with 256 threads, 4 with 512
    pf.pfmg_tune_set(key, 1, 10, 16)          # (10 + 2) / 2 = 6 rows per thread
    assert pf.pfmg_tune_lookup(key) == f"1 10 16 {4 * 13 * 8 + 8 * 7 * 4}"
    pf.pfmg_tune_set(key, 2, 10, 5)           # (10 + 2) / 4 = 3
    assert pf.pfmg_tune_lookup(key) == f"2 10 5 {4 * 13 * 26 + 8 * 7 * 13}"
    bad = [(key, 1, 11, 16),                  # 7 rows per thread
           (key, 2, 11, 16),                  # 4 with 512 threads
           (key, 3, 8, 8), (key, -2, 8, 8), (key, 1, 0, 8), (key, 1, 8, 0), (key, 1, 128, 8),
           ("testarch/rbgs/f64/256x1", 1, 2, 8), ("testarch/rbgs/f16/63x1", 0, 0, 0),
           ("testarch/rbgs/f64/63x1+", 0, 0, 0), ("testarch/rbgs/f64/63y1", 0, 0, 0),
           ("rbgs/f64/63x1", 0, 0, 0), ("testarch/rbgs/f64/63x0", 0, 0, 0)]
    for args in bad:
        with pytest.raises(pf.PfmgError) as ei:
            pf.pfmg_tune_set(*args)
        assert ei.value.status == pf.ERR_ARG, args
    assert pf.pfmg_tune_lookup(key) == f"2 10 5 {4 * 13 * 26 + 8 * 7 * 13}"
    # 255 rows: 256 lanes, one row a pass with 256 threads, two with 512
    pf.pfmg_tune_set("testarch/rbgs/f32/255x1", 1, 4, 8)
    pf.pfmg_tune_set("testarch/rbgs/f32/255x1", 2, 4, 8)
    with pytest.raises(pf.PfmgError):
        pf.pfmg_tune_set("testarch/rbgs/f32/255x1", 1, 5, 8)
    for k in (key, "testarch/rbgs/f32/255x1"):
        pf.pfmg_tune_set(k, -1)
        assert pf.pfmg_tune_lookup(k) == ""


def test_network_sizes_on_the_host(pf):
    from oracle import unet as U

    want = sum(w.size + b.size for w, b in U.init_params(0))
    assert pf.pfmg_nn_param_count() == want
    assert pf.pfmg_nn_workspace_bytes(63, 4, True) > pf.pfmg_nn_workspace_bytes(63, 4, False) > 0
    for n in (62, 29, 7, 0):     # even, odd with an even level, too few levels
        with pytest.raises(pf.PfmgError):
            pf.pfmg_nn_workspace_bytes(n, 1, False)
    with pytest.raises(pf.PfmgError) as ei:
        pf.pfmg_nn_create(63, 4, False, 0, 0, None)
    assert ei.value.status == pf.ERR_WORKSPACE
    with pytest.raises(pf.PfmgError):   # learned guess needs full solves
        pf.pfmg_workspace_bytes(pf.pfmg_default_params(n=63, guess=pf.GUESS_LEARNED))
    assert pf.pfmg_workspace_bytes(pf.pfmg_default_params(n=63, guess=pf.GUESS_LEARNED, vcycles_per_solve=0)) > 0


def test_stream_copy_checks_arguments_on_the_host(pf):
    """Sizes and pointers not multiples of 16, null and overlapping ranges
    are refused before any launch (no GPU needed)."""
    for dst, src, nb in ((1 << 20, 1 << 24, 24), (1 << 20 | 8, 1 << 24, 32), (0, 1 << 24, 32),
                         (1 << 20, (1 << 20) + 16, 64)):
        with pytest.raises(pf.PfmgError) as ei:
            pf.pfmg_stream_copy(dst, src, nb, None)
        assert ei.value.status == pf.ERR_ARG
    assert pf.pfmg_stream_copy(1 << 20, 1 << 24, 0, None) == pf.OK
