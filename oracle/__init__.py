"""Plain FP64 CPU oracle for IPFASST with multigrid node solves.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and
the CPU-baseline leg of the benchmark, never by the product path.  The C
sources next to this file implement the algorithm of arXiv:1407.6486 step
by step (collocation Sec. 2.1, SDC Sec. 2.2, MLSDC/FAS Sec. 2.3, PFASST
Sec. 2.4, multigrid Sec. 4.1.1 / 4.2.1); this module only marshals
numpy arrays through ctypes.

Arrays are dense ``n**dim`` float64 in C order with x fastest, i.e. numpy
shape ``(n, n, n)`` indexed ``[z, y, x]`` (1D: shape ``(n,)``).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "liboracle.so")
_lib = None

JACOBI, RBGS = 0, 1
LOBATTO, UNIFORM = 0, 1          # node families
UF, FF, UC, FC, TAU, UCOLD, FCOLD = range(7)
K_U, K_F, K_TAU, K_UOLD = range(4)

_dp = C.POINTER(C.c_double)
_fp = C.POINTER(C.c_float)


class MGPolicy(C.Structure):
    _fields_ = [("smoother", C.c_int), ("nu1", C.c_int), ("nu2", C.c_int),
                ("omega", C.c_double), ("cycles", C.c_int), ("tol", C.c_double),
                ("stall", C.c_double), ("max_cycles", C.c_int), ("mixed", C.c_int)]


class Params(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int), ("nu", C.c_double), ("dt", C.c_double),
                ("n_slices", C.c_int), ("nodes_fine", C.c_int), ("nodes_coarse", C.c_int),
                ("mg", MGPolicy), ("interp_order", C.c_int), ("node_family", C.c_int),
                ("stencil_order", C.c_int), ("f_solve", C.c_int), ("f_interp", C.c_int),
                ("residual_abs", C.c_int), ("nodes_middle", C.c_int), ("fine_send", C.c_int)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(_LIB_PATH)
        L.or_lobatto_nodes.argtypes = [C.c_int, _dp]
        L.or_qmat.argtypes = [C.c_int, _dp, _dp, _dp, _dp]
        L.or_uniform_nodes.argtypes = [C.c_int, _dp]
        L.or_qmat_family.argtypes = [C.c_int, _dp, C.c_int, _dp, _dp, _dp]
        L.or_interp_matrix.argtypes = [C.c_int, _dp, C.c_int, _dp, _dp]
        L.or_lap.argtypes = [C.c_int, C.c_int, _dp, _dp]
        L.or_helm.argtypes = [C.c_int, C.c_int, C.c_double, _dp, _dp]
        L.or_resid.argtypes = [C.c_int, C.c_int, C.c_double, _dp, _dp, _dp]
        L.or_norm_inf.argtypes = [C.c_size_t, _dp]
        L.or_norm_inf.restype = C.c_double
        L.or_smooth.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_double, _dp, _dp]
        L.or_restrict_fw.argtypes = [C.c_int, C.c_int, _dp, _dp]
        L.or_prolong_add.argtypes = [C.c_int, C.c_int, _dp, _dp]
        L.or_prolong4_add.argtypes = [C.c_int, C.c_int, _dp, _dp]
        L.or_coarsest.argtypes = [C.c_int, C.c_int, C.c_double, _dp, _dp]
        L.or_lap4.argtypes = [C.c_int, C.c_int, _dp, _dp]
        L.or_resid4.argtypes = [C.c_int, C.c_int, C.c_double, _dp, _dp, _dp]
        L.or_smooth4.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_double, _dp, _dp]
        L.or_vcycle4.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_double, C.c_int, C.c_int, _dp, _dp]
        L.or_mg_solve4.argtypes = [C.c_int, C.c_int, C.c_double, C.POINTER(MGPolicy), _dp, _dp, _dp]
        L.or_mg_solve4.restype = C.c_int
        L.or_vcycle.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_double,
                                C.c_int, C.c_int, _dp, _dp]
        L.orf_vcycle.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_double,
                                 C.c_int, C.c_int, _fp, _fp]
        L.orf_smooth.argtypes = [C.c_int, C.c_int, C.c_double, C.c_int, C.c_double, _fp, _fp]
        L.or_mg_solve.argtypes = [C.c_int, C.c_int, C.c_double, C.POINTER(MGPolicy), _dp, _dp, _dp]
        L.or_mg_solve.restype = C.c_int
        L.or_pfasst_create.argtypes = [C.POINTER(Params)]
        L.or_pfasst_create.restype = C.c_void_p
        L.or_pfasst_destroy.argtypes = [C.c_void_p]
        L.or_pfasst_spread.argtypes = [C.c_void_p, _dp]
        L.or_pfasst_predictor.argtypes = [C.c_void_p]
        L.or_pfasst_iter.argtypes = [C.c_void_p]
        L.or_pfasst_iter.restype = C.c_double
        L.or_pfasst_residual.argtypes = [C.c_void_p, _dp]
        L.or_pfasst_residual.restype = C.c_double
        L.or_sdc_sweep.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.or_fas_restrict.argtypes = [C.c_void_p, C.c_int]
        L.or_interpolate.argtypes = [C.c_void_p, C.c_int]
        L.or_pfasst_field.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int]
        L.or_pfasst_field.restype = _dp
        L.or_fas_restrict_level.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.or_interpolate_level.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.or_pfasst_level_field.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int]
        L.or_pfasst_level_field.restype = _dp
        L.or_pfasst_vcycles.argtypes = [C.c_void_p, C.c_int]
        L.or_pfasst_vcycles.restype = C.c_longlong
        L.or_pfasst_matrices.argtypes = [C.c_void_p, C.c_int, _dp, _dp]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags.c_contiguous
    if a.dtype == np.float64:
        return a.ctypes.data_as(_dp)
    assert a.dtype == np.float32
    return a.ctypes.data_as(_fp)


def shape(dim: int, n: int):
    return (n,) * dim


# --------------------------------------------------------------- collocation
def lobatto_nodes(nnodes: int) -> np.ndarray:
    s = np.zeros(nnodes)
    assert lib().or_lobatto_nodes(nnodes, _p(s)) == 0
    return s


def uniform_nodes(nnodes: int) -> np.ndarray:
    s = np.zeros(nnodes)
    assert lib().or_uniform_nodes(nnodes, _p(s)) == 0
    return s


def nodes(nnodes: int, family: int = LOBATTO) -> np.ndarray:
    return uniform_nodes(nnodes) if family == UNIFORM else lobatto_nodes(nnodes)


def qmat(s: np.ndarray, family: int = LOBATTO):
    """(Q, S, d): integration matrix, node-to-node rows, substep lengths."""
    s = np.ascontiguousarray(s, dtype=np.float64)
    nn = len(s)
    Q = np.zeros((nn, nn)); S = np.zeros((nn - 1, nn)); d = np.zeros(nn)
    assert lib().or_qmat_family(nn, _p(s), family, _p(Q), _p(S), _p(d)) == 0
    return Q, S, d


def interp_matrix(sf: np.ndarray, sc: np.ndarray) -> np.ndarray:
    sf = np.ascontiguousarray(sf, dtype=np.float64)
    sc = np.ascontiguousarray(sc, dtype=np.float64)
    L = np.zeros((len(sf), len(sc)))
    assert lib().or_interp_matrix(len(sf), _p(sf), len(sc), _p(sc), _p(L)) == 0
    return L


# ------------------------------------------------------------------- grids
def _out(u):
    return np.zeros_like(u)


def lap(dim, u):
    u = np.ascontiguousarray(u, dtype=np.float64); o = _out(u)
    lib().or_lap(dim, u.shape[0], _p(u), _p(o)); return o


def helm(dim, alpha, u):
    u = np.ascontiguousarray(u, dtype=np.float64); o = _out(u)
    lib().or_helm(dim, u.shape[0], alpha, _p(u), _p(o)); return o


def resid(dim, alpha, b, u):
    b = np.ascontiguousarray(b, dtype=np.float64); u = np.ascontiguousarray(u, dtype=np.float64)
    o = _out(u); lib().or_resid(dim, u.shape[0], alpha, _p(b), _p(u), _p(o)); return o


def smooth(dim, alpha, smoother, omega, b, u):
    """One sweep, returns the new u (input untouched)."""
    u = np.array(u, dtype=np.float64, order="C"); b = np.ascontiguousarray(b, dtype=np.float64)
    lib().or_smooth(dim, u.shape[0], alpha, smoother, omega, _p(b), _p(u)); return u


def restrict_fw(dim, r):
    r = np.ascontiguousarray(r, dtype=np.float64); n = r.shape[0]; nc = (n + 1) // 2 - 1
    o = np.zeros(shape(dim, nc)); lib().or_restrict_fw(dim, n, _p(r), _p(o)); return o


def prolong_add(dim, ec, u):
    ec = np.ascontiguousarray(ec, dtype=np.float64); u = np.array(u, dtype=np.float64, order="C")
    lib().or_prolong_add(dim, ec.shape[0], _p(ec), _p(u)); return u


def coarsest(dim, alpha, b):
    b = np.ascontiguousarray(b, dtype=np.float64); u = np.zeros_like(b)
    lib().or_coarsest(dim, b.shape[0], alpha, _p(b), _p(u)); return u


def vcycle(dim, alpha, b, u, smoother=RBGS, omega=1.0, nu1=2, nu2=2):
    u = np.array(u, dtype=np.float64, order="C"); b = np.ascontiguousarray(b, dtype=np.float64)
    lib().or_vcycle(dim, u.shape[0], alpha, smoother, omega, nu1, nu2, _p(b), _p(u)); return u


def vcycle32(dim, alpha, b, u, smoother=RBGS, omega=1.0, nu1=2, nu2=2):
    u = np.array(u, dtype=np.float32, order="C"); b = np.ascontiguousarray(b, dtype=np.float32)
    lib().orf_vcycle(dim, u.shape[0], alpha, smoother, omega, nu1, nu2, _p(b), _p(u)); return u


def lap4(dim, u):
    u = np.ascontiguousarray(u, dtype=np.float64); o = _out(u)
    lib().or_lap4(dim, u.shape[0], _p(u), _p(o)); return o


def resid4(dim, alpha, b, u):
    b = np.ascontiguousarray(b, dtype=np.float64); u = np.ascontiguousarray(u, dtype=np.float64)
    o = _out(u); lib().or_resid4(dim, u.shape[0], alpha, _p(b), _p(u), _p(o)); return o


def smooth4(dim, alpha, smoother, omega, b, u):
    u = np.array(u, dtype=np.float64, order="C"); b = np.ascontiguousarray(b, dtype=np.float64)
    lib().or_smooth4(dim, u.shape[0], alpha, smoother, omega, _p(b), _p(u)); return u


def vcycle4(dim, alpha, b, u, smoother=RBGS, omega=1.0, nu1=2, nu2=2):
    u = np.array(u, dtype=np.float64, order="C"); b = np.ascontiguousarray(b, dtype=np.float64)
    lib().or_vcycle4(dim, u.shape[0], alpha, smoother, omega, nu1, nu2, _p(b), _p(u)); return u


def mg_solve4(dim, alpha, b, u, pol):
    """Returns (u, cycles, relres) for (I - alpha L4) u = b."""
    u = np.array(u, dtype=np.float64, order="C"); b = np.ascontiguousarray(b, dtype=np.float64)
    rr = C.c_double(0.0)
    nc = lib().or_mg_solve4(dim, u.shape[0], alpha, C.byref(pol), _p(b), _p(u), C.byref(rr))
    return u, nc, rr.value


def policy(smoother=RBGS, nu1=2, nu2=2, omega=1.0, cycles=1, tol=1e-12, stall=0.75,
           max_cycles=50, mixed=0) -> MGPolicy:
    return MGPolicy(smoother, nu1, nu2, omega, cycles, tol, stall, max_cycles, mixed)


def mg_solve(dim, alpha, b, u, pol: MGPolicy):
    """Returns (u, cycles, relres)."""
    u = np.array(u, dtype=np.float64, order="C"); b = np.ascontiguousarray(b, dtype=np.float64)
    rr = C.c_double(0.0)
    nc = lib().or_mg_solve(dim, u.shape[0], alpha, C.byref(pol), _p(b), _p(u), C.byref(rr))
    return u, nc, rr.value


# ------------------------------------------------------------------ PFASST
class Pfasst:
    """Serial emulation of P time slices (two levels, or one when
    ``nodes_coarse == 0``)."""

    def __init__(self, dim, n, nu, dt, n_slices, nodes_fine=5, nodes_coarse=3,
                 mg: MGPolicy | None = None, interp_order: int = 2, node_family: int = LOBATTO,
                 stencil_order: int = 2, f_solve: int = 0, f_interp: int = 0, residual_abs: int = 0,
                 nodes_middle: int = 0, fine_send: int = 0):
        self.prm = Params(dim, n, nu, dt, n_slices, nodes_fine, nodes_coarse,
                          mg if mg is not None else policy(), interp_order, node_family, stencil_order,
                          f_solve, f_interp, residual_abs, nodes_middle, fine_send)
        self.dim, self.n, self.P = dim, n, n_slices
        self.nn = [nodes_fine, nodes_coarse] if nodes_middle == 0 else [nodes_fine, nodes_middle, nodes_coarse]
        self.nc = (n + 1) // 2 - 1
        self.ns = [n]
        for _ in range(len(self.nn) - 1 if nodes_coarse else 0):
            self.ns.append((self.ns[-1] + 1) // 2 - 1)
        h = lib().or_pfasst_create(C.byref(self.prm))
        if not h:
            raise ValueError("oracle rejected the parameters")
        self._h = C.c_void_p(h)

    def __del__(self):
        if getattr(self, "_h", None):
            try:
                lib().or_pfasst_destroy(self._h)
            except (TypeError, AttributeError):    # interpreter shutdown: the module is gone
                pass
            self._h = None

    def spread(self, u0):
        u0 = np.ascontiguousarray(u0, dtype=np.float64)
        lib().or_pfasst_spread(self._h, _p(u0))

    def predictor(self):
        lib().or_pfasst_predictor(self._h)

    def set_initial(self, u0):
        self.spread(u0)
        self.predictor()

    def iterate(self) -> float:
        return lib().or_pfasst_iter(self._h)

    def residual(self):
        r = np.zeros(self.P)
        blk = lib().or_pfasst_residual(self._h, _p(r))
        return blk, r

    def sweep(self, level, p):
        lib().or_sdc_sweep(self._h, level, p)

    def fas_restrict(self, p):
        lib().or_fas_restrict(self._h, p)

    def interpolate(self, p):
        lib().or_interpolate(self._h, p)

    def fas_restrict_level(self, level, p):
        lib().or_fas_restrict_level(self._h, level, p)

    def interpolate_level(self, level, p):
        lib().or_interpolate_level(self._h, level, p)

    def level_field(self, level, kind, p, m) -> np.ndarray:
        """A copy of level `level`'s field (kind: K_U, K_F, K_TAU, K_UOLD)."""
        ptr = lib().or_pfasst_level_field(self._h, level, kind, p, m)
        if not ptr:
            raise ValueError("no such field")
        n = self.ns[level]
        a = np.ctypeslib.as_array(ptr, shape=(n ** self.dim,))
        return a.reshape(shape(self.dim, n)).copy()

    def vcycles(self, level=0) -> int:
        return lib().or_pfasst_vcycles(self._h, level)

    def field(self, which, p, m) -> np.ndarray:
        """A copy of the field (U_f, F_f, U_c, F_c, tau, U_c_old, F_c_old) at slice p, node m."""
        n = self.n if which in (UF, FF) else self.nc
        ptr = lib().or_pfasst_field(self._h, which, p, m)
        if not ptr:
            raise ValueError("no such field")
        a = np.ctypeslib.as_array(ptr, shape=(n ** self.dim,))
        return a.reshape(shape(self.dim, n)).copy()

    def set_field(self, which, p, m, v):
        n = self.n if which in (UF, FF) else self.nc
        ptr = lib().or_pfasst_field(self._h, which, p, m)
        a = np.ctypeslib.as_array(ptr, shape=(n ** self.dim,))
        a[:] = np.asarray(v, dtype=np.float64).reshape(-1)

    def set_level_field(self, level, kind, p, m, v):
        ptr = lib().or_pfasst_level_field(self._h, level, kind, p, m)
        if not ptr:
            raise ValueError("no such field")
        a = np.ctypeslib.as_array(ptr, shape=(self.ns[level] ** self.dim,))
        a[:] = np.asarray(v, dtype=np.float64).reshape(-1)

    def matrices(self, level):
        nn = self.nn[level]
        s = np.zeros(nn); Q = np.zeros((nn, nn))
        lib().or_pfasst_matrices(self._h, level, _p(s), _p(Q))
        return s, Q


def prolong4_add(dim, ec, u):
    ec = np.ascontiguousarray(ec, dtype=np.float64); u = np.array(u, dtype=np.float64, order="C")
    lib().or_prolong4_add(dim, ec.shape[0], _p(ec), _p(u)); return u
