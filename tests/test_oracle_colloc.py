"""Pins for the oracle's collocation matrices (Sec. 2.1, eq. BT, eq. Qbe)."""
import numpy as np
import pytest

import oracle as O
from tests import pins


def test_lobatto3_matches_lobatto_iiia_tableau():
    g = pins.golden("lobatto_iiia.json")
    s = O.lobatto_nodes(3)
    assert np.array_equal(s, [pins.frac(p) for p in g["nodes3"]])
    Q, S, d = O.qmat(s)
    Qg = np.array([[pins.frac(p) for p in row] for row in g["Q3"]])
    assert np.max(np.abs(Q - Qg)) <= 2 * np.finfo(float).eps


def test_lobatto5_nodes_closed_form_and_last_row():
    g = pins.golden("lobatto_iiia.json")
    s = O.lobatto_nodes(5)
    assert np.max(np.abs(s - pins.lobatto5())) <= 2 * np.finfo(float).eps
    Q, _, _ = O.qmat(s)
    last = np.array([pins.frac(p) for p in g["Q5_last_row"]])
    assert np.max(np.abs(Q[-1] - last)) <= 2 * np.finfo(float).eps
    assert np.all(Q[0] == 0.0)          # first row of Q is zero (Sec. 2.1)


@pytest.mark.parametrize("nn", [2, 3, 4, 5, 6, 7])
def test_q_exact_on_polynomials_and_row_sums(nn):
    s = O.lobatto_nodes(nn)
    Q, S, d = O.qmat(s)
    # row sums are the nodes: integral of 1 from 0 to s_m
    assert np.max(np.abs(Q.sum(axis=1) - s)) <= 4 * np.finfo(float).eps
    # exact for every polynomial of degree <= M
    for j in range(nn):
        lhs = Q @ s ** j
        assert np.max(np.abs(lhs - s ** (j + 1) / (j + 1))) <= 1e-15
    # independent Vandermonde construction (its float64 solve loses digits
    # with the conditioning of the Vandermonde matrix beyond 5 nodes)
    assert np.max(np.abs(Q - pins.q_vandermonde(s))) <= (1e-14 if nn <= 5 else 1e-12)
    # node-to-node rows and substeps
    assert np.max(np.abs(S - (Q[1:] - Q[:-1]))) <= 2 * np.finfo(float).eps
    assert d[0] == 0.0 and np.max(np.abs(d[1:] - np.diff(s))) <= np.finfo(float).eps
    # the Lobatto nodes integrate degree 2M-1 exactly over [0,1]
    M = nn - 1
    for j in range(2 * M):
        assert abs(Q[-1] @ s ** j - 1.0 / (j + 1)) <= 1e-15


def test_collocation_stability_function_is_pade():
    """eq. BT: collocation = IRK with A = Q, b = last row of Q; for Lobatto
    nodes this is Lobatto IIIA with R(z) = diagonal Pade (closed form)."""
    g = pins.golden("lobatto_iiia.json")
    for nn, key in ((3, "pade22_num"), (5, "pade44_num")):
        Q, _, _ = O.qmat(O.lobatto_nodes(nn))
        for z in (-0.5, -5.0, -200.0, 0.3):
            R = np.linalg.solve(np.eye(nn) - z * Q, np.ones(nn))[-1]
            assert abs(R - pins.pade(z, g[key])) <= 1e-13 * max(1.0, abs(R))


def test_interp_matrix_reproduces_quadratics():
    sf = O.lobatto_nodes(5)
    sc = O.lobatto_nodes(3)
    L = O.interp_matrix(sf, sc)
    for j in range(3):
        assert np.max(np.abs(L @ sc ** j - sf ** j)) <= 1e-15
    # fine nodes 0, 2, 4 coincide with the coarse nodes
    assert np.array_equal(L[[0, 2, 4]], np.eye(3))
