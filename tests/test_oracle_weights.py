"""Pins of the oracle's quadrature (paper §3 Multi-rate SDC: node sets, the
weight definitions of s, hat s, tilde s, s_pq, Table tab:weights, and the
consistency identities that follow eq. discrete-node-to-node-embedded).

The pin is an independent derivation: the weights of an interpolatory rule on
n nodes are the unique weights exact for polynomials of degree < n, so they
solve the moment (Vandermonde) system.  Solved here in exact rational
arithmetic (equidistant and Lobatto M=3 nodes are rational) or with 60-digit
mpmath (Lobatto M=4, 5).  The oracle expands Lagrange polynomials instead.
"""
import numpy as np
import pytest

import oracle
from quadref import oracle_EQUI, oracle_LOB, reference


CASES = [(3, oracle_LOB, 10, 1.0), (5, oracle_LOB, 5, 5.0), (4, oracle_LOB, 3, 2.0),
         (3, oracle_EQUI, 4, 1.0), (5, oracle_EQUI, 8, 0.5), (2, oracle_LOB, 1, 1.0),
         (5, oracle_LOB, 20, 5.0)]


@pytest.mark.parametrize("M,fam,P,dt", CASES)
def test_weights_match_moment_solution(M, fam, P, dt):
    got = oracle.weights(M, fam, P, dt)
    ref = reference(M, fam, P, dt)
    for g, r, name in zip(got, ref, ["tau", "s", "shat", "stil", "spq"]):
        scale = max(np.abs(r).max(), 1e-300)
        assert np.abs(g - r).max() <= 4e-16 * scale, name


def test_lobatto3_rows_are_textbook():
    """Lobatto M=3 on [0,1]: node-to-node weights (5/24, 1/3, -1/24) and (-1/24, 1/3, 5/24)."""
    tau, s, *_ = oracle.weights(3, oracle_LOB, 2, 1.0)
    assert np.allclose(tau, [0, 0, 0.5, 1.0], atol=0)
    assert np.array_equal(s[1, 1:], [0, 0, 0])  # degenerate first interval
    assert np.allclose(s[2, 1:], [5 / 24, 1 / 3, -1 / 24], rtol=0, atol=1e-16)
    assert np.allclose(s[3, 1:], [-1 / 24, 1 / 3, 5 / 24], rtol=0, atol=1e-16)


def test_lobatto5_nodes():
    tau, *_ = oracle.weights(5, oracle_LOB, 2, 1.0)
    r = np.sqrt(3 / 7)
    assert np.allclose(tau, [0, 0, (1 - r) / 2, 0.5, (1 + r) / 2, 1], rtol=0, atol=1e-16)


@pytest.mark.parametrize("M,fam,P,dt", CASES)
def test_consistency_identities(M, fam, P, dt):
    """s_{m,j} = sum_p tilde s_{m,p,j};  hat s_{m,q} = sum_p s_{m,p,q};
    sum_j s_{m,j} = dtau_m;  sum_q s_{m,p,q} = dtau_m / P (constants integrate exactly)."""
    tau, s, shat, stil, spq = oracle.weights(M, fam, P, dt)
    big = max(np.abs(shat).max(), np.abs(s).max(), 1.0)
    for m in range(1, M + 1):
        dtm = tau[m] - tau[m - 1]
        assert np.allclose(stil[m, 1:, :].sum(axis=0), s[m], rtol=0, atol=1e-14 * big)
        assert np.allclose(spq[m, 1:, :].sum(axis=0), shat[m], rtol=0, atol=1e-13 * big)
        assert s[m].sum() == pytest.approx(dtm, abs=1e-14 * dt)
        assert shat[m].sum() == pytest.approx(dtm, abs=1e-13 * big)
        for p in range(1, P + 1):
            assert spq[m, p].sum() == pytest.approx(dtm / P, abs=1e-13 * big)


def test_embedded_weight_growth_is_the_papers_rule():
    """The equidistant no-left embedded rule extrapolates to tau_{m-1}; its
    weights grow fast with P (max|hat s|/dtau = 2.6 at P=8, 7.5 at P=10, ~2.3e3 at P=20)."""
    for P, expect in [(8, 2.6), (10, 7.5), (20, 2.3e3)]:
        _, _, shat, _, _ = oracle.weights(3, oracle_EQUI, P, 3.0)
        dtm = 1.0
        assert np.abs(shat[1]).max() / dtm == pytest.approx(expect, rel=0.05)
