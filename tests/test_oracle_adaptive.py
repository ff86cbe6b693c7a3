"""Residual-controlled sweeps: a step stops sweeping once the residual (eq.
residual) of its latest iterate is at or below sweep_tol, and runs at most K
sweeps.  Pinned against runs with a fixed number of sweeps: the controlled
run must equal, bitwise, the fixed run with the number of sweeps the rule
picks from that run's own residual sequence."""
import dataclasses

import numpy as np
import pytest

import mrsdc_inputs as mi
import oracle


def machine(**kw):
    sc = mi.Scheme(M=5, family=mi.LOBATTO, P=5, K=4, dt=5.0)
    return mi.machine(stand_nodes=(5, 7, 19), stock_nodes=(4, 5, 7), stand_L=(0.2, 0.3, 0.9),
                      stock_L=(0.15, 0.2, 0.3), period=3.0, stroke=0.5, scheme=sc, nsteps=1, **kw)


def run(pb, nsteps, K, tol):
    sc = dataclasses.replace(pb.scheme, K=K, sweep_tol=tol)
    return oracle.run(pb, nsteps=nsteps, scheme=sc)


def test_zero_tolerance_is_the_fixed_scheme():
    pb = machine()
    a, sa = run(pb, 3, 4, 0.0)
    b, sb = run(pb, 3, 4, 0.0)
    assert np.array_equal(a, b) and sa["sweeps"] == 12


def test_huge_tolerance_stops_after_the_predictor():
    pb = machine()
    a, sa = run(pb, 3, 4, 1e300)
    b, _ = run(pb, 3, 0, 0.0)
    assert np.array_equal(a, b) and sa["sweeps"] == 0


@pytest.mark.parametrize("j", [1, 2, 3])
def test_stops_where_the_residual_first_drops_below(j):
    pb = machine()
    _, _, res = oracle.run(pb, nsteps=1, residuals=True)
    r = res[0]  # residual of iterates 0..K of the one step
    assert np.all(np.diff(np.log(r[: j + 1])) < 0), r
    tol = np.sqrt(r[j] * r[j - 1])  # between iterate j-1 and iterate j
    got, st = run(pb, 1, 4, tol)
    ref, _ = run(pb, 1, j, 0.0)
    assert st["sweeps"] == j
    assert np.array_equal(got, ref)
