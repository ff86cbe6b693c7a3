"""Stationary initial field (the numerical example's initial data, section 5):
(K + h R) T = g with g = h T_env r.  Because K 1 = 0 and R 1 = r (the Robin
mass rows sum to the Robin load), the exact solution is T = T_env on every
body with a Robin term, whatever the mesh; the oracle must reach it from any
start.  A dropped Robin operator, a wrong sign or a stray mass term breaks it."""
import numpy as np
import pytest

import mrsdc_inputs as mi
import oracle


@pytest.mark.parametrize("make", [
    lambda: mi.patch_box(L=(0.2, 0.2, 0.5), nodes=(6, 7, 21), nsteps=1),
    lambda: mi.machine(stand_nodes=(5, 7, 19), stock_nodes=(4, 5, 7), stand_L=(0.2, 0.3, 0.9),
                       stock_L=(0.15, 0.2, 0.3), nsteps=1),
])
def test_stationary_is_the_ambient_temperature(make):
    pb = make()
    T0 = pb.T0 + np.random.default_rng(3).uniform(-30.0, 30.0, size=pb.N)
    T, it = oracle.stationary(pb, T0=T0)
    assert it > 0
    Tenv = np.concatenate([np.full(b.n, t) for b, t in zip(pb.bodies, pb.T_amb)])
    assert np.abs(T - Tenv).max() < 1e-9


def test_stationary_other_ambient_per_body():
    pb = mi.machine(stand_nodes=(5, 7, 19), stock_nodes=(4, 5, 7), stand_L=(0.2, 0.3, 0.9),
                    stock_L=(0.15, 0.2, 0.3), nsteps=1)
    pb.T_amb = [15.0, 35.0]
    T, _ = oracle.stationary(pb)
    n0 = pb.bodies[0].n
    assert np.abs(T[:n0] - 15.0).max() < 1e-9 and np.abs(T[n0:] - 35.0).max() < 1e-9


def test_stationary_residual_of_the_assembled_system():
    """Independent check of the equation itself on a tiny mesh: a dense solve
    of (K + h R) T = g with the harness's own matrices."""
    pb = mi.patch_box(L=(0.1, 0.1, 0.2), nodes=(3, 3, 4), nsteps=1)
    b = pb.bodies[0]
    n = b.n
    A = np.zeros((n, n))
    for i in range(n):
        for e in range(b.rowptr[i], b.rowptr[i + 1]):
            A[i, b.col[e]] += b.K[e] + pb.h[0] * b.R[e]
    g = pb.h[0] * pb.T_amb[0] * b.rload
    ref = np.linalg.solve(A, g)
    T, _ = oracle.stationary(pb)
    assert np.abs(T - ref).max() < 1e-9
