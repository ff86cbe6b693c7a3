"""Pins of the oracle's single-rate SDC (paper §3, "Single-rate spectral
deferred correction", in the form §5 compares against: the part of f^E linear
in T sits in the implicit operator) and of implicit Euler (one equidistant
node, no sweep), against facts that do not come from the oracle's stepper:

  * implicit Euler and the predictor solved densely node by node, with the
    affine map T -> f^E(T, t) probed column by column;
  * many sweeps reach the collocation solution (eq. collocation), built from
    exact rational quadrature weights and solved densely;
  * without a coupling the method is the same SISDC iteration as the
    multi-rate one with f^E = 0 (the embedded nodes then only subdivide a
    linear update), so both agree to round-off;
  * heat balance of insulated bodies: conduction and exchange conserve heat,
    the friction adds P_f per second whatever K is;
  * observed order min(K + 1, 4) on 3 Lobatto nodes against the matrix
    exponential of a time-invariant coupled problem, and order 1 for
    implicit Euler.
"""
import math
from dataclasses import replace
from fractions import Fraction

import numpy as np
import pytest

import mrsdc_inputs as mi
import oracle
from quadref import moment_weights, std_nodes
from test_oracle_stepper import exact_order_solution, fE_affine, order_problem

SR = mi.SINGLE_RATE


def small_contact(sc, h=30.0, robin=True):
    return mi.machine(stand_nodes=(3, 3, 5), stock_nodes=(2, 3, 3), stand_L=(0.2, 0.4, 1.0),
                      stock_L=(0.1, 0.3, 0.3), y_offset=0.05, scheme=sc, period=2.0, stroke=0.4,
                      alpha=900.0, friction_W=60.0, h=h, robin=robin)


def dense_parts(p):
    """L = K + h R, g and the lumped mass of the concatenated system."""
    N = p.N
    L = np.zeros((N, N))
    g = np.zeros(N)
    mass = np.zeros(N)
    off = p.offsets
    for i, bb in enumerate(p.bodies):
        sl = slice(off[i], off[i + 1])
        L[sl, sl] = bb.csr("K").toarray() + p.h[i] * bb.csr("R").toarray()
        g[sl] = p.h[i] * p.T_amb[i] * bb.rload
        mass[sl] = bb.mass
    return L, g, mass


@pytest.mark.parametrize("M,fam", [(1, mi.EQUI_NOLEFT), (3, mi.LOBATTO), (2, mi.EQUI_NOLEFT)])
def test_predictor_is_implicit_euler_with_coupling(M, fam):
    """K = 0: node to node, (diag(m) + dtau (L - E(tau_m))) T_m
    = diag(m) T_{m-1} + dtau (g + e(tau_m)), f^E(T, t) = E(t) T + e(t)."""
    sc = mi.Scheme(M=M, family=fam, P=2, K=0, dt=0.3, pcg_rtol=1e-15, method=SR)
    p = small_contact(sc)
    T, st = oracle.run(p, nsteps=3)
    tau, *_ = oracle.weights(M, fam, 2, sc.dt)
    L, g, mass = dense_parts(p)
    x = p.T0.copy()
    for n in range(3):
        for m in range(1, M + 1):
            dtau = tau[m] - tau[m - 1]
            if dtau == 0.0:
                continue
            E, e = fE_affine(p, n * sc.dt + tau[m])
            x = np.linalg.solve(np.diag(mass) + dtau * (L - E), mass * x + dtau * (g + e))
    assert np.abs(T - x).max() < 1e-11 * np.abs(x).max()
    assert st["sweeps"] == 0


@pytest.mark.parametrize("M,fam", [(3, mi.LOBATTO), (3, mi.EQUI_NOLEFT)])
def test_sweeps_converge_to_collocation(M, fam):
    """eq. collocation: diag(m) T_m = diag(m) T_n + sum_j q_{m,j} F(T_j, tau_j),
    q_{m,j} = dt int_0^{x_m} l_j, exact weights; F = -L T + g + E(tau_j) T + e(tau_j)."""
    sc = mi.Scheme(M=M, family=fam, P=2, K=60, dt=0.25, pcg_rtol=1e-15, method=SR)
    p = small_contact(sc)
    T, _, res = oracle.run(p, nsteps=1, residuals=True)
    x = std_nodes(M, fam)
    q = np.array([[float(w) for w in moment_weights(x, Fraction(0), xm)] for xm in x]) * sc.dt
    L, g, mass = dense_parts(p)
    N = p.N
    A = np.zeros((M * N, M * N))
    rhs = np.zeros(M * N)
    Ej = [fE_affine(p, float(xj) * sc.dt) for xj in x]
    for m in range(M):
        r = slice(m * N, (m + 1) * N)
        A[r, r] += np.diag(mass)
        rhs[r] += mass * p.T0
        for j in range(M):
            E, e = Ej[j]
            A[r, j * N:(j + 1) * N] -= q[m, j] * (E - L)
            rhs[r] += q[m, j] * (g + e)
    U = np.linalg.solve(A, rhs)
    ref = U[(M - 1) * N:]
    assert np.abs(T - ref).max() < 1e-11 * np.abs(ref).max()
    assert res[0, -1] < 1e-14 * np.abs(mass * T).max()
    assert res[0, 0] > 1e5 * res[0, -1]


@pytest.mark.parametrize("K", [0, 2])
def test_without_coupling_equals_multirate(K):
    sc = mi.Scheme(M=3, family=mi.LOBATTO, P=3, K=K, dt=2.0, pcg_rtol=1e-15)
    p = small_contact(sc)
    p.coupling = None
    a, _ = oracle.run(p, nsteps=3)
    b, _ = oracle.run(p, nsteps=3, scheme=replace(sc, method=SR))
    assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()


@pytest.mark.parametrize("M,fam,K", [(3, mi.LOBATTO, 2), (1, mi.EQUI_NOLEFT, 0)])
def test_heat_balance_contact_insulated(M, fam, K):
    sc = mi.Scheme(M=M, family=fam, P=3, K=K, dt=0.4, method=SR)
    p = mi.machine(stand_nodes=(4, 5, 11), stock_nodes=(3, 4, 5), stand_L=(0.2, 0.4, 1.0),
                   stock_L=(0.1, 0.3, 0.3), y_offset=0.05, robin=False, scheme=sc, period=2.0,
                   stroke=0.4, alpha=800.0, friction_W=75.0)
    m = np.concatenate([bb.mass for bb in p.bodies])
    p.T0 = p.T0 - 20.0
    E0 = m @ p.T0
    T, _ = oracle.run(p, nsteps=5)
    assert m @ T - E0 == pytest.approx(75.0 * 5 * sc.dt, rel=1e-10)


@pytest.mark.parametrize("M,fam,K,expected", [(3, mi.LOBATTO, 0, 1), (3, mi.LOBATTO, 1, 2),
                                              (3, mi.LOBATTO, 2, 3), (3, mi.LOBATTO, 4, 4),
                                              (1, mi.EQUI_NOLEFT, 0, 1)])
def test_observed_order(M, fam, K, expected):
    """Order min(K+1, 4) on 3 Lobatto nodes (collocation order 4), order 1 for
    implicit Euler, against the matrix exponential."""
    Tend = 0.2
    ref = exact_order_solution(order_problem(0.1, K, 2), Tend)
    errs = []
    for n in (32, 64, 128):
        p = order_problem(Tend / n, K, 2)
        p.scheme = replace(p.scheme, M=M, family=fam, method=SR)
        T, _ = oracle.run(p, nsteps=n)
        errs.append(np.abs(T - ref).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert orders[-1] == pytest.approx(expected, abs=0.3), (errs, orders)


def test_rejects_lobatto_with_one_node():
    sc = mi.Scheme(M=1, family=mi.LOBATTO, P=2, K=0, dt=0.3, method=SR)
    p = small_contact(sc)
    with pytest.raises(Exception):
        oracle.run(p, nsteps=1)
