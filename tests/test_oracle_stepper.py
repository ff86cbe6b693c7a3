"""Pins of the oracle's time stepper: predictor (Alg. 1), sweep (Alg. 2) and
residual (eq. residual) of paper §3, against facts that do not come from it.

  * decay of a discrete cosine eigenmode: K = 0 gives backward Euler on each
    interval; many sweeps give the collocation method (for 3 Lobatto nodes the
    (2,2) Pade approximant of exp) -- textbook stability functions;
  * heat balance of an insulated body (conduction conserves heat; the fast term
    injects q0|patch| or P_f per second);
  * the sweep's fixed point solves the discrete node-to-node equations
    (eqs. discrete-node-to-node / discrete-node-to-node-embedded), built and
    solved densely here;
  * residual contraction per sweep proportional to dt (property (i));
  * observed order min(K+1, collocation order, P) against the matrix
    exponential of the semi-discrete system (property (ii)).
"""
import math
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla

import mrsdc_inputs as mi
import oracle
from mrsdc_inputs.mesh import box
from quadref import moment_weights, std_nodes
from test_inputs import cos_mode, lam_h


def insulated_box(L=(0.2, 0.3, 0.5), nodes=(4, 5, 7), scheme=None):
    p = mi.patch_box(L=L, nodes=nodes, robin=False, scheme=scheme)
    p.coupling = None
    return p


def collocation_R(z, M, fam):
    """Stability function of the collocation method on the scheme's standard
    nodes for y' = -lam y, z = lam dt: solve (I + z Q) y = 1, R = y_M."""
    x = std_nodes(M, fam)
    Q = np.array([[float(w) for w in moment_weights(x, Fraction(0) if isinstance(x[0], Fraction) else 0, xm)]
                  for xm in x])
    y = np.linalg.solve(np.eye(M) + z * Q, np.ones(M))
    return y[-1]


@pytest.mark.parametrize("M,fam,P", [(3, mi.LOBATTO, 4), (5, mi.LOBATTO, 3), (3, mi.EQUI_NOLEFT, 2)])
def test_eigenmode_backward_euler_limit(M, fam, P):
    sc = mi.Scheme(M=M, family=fam, P=P, K=0, dt=40.0)
    p = insulated_box(scheme=sc)
    b = p.bodies[0]
    v = cos_mode(b)
    lam = lam_h(b.lengths, b.dims)
    p.T0 = 20.0 + 3.0 * v
    T, _ = oracle.run(p, nsteps=4)
    tau, *_ = oracle.weights(M, fam, P, sc.dt)
    R = np.prod([1.0 / (1.0 + lam * (tau[m] - tau[m - 1])) for m in range(1, M + 1)])
    assert np.abs(T - (20.0 + 3.0 * R**4 * v)).max() < 1e-11


@pytest.mark.parametrize("M,fam", [(3, mi.LOBATTO), (5, mi.LOBATTO), (3, mi.EQUI_NOLEFT)])
def test_eigenmode_collocation_limit(M, fam):
    sc = mi.Scheme(M=M, family=fam, P=3, K=40, dt=60.0)
    p = insulated_box(scheme=sc)
    b = p.bodies[0]
    v = cos_mode(b)
    lam = lam_h(b.lengths, b.dims)
    p.T0 = 20.0 + 3.0 * v
    T, _ = oracle.run(p, nsteps=3)
    z = lam * sc.dt
    R = collocation_R(z, M, fam)
    if (M, fam) == (3, mi.LOBATTO):
        pade = (1 - z / 2 + z * z / 12) / (1 + z / 2 + z * z / 12)
        assert R == pytest.approx(pade, rel=1e-13)
    assert np.abs(T - (20.0 + 3.0 * R**3 * v)).max() < 1e-11
    assert abs(R - math.exp(-z)) < 0.05 * math.exp(-z)  # sanity: a good approximation


def test_heat_balance_patch_insulated():
    sc = mi.Scheme(M=3, family=mi.LOBATTO, P=4, K=2, dt=0.5)
    p = mi.patch_box(L=(0.2, 0.3, 0.6), nodes=(4, 5, 9), robin=False, scheme=sc, width=0.06,
                     u_center=0.15, motion=mi.Motion(0.3, 0.2, 2.0, 0.3))
    b = p.bodies[0]
    p.T0 = p.T0 - 20.0  # linear, insulated: a shift keeps E - E0 free of cancellation
    E0 = b.mass @ p.T0
    T, _ = oracle.run(p, nsteps=6)
    gain = b.mass @ T - E0
    assert gain == pytest.approx(p.coupling.q0 * 0.06 * 0.06 * 6 * sc.dt, rel=1e-11)


def test_heat_balance_contact_insulated():
    sc = mi.Scheme(M=3, family=mi.LOBATTO, P=3, K=2, dt=0.4)
    p = mi.machine(stand_nodes=(4, 5, 11), stock_nodes=(3, 4, 5), stand_L=(0.2, 0.4, 1.0),
                   stock_L=(0.1, 0.3, 0.3), y_offset=0.05, robin=False, scheme=sc, period=2.0,
                   stroke=0.4, alpha=800.0, friction_W=75.0)
    m = np.concatenate([bb.mass for bb in p.bodies])
    p.T0 = p.T0 - 20.0
    E0 = m @ p.T0
    T, _ = oracle.run(p, nsteps=5)
    assert m @ T - E0 == pytest.approx(75.0 * 5 * sc.dt, rel=1e-10)


def fE_affine(p, t):
    """Matrix and offset of the affine map T -> f^E(T, t), probed column by column."""
    N = p.N
    e = oracle.fE(p, t, np.zeros(N))
    E = np.zeros((N, N))
    for i in range(N):
        x = np.zeros(N)
        x[i] = 1.0
        E[:, i] = oracle.fE(p, t, x) - e
    return E, e


def dense_node_to_node(p, t0, T0):
    """Solve the discrete node-to-node equations of one step densely.

    Unknowns T_{m,p} (p = 1..P) of the non-degenerate intervals, T_{m,P} = T_m.
    M T_{m,p} = M T_{m,p-1} + sum_j tilde s_{m,p,j} (f^I(T_j) + g)
                            + sum_q s_{m,p,q} f^E(T_{m,q}, tau_{m,q})
    """
    sc = p.scheme
    M, P, N = sc.M, sc.P, p.N
    tau, s, shat, stil, spq = oracle.weights(M, sc.family, P, sc.dt)
    b = p.bodies
    L = np.zeros((N, N))
    g = np.zeros(N)
    mass = np.zeros(N)
    off = p.offsets
    for i, bb in enumerate(b):
        sl = slice(off[i], off[i + 1])
        L[sl, sl] = bb.csr("K").toarray() + p.h[i] * bb.csr("R").toarray()
        g[sl] = p.h[i] * p.T_amb[i] * bb.rload
        mass[sl] = bb.mass
    ints = [m for m in range(1, M + 1) if tau[m] > tau[m - 1]]
    idx = {}
    for m in ints:
        for q in range(1, P + 1):
            idx[(m, q)] = len(idx)
    nU = len(idx) * N
    A = np.zeros((nU, nU))
    rhs = np.zeros(nU)

    def std_block(j):  # standard node j as (block index or None for T_n)
        k = j
        while k >= 1 and (k not in ints):
            k -= 1
        return None if k < 1 else idx[(k, P)]

    Ecache = {}
    for m in ints:
        for q in range(1, P + 1):
            Ecache[(m, q)] = fE_affine(p, t0 + tau[m - 1] + q * (tau[m] - tau[m - 1]) / P)
    for m in ints:
        for pp in range(1, P + 1):
            r = slice(idx[(m, pp)] * N, (idx[(m, pp)] + 1) * N)
            A[r, r] += np.diag(mass)
            if pp > 1:
                c = idx[(m, pp - 1)]
                A[r, c * N:(c + 1) * N] -= np.diag(mass)
            else:
                prev = std_block(m - 1)
                if prev is None:
                    rhs[r] += mass * T0
                else:
                    A[r, prev * N:(prev + 1) * N] -= np.diag(mass)
            for j in range(1, M + 1):
                w = stil[m, pp, j]
                rhs[r] += w * g
                blk = std_block(j)
                if blk is None:
                    rhs[r] += w * (-L @ T0)
                else:
                    A[r, blk * N:(blk + 1) * N] += w * L
            for q in range(1, P + 1):
                w = spq[m, pp, q]
                E, e = Ecache[(m, q)]
                c = idx[(m, q)]
                A[r, c * N:(c + 1) * N] -= w * E
                rhs[r] += w * e
    U = np.linalg.solve(A, rhs)
    last = idx[(ints[-1], P)]
    return U[last * N:(last + 1) * N]


@pytest.mark.parametrize("M,fam,P", [(3, mi.LOBATTO, 3), (3, mi.EQUI_NOLEFT, 2)])
def test_sweeps_converge_to_node_to_node_solution(M, fam, P):
    sc = mi.Scheme(M=M, family=fam, P=P, K=60, dt=0.25, pcg_rtol=1e-15)
    p = mi.machine(stand_nodes=(3, 3, 5), stock_nodes=(2, 3, 3), stand_L=(0.2, 0.4, 1.0),
                   stock_L=(0.1, 0.3, 0.3), y_offset=0.05, scheme=sc, period=2.0, stroke=0.4,
                   alpha=900.0, friction_W=60.0, h=30.0)
    T, st, res = oracle.run(p, nsteps=1, residuals=True)
    ref = dense_node_to_node(p, 0.0, p.T0)
    assert np.abs(T - ref).max() < 1e-11 * np.abs(ref).max()
    # the residual reaches round-off level of M T (the paper's collocation limit)
    mass = np.concatenate([bb.mass for bb in p.bodies])
    assert res[0, -1] < 1e-14 * np.abs(mass * T).max()
    assert res[0, 0] > 1e5 * res[0, -1]


def test_residual_contraction_proportional_to_dt():
    """Per-sweep contraction of the residual (eq. residual) halves with dt
    (property (i)); checked in the non-stiff regime of the unit-scale problem."""
    rates = []
    for dt in (0.01, 0.005, 0.0025):
        p = order_problem(dt, 4, 3, M=5)
        _, _, res = oracle.run(p, nsteps=1, residuals=True)
        r = res[0]
        rates.append(np.exp(np.mean(np.log(r[1:4] / r[0:3]))))
    assert rates[0] < 0.05
    assert rates[1] / rates[0] == pytest.approx(0.5, abs=0.12)
    assert rates[2] / rates[1] == pytest.approx(0.5, abs=0.12)


def order_problem(dt, K, P, M=3):
    """Unit box, k = rho c = 1: static patch with exchange alpha (T_fixed - T)
    plus flux, Robin elsewhere.  Linear and time-invariant, so the exact
    solution is a matrix exponential."""
    sc = mi.Scheme(M=M, family=mi.LOBATTO, P=P, K=K, dt=dt, pcg_rtol=1e-15)
    b = box((1.0, 1.0, 1.0), (3, 3, 4), 1.0, 1.0, ("x0", "y0", "z1"))
    p = mi.patch_box(scheme=sc, robin=False)
    p.bodies = [b]
    p.h, p.T_amb = [0.7], [1.0]
    p.coupling = mi.Patch(body=0, face="x1", width_u=0.8, width_v=0.55, u_center=0.45, q0=0.9,
                          alpha=3.0, T_fixed=2.0)
    p.motion = mi.Motion(0.5, 0.0, 1.0, 0.0)
    p.T0 = np.linspace(-1.0, 1.0, b.n) ** 2
    return p


def exact_order_solution(p, t):
    b = p.bodies[0]
    E, e = fE_affine(p, 0.0)
    A = -(b.csr("K").toarray() + p.h[0] * b.csr("R").toarray()) + E
    c = p.h[0] * p.T_amb[0] * b.rload + e
    Minv = 1.0 / b.mass
    J = Minv[:, None] * A
    Tinf = np.linalg.solve(A, -c)
    return Tinf + sla.expm(J * t) @ (p.T0 - Tinf)


@pytest.mark.parametrize("K,expected", [(0, 1), (1, 2), (2, 3), (3, 4), (4, 4)])
def test_observed_order(K, expected):
    """Order min(K+1, 4, P) for 3 Lobatto nodes (collocation order 4), P = 4,
    measured in the asymptotic range against the matrix exponential."""
    Tend = 0.2
    errs = []
    ref = exact_order_solution(order_problem(0.1, K, 4), Tend)
    for n in (32, 64, 128):
        p = order_problem(Tend / n, K, 4)
        T, _ = oracle.run(p, nsteps=n)
        errs.append(np.abs(T - ref).max())
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert orders[-1] == pytest.approx(expected, abs=0.3), (errs, orders)
