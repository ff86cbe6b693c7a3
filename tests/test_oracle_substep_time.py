"""Pins of the times at which the oracle evaluates the fast term f^E.

Alg. 1 steps each embedded node with f^E taken at the LEFT end of the substep,
f^E(T_{m,p-1}, tau_{m,p-1}); Alg. 2's quadratures I_{m-1}^m and I_{m,p-1}^p
(eqs. standard_quad, embedded_quad) use f^E at the embedded nodes
tau_{m,q}, q = 1..P (equidistant, no left node, §3).

On an insulated body with no exchange (h = 0, alpha = 0) conduction conserves
heat: 1^T K = 0, so 1^T f*_m = 0 and 1^T F_j = 0 and only the patch injects
heat, at the rate Q(t) = q0 |patch(t) n face| (the hat functions sum to one on
the face).  Summing the substep formulas with the lumped mass:

  * K = 0 (predictor only):  E_{n+1} - E_n = sum_{m,p} dtau_{m,p} Q(tau_{m,p-1})
    -- a left Riemann sum over the substeps;
  * K >= 1 (the last sweep's substeps add up the embedded quadrature, the
    correction terms E^new - E^old cancel):
        E_{n+1} - E_n = sum_m sum_q hat s_{m,q} Q(tau_{m,q}).

A patch sliding partly off the face makes Q(t) vary within the step, so a
right-point (tau_{m,p}) substep or a shifted quadrature node fails these pins.
Q and the weights come from closed forms and exact moment matching here, not
from the oracle.
"""
import math

import numpy as np
import pytest

import mrsdc_inputs as mi
import oracle
from quadref import reference

LZ = 0.6
WU, WV, UC, Q0 = 0.06, 0.12, 0.15, 1500.0


def sliding_patch_problem(scheme, motion):
    p = mi.patch_box(L=(0.2, 0.3, LZ), nodes=(4, 5, 9), robin=False, scheme=scheme, width=WU,
                     u_center=UC, motion=motion)
    p.coupling.width_v = WV
    p.coupling.q0 = Q0
    p.coupling.alpha = 0.0
    p.T0 = p.T0 - 20.0  # insulated and linear: a shift keeps the energy free of cancellation
    return p


def heat_rate(motion, t):
    """q0 times the area of the patch rectangle inside the face [0,0.3] x [0,LZ]."""
    s = motion.s(t)
    ov = max(0.0, min(s + 0.5 * WV, LZ) - max(s - 0.5 * WV, 0.0))
    return Q0 * WU * ov


def node_times(M, fam, P, dt):
    tau, *_ = reference(M, fam, P, dt)
    return tau


MOTION = mi.Motion(s0=0.56, a=0.16, period=2.0, phase=0.3)


@pytest.mark.parametrize("M,fam,P", [(3, mi.LOBATTO, 4), (3, mi.EQUI_NOLEFT, 3),
                                     (5, mi.LOBATTO, 2)])
def test_predictor_uses_left_substep_time(M, fam, P):
    dt, nsteps = 0.4, 3
    sc = mi.Scheme(M=M, family=fam, P=P, K=0, dt=dt, pcg_rtol=1e-14)
    p = sliding_patch_problem(sc, MOTION)
    m = p.bodies[0].mass
    E0 = m @ p.T0
    T, _ = oracle.run(p, nsteps=nsteps)
    tau = node_times(M, fam, P, dt)
    left = right = 0.0
    for n in range(nsteps):
        tn = n * dt
        for mm in range(1, M + 1):
            dtm = tau[mm] - tau[mm - 1]
            for pp in range(1, P + 1):
                left += dtm / P * heat_rate(MOTION, tn + tau[mm - 1] + (pp - 1) * dtm / P)
                right += dtm / P * heat_rate(MOTION, tn + tau[mm - 1] + pp * dtm / P)
    gain = m @ T - E0
    # the two Riemann sums differ well beyond the tolerance: the pin can tell them apart
    assert abs(left - right) > 1e-4 * abs(left)
    assert gain == pytest.approx(left, rel=1e-11, abs=1e-12 * abs(E0))


@pytest.mark.parametrize("M,fam,P,K", [(3, mi.LOBATTO, 4, 1), (3, mi.LOBATTO, 4, 3),
                                       (3, mi.EQUI_NOLEFT, 3, 2), (5, mi.LOBATTO, 2, 2)])
def test_sweeps_integrate_fE_at_embedded_nodes(M, fam, P, K):
    dt, nsteps = 0.4, 3
    sc = mi.Scheme(M=M, family=fam, P=P, K=K, dt=dt, pcg_rtol=1e-14)
    p = sliding_patch_problem(sc, MOTION)
    m = p.bodies[0].mass
    E0 = m @ p.T0
    T, _ = oracle.run(p, nsteps=nsteps)
    tau, s, shat, stil, spq = reference(M, fam, P, dt)
    quad = 0.0
    shifted = 0.0  # the same weights on the left-shifted nodes tau_{m,q-1}
    for n in range(nsteps):
        tn = n * dt
        for mm in range(1, M + 1):
            dtm = tau[mm] - tau[mm - 1]
            for q in range(1, P + 1):
                quad += shat[mm, q] * heat_rate(MOTION, tn + tau[mm - 1] + q * dtm / P)
                shifted += shat[mm, q] * heat_rate(MOTION, tn + tau[mm - 1] + (q - 1) * dtm / P)
    gain = m @ T - E0
    assert abs(quad - shifted) > 1e-4 * abs(quad)
    assert gain == pytest.approx(quad, rel=1e-11, abs=1e-12 * abs(E0))


def test_heat_rate_closed_form_against_oracle_fE():
    """The closed-form injected power equals the sum of the oracle's f^E
    (patch partly off the face, alpha = 0) -- ties the two pins above to the
    oracle's own f^E at a given time."""
    sc = mi.Scheme(M=3, family=mi.LOBATTO, P=2, K=0, dt=0.4)
    p = sliding_patch_problem(sc, MOTION)
    for t in (0.0, 0.13, 0.5, 0.77, 1.21):
        e = oracle.fE(p, t, np.zeros(p.N))
        assert e.sum() == pytest.approx(heat_rate(MOTION, t), rel=1e-13)
    # the motion really slides the patch across the face edge z = LZ
    s = [MOTION.s(t) for t in np.linspace(0.0, 2.0, 41)]
    assert max(s) + 0.5 * WV > LZ > min(s) + 0.5 * WV
    assert not math.isclose(heat_rate(MOTION, 0.0), heat_rate(MOTION, 0.4))
