"""Pins of the oracle's fast term f^E (paper §2: the contact/friction terms of
eqs. femContFix/femContMov on Gamma_R(t), the matrices M_B, C_B (eq. defCB) and
the friction source b_X(t)).

Independent derivations used here:
  * for fields that bilinear interpolation reproduces exactly (a + b u + c v + d uv)
    each face integral factorises into 1D moments of clipped hat functions,
    evaluated in closed form (trapezoid/Simpson on each linear piece);
  * on matching grids the coupling matrix equals the face mass matrix, taken
    from the separately assembled Robin operator of that face.
"""
import numpy as np
import pytest

import mrsdc_inputs as mi
import oracle
from mrsdc_inputs.mesh import box


def hat_moments(x, a, lo, hi):
    """(int psi_a, int psi_a * t) over [lo,hi] for the hat psi_a on nodes x."""
    m0 = m1 = 0.0
    pieces = []
    if a > 0:
        pieces.append((x[a - 1], x[a], lambda t, a=a: (t - x[a - 1]) / (x[a] - x[a - 1])))
    if a < len(x) - 1:
        pieces.append((x[a], x[a + 1], lambda t, a=a: (x[a + 1] - t) / (x[a + 1] - x[a])))
    for c, d, f in pieces:
        e, g = max(c, lo), min(d, hi)
        if g <= e:
            continue
        mid = 0.5 * (e + g)
        m0 += (g - e) * (f(e) + f(g)) / 2.0                                 # exact: linear
        m1 += (g - e) * (f(e) * e + 4 * f(mid) * mid + f(g) * g) / 6.0      # exact: quadratic
    return m0, m1


def face_integral(F, ids_off, coef, lo_u, hi_u, lo_v, hi_v, vshift=0.0):
    """out[node] = int_{rect} phi_node (c0 + c1 u + c2 v + c3 u v) for nodes of grid F
    (grid v coordinates shifted by vshift)."""
    out = {}
    v = F.v + vshift
    for a in range(F.nu):
        mu = hat_moments(F.u, a, lo_u, hi_u)
        if mu == (0.0, 0.0):
            continue
        for b in range(F.nv):
            mv = hat_moments(v, b, lo_v, hi_v)
            val = coef[0] * mu[0] * mv[0] + coef[1] * mu[1] * mv[0] + coef[2] * mu[0] * mv[1] \
                + coef[3] * mu[1] * mv[1]
            out[ids_off + F.ids[a * F.nv + b]] = val
    return out


def bilinear_field(F, c, vshift=0.0):
    U, V = np.meshgrid(F.u, F.v + vshift, indexing="ij")
    return (c[0] + c[1] * U + c[2] * V + c[3] * U * V).ravel()


@pytest.mark.parametrize("t", [0.0, 0.37, 1.1])
@pytest.mark.parametrize("alpha", [0.0, 40.0])
def test_patch_against_clipped_hat_moments(t, alpha):
    p = mi.patch_box(L=(0.2, 0.3, 0.7), nodes=(4, 7, 12), alpha=alpha, T_fixed=30.0, width=0.083,
                     u_center=0.13, motion=mi.Motion(0.33, 0.21, 1.7, 0.4))
    b = p.bodies[0]
    F = b.faces["x1"]
    cT = (21.0, 3.0, -2.0, 5.0)
    T = np.full(p.N, 7.0)
    T[F.ids] = bilinear_field(F, cT)
    got = oracle.fE(p, t, T)
    c = p.coupling
    s = p.motion.s(t)
    lo_u, hi_u = c.u_center - c.width_u / 2, c.u_center + c.width_u / 2
    lo_v, hi_v = s - c.width_v / 2, s + c.width_v / 2
    # integrand q0 + alpha (T_fixed - T) = (q0 + alpha(Tf - c0)) - alpha c1 u - alpha c2 v - alpha c3 uv
    coef = (c.q0 + alpha * (c.T_fixed - cT[0]), -alpha * cT[1], -alpha * cT[2], -alpha * cT[3])
    ref = np.zeros(p.N)
    for k, v in face_integral(F, 0, coef, lo_u, hi_u, lo_v, hi_v).items():
        ref[k] = v
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref).max()
    # total patch heat for alpha = 0 is q0 * |patch| when the patch lies on the face
    if alpha == 0.0:
        assert got.sum() == pytest.approx(c.q0 * c.width_u * c.width_v, rel=1e-13)


def small_machine(**kw):
    base = dict(stand_nodes=(4, 6, 13), stock_nodes=(3, 5, 7), stand_L=(0.2, 0.4, 1.0),
                stock_L=(0.15, 0.23, 0.31), y_offset=0.07, alpha=850.0, friction_W=120.0,
                period=3.0, stroke=0.5, nsteps=3)
    base.update(kw)
    return mi.machine(**base)


@pytest.mark.parametrize("t", [0.0, 0.4, 1.3, 2.2])
def test_contact_against_clipped_hat_moments(t):
    """Non-matching stand/stock grids, bilinear temperature fields on both faces."""
    p = small_machine()
    c = p.coupling
    st, sk = p.bodies
    F, G = st.faces["x1"], sk.faces["x0"]
    Gf = mi.Face(u=c.mov_u, v=c.mov_v, ids=G.ids)  # stock grid in the stand's face frame
    s = p.motion.s(t)
    cf = (20.5, 2.0, -1.5, 3.0)      # T on the stand face as a function of (u, v)
    cm = (24.0, -3.0, 0.5, -2.0)     # T on the stock face, same frame
    T = np.full(p.N, 0.0)
    off = st.n
    T[F.ids] = bilinear_field(F, cf)
    T[off + G.ids] = bilinear_field(Gf, cm, vshift=s)
    got = oracle.fE(p, t, T)
    lo_u, hi_u = max(F.u[0], Gf.u[0]), min(F.u[-1], Gf.u[-1])
    lo_v, hi_v = max(F.v[0], Gf.v[0] + s), min(F.v[-1], Gf.v[-1] + s)
    area = (hi_u - lo_u) * (hi_v - lo_v)
    qf = c.friction_W / area
    d = [cm[i] - cf[i] for i in range(4)]
    ref = np.zeros(p.N)
    cfix = (c.alpha * d[0] + c.split * qf, c.alpha * d[1], c.alpha * d[2], c.alpha * d[3])
    cmov = (-c.alpha * d[0] + (1 - c.split) * qf, -c.alpha * d[1], -c.alpha * d[2], -c.alpha * d[3])
    for k, v in face_integral(F, 0, cfix, lo_u, hi_u, lo_v, hi_v).items():
        ref[k] += v
    for k, v in face_integral(Gf, off, cmov, lo_u, hi_u, lo_v, hi_v, vshift=s).items():
        ref[k] += v
    assert np.abs(got - ref).max() < 1e-11 * np.abs(ref).max()
    # energy: the exchange terms cancel between the bodies, friction adds P_f
    assert got.sum() == pytest.approx(c.friction_W, rel=1e-12)


def test_contact_matching_grids_equals_face_mass():
    """Stock face grid identical to the stand face grid, no offset: C_B = M_B = face mass."""
    st = box((0.2, 0.3, 0.5), (3, 4, 6), 15.0, 3.6e6, ("x1",))
    sk = box((0.1, 0.3, 0.5), (2, 4, 6), 15.0, 3.6e6, ("x0",))
    p = small_machine()
    p.bodies = [st, sk]
    p.T0 = np.zeros(st.n + sk.n)
    F, G = st.faces["x1"], sk.faces["x0"]
    p.coupling = mi.Contact(0, "x1", 1, "x0", mov_u=G.u.copy(), mov_v=G.v.copy(), alpha=700.0,
                            friction_W=90.0, split=0.3)
    p.motion = mi.Motion(0.0, 0.0, 1.0, 0.0)
    rng = np.random.default_rng(5)
    T = rng.uniform(10, 30, p.N)
    got = oracle.fE(p, 0.0, T)
    Rs = st.csr("R")  # face mass of the stand's x1 face (assembled as a Robin term)
    Tm_on_fix = np.zeros(st.n)
    Tm_on_fix[F.ids] = T[st.n + G.ids]   # grids coincide node by node
    area = 0.3 * 0.5
    ones_face = np.zeros(st.n)
    ones_face[F.ids] = 1.0
    ref_fix = 700.0 * (Rs @ (Tm_on_fix - T[:st.n] * ones_face)) + 0.3 * 90.0 / area * (Rs @ ones_face)
    assert np.abs(got[:st.n] - ref_fix).max() < 1e-12 * np.abs(ref_fix).max()
    Rk = sk.csr("R")
    Tf_on_mov = np.zeros(sk.n)
    Tf_on_mov[G.ids] = T[F.ids]
    ones_m = np.zeros(sk.n)
    ones_m[G.ids] = 1.0
    ref_mov = 700.0 * (Rk @ (Tf_on_mov - T[st.n:] * ones_m)) + 0.7 * 90.0 / area * (Rk @ ones_m)
    assert np.abs(got[st.n:] - ref_mov).max() < 1e-12 * np.abs(ref_mov).max()


def test_no_overlap_gives_zero():
    p = small_machine()
    p.motion = mi.Motion(5.0, 0.0, 1.0, 0.0)  # stock far above the stand
    got = oracle.fE(p, 0.0, np.full(p.N, 20.0))
    assert np.all(got == 0.0)


@pytest.mark.parametrize("nodes", [(3, 3, 3), (4, 4, 6)])
def test_implicit_solve_matches_dense(nodes):
    """One implicit node solve (diag(m) + dtau (K + h R)) x = b vs numpy's dense LU."""
    p = mi.patch_box(L=(0.2, 0.2, 0.3), nodes=nodes, h=25.0)
    b = p.bodies[0]
    A = np.diag(b.mass) + 0.7 * (b.csr("K").toarray() + 25.0 * b.csr("R").toarray())
    rng = np.random.default_rng(1)
    rhs = rng.uniform(-1, 1, b.n) * b.mass * 20
    x, it = oracle.solve(p, 0.7, rhs, x0=np.full(b.n, 20.0), rtol=1e-14)
    ref = np.linalg.solve(A, rhs)
    assert np.abs(x - ref).max() < 1e-12 * np.abs(ref).max()
    assert it > 0
    # stiff case: large dtau makes conduction dominate
    A = np.diag(b.mass) + 1e4 * (b.csr("K").toarray() + 25.0 * b.csr("R").toarray())
    x, it = oracle.solve(p, 1e4, rhs, rtol=1e-14)
    assert np.abs(x - np.linalg.solve(A, rhs)).max() < 1e-10 * np.abs(x).max()
