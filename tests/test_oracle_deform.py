"""Pins of the thermo-elastic deformation inputs and oracle (§5: linear
elasticity with the temperature as load, K_u u = G (T - T_ref)), against
facts that do not come from them:

  * uniform heating of a body held only by three symmetry rollers expands
    freely: u = alpha dT (x - x_corner), stress free, which Q1 reproduces
    exactly (a linear field);
  * the unconstrained stiffness annihilates the six rigid-body motions (the
    rotations only with the correct lambda / mu form);
  * the Kronecker-product assembly equals a textbook element-by-element
    assembly, B^T D B and B^T D m with 2x2x2 Gauss points, on a small mesh;
  * the clamped stiffness is symmetric positive definite; Maxwell-Betti
    reciprocity u1 . f2 = u2 . f1 for two temperature fields.
"""
import itertools

import numpy as np
import pytest

import oracle.deform as od
from mrsdc_inputs.elastic import elastic_box
from mrsdc_inputs.mesh import box

ROLLERS = (("x0", (0,)), ("y0", (1,)), ("z0", (2,)))


def body(L=(0.2, 0.3, 0.5), nodes=(4, 5, 7)):
    return box(L, nodes, 15.0, 3.6e6, ())


@pytest.mark.parametrize("L,nodes", [((0.2, 0.3, 0.5), (4, 5, 7)), ((0.4, 0.4, 1.6), (3, 4, 9))])
def test_uniform_heating_expands_freely(L, nodes):
    b = body(L, nodes)
    el = elastic_box(b, fixed=ROLLERS)
    dT = 12.5
    u = od.deform(el, np.full(b.n, el.T_ref + dT))
    exact = (el.alpha * dT * b.coords).ravel()[el.free]
    assert np.abs(u - exact).max() <= 1e-12 * np.abs(exact).max()


def test_rigid_body_modes_are_in_the_kernel():
    b = body()
    el = elastic_box(b, fixed=())
    K = el.csr()
    X = b.coords - b.coords.mean(axis=0)
    modes = []
    for c in range(3):
        t = np.zeros((b.n, 3))
        t[:, c] = 1.0
        modes.append(t)
    for a, c in ((0, 1), (1, 2), (2, 0)):
        r = np.zeros((b.n, 3))
        r[:, a] = -X[:, c]
        r[:, c] = X[:, a]
        modes.append(r)
    scale = np.abs(K.data).max() * np.abs(X).max()
    for m in modes:
        assert np.abs(K @ m.ravel()).max() <= 1e-12 * scale


def _element_reference(b, E, nu, alpha):
    """Element-by-element Q1 assembly with 2x2x2 Gauss points."""
    nx, ny, nz = b.dims
    hx, hy, hz = (L / (n - 1) for L, n in zip(b.lengths, b.dims))
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] += 2 * mu
    D[np.arange(3, 6), np.arange(3, 6)] = mu
    m = np.array([1, 1, 1, 0, 0, 0.0])
    K = np.zeros((3 * b.n, 3 * b.n))
    G = np.zeros((3 * b.n, b.n))
    g = 1 / np.sqrt(3.0)
    corners = list(itertools.product((0, 1), repeat=3))  # (dx, dy, dz)
    for ez, ey, ex in itertools.product(range(nz - 1), range(ny - 1), range(nx - 1)):
        nodes = [(ex + a) + nx * ((ey + c) + ny * (ez + d)) for a, c, d in corners]
        Ke = np.zeros((24, 24))
        Ge = np.zeros((24, 8))
        for qx, qy, qz in itertools.product((-g, g), repeat=3):
            xi = np.array([(1 + qx) / 2, (1 + qy) / 2, (1 + qz) / 2])
            N = np.zeros(8)
            dN = np.zeros((8, 3))
            for k, (a, c, d) in enumerate(corners):
                fx = xi[0] if a else 1 - xi[0]
                fy = xi[1] if c else 1 - xi[1]
                fz = xi[2] if d else 1 - xi[2]
                N[k] = fx * fy * fz
                dN[k] = [(1 if a else -1) / hx * fy * fz, fx * (1 if c else -1) / hy * fz,
                         fx * fy * (1 if d else -1) / hz]
            B = np.zeros((6, 24))
            for k in range(8):
                B[0, 3 * k] = dN[k, 0]
                B[1, 3 * k + 1] = dN[k, 1]
                B[2, 3 * k + 2] = dN[k, 2]
                B[3, 3 * k], B[3, 3 * k + 1] = dN[k, 1], dN[k, 0]
                B[4, 3 * k + 1], B[4, 3 * k + 2] = dN[k, 2], dN[k, 1]
                B[5, 3 * k], B[5, 3 * k + 2] = dN[k, 2], dN[k, 0]
            w = hx * hy * hz / 8
            Ke += w * B.T @ D @ B
            Ge += w * alpha * np.outer(B.T @ D @ m, N)
        dofs = np.array([3 * nd + c for nd in nodes for c in range(3)])
        K[np.ix_(dofs, dofs)] += Ke
        G[np.ix_(dofs, nodes)] += Ge
    return K, G


def test_kronecker_assembly_matches_element_assembly():
    b = body((0.2, 0.3, 0.5), (3, 4, 3))
    el = elastic_box(b, fixed=())
    Kr, Gr = _element_reference(b, el.E, el.nu, el.alpha)
    K = el.csr().toarray()
    G = el.gcsr().toarray()
    assert np.abs(K - Kr).max() <= 1e-12 * np.abs(Kr).max()
    assert np.abs(G - Gr).max() <= 1e-12 * np.abs(Gr).max()


def test_clamped_spd_and_reciprocity():
    b = body()
    el = elastic_box(b)
    K = el.csr().toarray()
    assert np.abs(K - K.T).max() == 0.0
    np.linalg.cholesky(K)
    rng = np.random.default_rng(5)
    T1 = 20 + rng.uniform(-5, 5, b.n)
    T2 = 20 + rng.uniform(-5, 5, b.n)
    solve = od.Deformation(el)
    u1, u2 = solve(T1), solve(T2)
    f1, f2 = solve.load(T1), solve.load(T2)
    assert u1 @ f2 == pytest.approx(u2 @ f1, rel=1e-12)
    assert np.abs(K @ u1 - f1).max() <= 1e-12 * np.abs(f1).max()
