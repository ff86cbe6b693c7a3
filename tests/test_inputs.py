"""Pins of the seeded inputs: the assembled Q1 operators both sides receive.

Invariants fixed by the finite element definitions of paper §2 (eq. femDiscr
and the matrices defined after it) and by textbook facts about Q1 elements.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import mrsdc_inputs as mi
from mrsdc_inputs.mesh import box

K, RC = 15.0, 3.6e6


@pytest.mark.parametrize("L,nodes", [((0.2, 0.3, 0.5), (3, 4, 6)), ((0.2, 0.2, 0.8), (9, 9, 33)),
                                     ((1.0, 0.5, 0.25), (5, 2, 3))])
def test_q1_invariants(L, nodes):
    b = box(L, nodes, K, RC, ("x0", "y1", "z0"))
    Km, Rm = b.csr("K"), b.csr("R")
    n = b.n
    # conduction conserves heat: constants are in the kernel of K
    assert np.abs(Km @ np.ones(n)).max() < 1e-12 * np.abs(b.K).max()
    assert abs(Km - Km.T).max() < 1e-14 * np.abs(b.K).max()
    assert abs(Rm - Rm.T).max() == 0.0
    # lumped mass sums to rho c |Omega|
    assert b.mass.sum() == pytest.approx(RC * L[0] * L[1] * L[2], rel=1e-13)
    # Robin load integrates 1 over the three Robin faces
    area = L[1] * L[2] + L[0] * L[2] + L[0] * L[1]
    assert b.rload.sum() == pytest.approx(area, rel=1e-13)
    # R is positive semidefinite and supported on Robin-face nodes only
    assert np.all(np.linalg.eigvalsh(Rm.toarray()) > -1e-15)
    # stiffness is positive semidefinite with a one-dimensional kernel
    ev = np.linalg.eigvalsh(Km.toarray())
    assert ev[0] > -1e-12 and ev[1] > 1e-6


def test_q1_element_matrix_cube():
    """A single unit-cube Q1 element: textbook stiffness entries (diagonal 1/3,
    face neighbour 0, edge neighbour -1/12, opposite corner -1/12)."""
    b = box((1.0, 1.0, 1.0), (2, 2, 2), 1.0, 1.0)
    Kd = b.csr("K").toarray()
    assert Kd[0, 0] == pytest.approx(1.0 / 3.0)
    assert Kd[0, 1] == pytest.approx(0.0, abs=1e-16)   # (1,0,0): cube edge neighbour
    assert Kd[0, 3] == pytest.approx(-1.0 / 12.0)      # (1,1,0): face diagonal
    assert Kd[0, 7] == pytest.approx(-1.0 / 12.0)      # (1,1,1): body diagonal
    # consistent-mass row sums of a unit cube: 1/8 each
    assert np.allclose(b.mass, 1.0 / 8.0)
    # full pattern is stored (explicit zeros kept)
    assert b.nnz == 64


def lam_h(L, nodes, k=K, rc=RC):
    """Discrete eigenvalue of the sampled cosine mode under K v = lam M_lumped v."""
    mk, mm = [], []
    for Ld, n in zip(L, nodes):
        h = Ld / (n - 1)
        th = np.pi * h / Ld
        mk.append((2 - 2 * np.cos(th)) / h**2)
        mm.append((4 + 2 * np.cos(th)) / 6)
    return k / rc * (mk[0] * mm[1] * mm[2] + mm[0] * mk[1] * mm[2] + mm[0] * mm[1] * mk[2])


def cos_mode(b):
    x = b.coords
    L = b.lengths
    return np.cos(np.pi * x[:, 0] / L[0]) * np.cos(np.pi * x[:, 1] / L[1]) * np.cos(np.pi * x[:, 2] / L[2])


@pytest.mark.parametrize("L,nodes", [((0.2, 0.3, 0.5), (4, 5, 7)), ((0.2, 0.2, 0.8), (9, 9, 33))])
def test_cosine_mode_is_discrete_eigenvector(L, nodes):
    b = box(L, nodes, K, RC)
    v = cos_mode(b)
    lam = lam_h(L, nodes)
    Kv = b.csr("K") @ v
    assert np.abs(Kv - lam * b.mass * v).max() < 1e-12 * np.abs(Kv).max()
    # continuum limit: lam_h -> (k/rc) pi^2 sum 1/L^2 as h -> 0
    fine = lam_h(L, (401, 401, 401))
    exact = K / RC * np.pi**2 * sum(1 / l**2 for l in L)
    assert fine == pytest.approx(exact, rel=1e-4)


def test_face_grids_and_machine_sizes():
    p = mi.box_patch_2673()
    assert (p.N, p.nnz) == (2673, 60625)
    b = p.bodies[0]
    f = b.faces["x1"]
    assert np.allclose(b.coords[f.ids, 0], 0.2)
    assert np.allclose(b.coords[f.ids.reshape(f.nu, f.nv), 1], f.u[:, None])
    assert np.allclose(b.coords[f.ids.reshape(f.nu, f.nv), 2], f.v[None, :])
    m = mi.machine(stand_nodes=(5, 5, 9), stock_nodes=(4, 4, 5))
    assert m.N == 5 * 5 * 9 + 4 * 4 * 5
    # the rail face of the stand and the contact face of the stock carry no Robin term
    st, sk = m.bodies
    inner = st.faces["x1"].ids.reshape(5, 9)[1:-1, 1:-1].ravel()
    assert np.all(st.rload[inner] == 0)
    inner = sk.faces["x0"].ids.reshape(4, 5)[1:-1, 1:-1].ravel()
    assert np.all(sk.rload[inner] == 0)


def test_seeded_inputs_are_reproducible():
    a, b = mi.box_patch_2673(), mi.box_patch_2673()
    assert np.array_equal(a.T0, b.T0)
    s0 = mi.scenario_params(3)[:4]
    assert s0 == mi.scenario_params(3)[:4]
    assert 5 <= s0[0] <= 25 and 500 <= s0[1] <= 2000 and 50 <= s0[2] <= 400 and 2 <= s0[3] <= 8
