"""Linear thermo-elasticity of a box body on the Q1 mesh of its heat problem.

Seeded input generation only: the arrays a caller hands to the deformation
solve (the library and the oracle alike).  The method itself -- factorising
the stiffness once and solving for each output temperature field -- is not
here.

Small-strain isotropic elasticity with thermal strain alpha (T - T_ref) I
(the deformation model behind the paper's §5 deformation results, which
states only that it is linear elasticity driven by the temperature).  With
displacement basis phi_j e_b and test function phi_i e_a:

    K^{ab}_{ij} = int lam d_a phi_i d_b phi_j + mu d_b phi_i d_a phi_j
                  + mu delta_ab grad phi_i . grad phi_j
    f^a_i       = (3 lam + 2 mu) alpha int d_a phi_i (T - T_ref)
                = sum_j G^a_{ij} (T_j - T_ref),
    G^a_{ij}    = (3 lam + 2 mu) alpha int d_a phi_i phi_j

(traction-free faces, no body force).  On a tensor grid every integral is a
product of 1D integrals: stiffness int psi_a' psi_b', mass int psi_a psi_b
and the mixed int psi_a' psi_b.  DOF 3*node + c (c = x, y, z), nodes x
fastest; Dirichlet DOFs (u_c = 0 on a face) are removed from rows and
columns, which keeps the rest in node order, banded with half-bandwidth
about 3 (nx ny + nx + 1).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .mesh import FACES, Body

E_STEEL = 210e9  # Pa
NU_STEEL = 0.3
ALPHA_STEEL = 1.2e-5  # 1/K


def _one_d(n: int, L: float):
    """Dense 1D stiffness, mass and mixed (derivative on the row index)."""
    h = L / (n - 1)
    Kd = np.zeros((n, n))
    Md = np.zeros((n, n))
    Cd = np.zeros((n, n))
    for e in range(n - 1):
        i = np.array([e, e + 1])
        Kd[np.ix_(i, i)] += np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
        Md[np.ix_(i, i)] += np.array([[2.0, 1.0], [1.0, 2.0]]) * h / 6.0
        Cd[np.ix_(i, i)] += np.array([[-0.5, -0.5], [0.5, 0.5]])
    return Kd, Md, Cd


@dataclass
class Elastic:
    """The deformation problem of one body over its free DOFs."""

    n: int  # free displacement DOFs
    rowptr: np.ndarray  # int64 [n+1]
    col: np.ndarray  # int32
    K: np.ndarray  # SPD stiffness values
    g_rowptr: np.ndarray  # int64 [n+1], thermal load operator (n x nodes)
    g_col: np.ndarray  # int32
    G: np.ndarray
    free: np.ndarray  # int64 [n]: full DOF index 3*node + c of each free DOF
    n_nodes: int
    T_ref: float
    E: float
    nu: float
    alpha: float

    def csr(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.K, self.col, self.rowptr), shape=(self.n, self.n))

    def gcsr(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.G, self.g_col, self.g_rowptr), shape=(self.n, self.n_nodes))

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def half_bandwidth(self) -> int:
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        return int(np.abs(self.col.astype(np.int64) - rows).max())


def elastic_box(body: Body, fixed=(("z0", (0, 1, 2)),), E=E_STEEL, nu=NU_STEEL,
                alpha=ALPHA_STEEL, T_ref=20.0) -> Elastic:
    """Thermo-elastic operators on the nodes of a box body (built by
    mesh.box).  fixed: (face, components) pairs with u_c = 0 on that face;
    the default clamps the floor face z0 (the stand stands on it)."""
    nx, ny, nz = body.dims
    Lx, Ly, Lz = body.lengths
    one = [_one_d(nx, Lx), _one_d(ny, Ly), _one_d(nz, Lz)]
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    n = nx * ny * nz

    # node-pair pattern (the heat operator's 27-point pattern)
    rp = body.rowptr
    cn = body.col.astype(np.int64)
    npair = len(cn)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))

    def split(idx):
        return idx % nx, (idx // nx) % ny, idx // (nx * ny)

    ri, ci = split(rows), split(cn)
    Kd = [o[0][r, c] for o, r, c in zip(one, ri, ci)]
    Md = [o[1][r, c] for o, r, c in zip(one, ri, ci)]
    Cr = [o[2][r, c] for o, r, c in zip(one, ri, ci)]  # int psi_i' psi_j
    Cc = [o[2][c, r] for o, r, c in zip(one, ri, ci)]  # int psi_i psi_j'
    del ri, ci

    def D(a, b):
        """int d_a phi_i d_b phi_j for every node pair."""
        f = np.ones(npair)
        for d in range(3):
            if d == a and d == b:
                f = f * Kd[d]
            elif d == a:
                f = f * Cr[d]
            elif d == b:
                f = f * Cc[d]
            else:
                f = f * Md[d]
        return f

    Dm = [[D(a, b) for b in range(3)] for a in range(3)]
    lap = Dm[0][0] + Dm[1][1] + Dm[2][2]
    V = np.empty((npair, 3, 3))
    for a in range(3):
        for b in range(3):
            V[:, a, b] = lam * Dm[a][b] + mu * Dm[b][a] + (mu * lap if a == b else 0.0)
    del Dm, lap

    # DOF-level CSR: row 3i+a lists, per neighbour node j (sorted), 3j+0..2
    deg = np.diff(rp)
    drp = np.zeros(3 * n + 1, dtype=np.int64)
    drp[1:] = np.cumsum(np.repeat(3 * deg, 3))
    p = np.arange(npair, dtype=np.int64)
    local = p - rp[rows]
    vals = np.empty(9 * npair)
    dcol = np.empty(9 * npair, dtype=np.int64)
    for a in range(3):
        base = drp[3 * rows + a] + 3 * local
        for b in range(3):
            vals[base + b] = V[:, a, b]
            dcol[base + b] = 3 * cn + b
    del V, base
    Kfull = sp.csr_matrix((vals, dcol, drp), shape=(3 * n, 3 * n))
    del vals, dcol

    # thermal load operator on the node pattern: G^a_ij
    s = (3.0 * lam + 2.0 * mu) * alpha
    gv = np.empty((npair, 3))
    for a in range(3):
        f = np.full(npair, s)
        for d in range(3):
            f = f * (Cr[d] if d == a else Md[d])
        gv[:, a] = f
    grp = np.zeros(3 * n + 1, dtype=np.int64)
    grp[1:] = np.cumsum(np.repeat(deg, 3))
    gval = np.empty(3 * npair)
    gcol = np.empty(3 * npair, dtype=np.int64)
    for a in range(3):
        pos = grp[3 * rows + a] + local
        gval[pos] = gv[:, a]
        gcol[pos] = cn
    Gfull = sp.csr_matrix((gval, gcol, grp), shape=(3 * n, n))
    del gval, gcol, gv

    keep = np.ones(3 * n, dtype=bool)
    for face, comps in fixed:
        axis, side = FACES[face]
        dims = (nx, ny, nz)
        target = 0 if side == 0 else dims[axis] - 1
        nodes = np.nonzero(split(np.arange(n))[axis] == target)[0]
        for c in comps:
            keep[3 * nodes + c] = False
    free = np.nonzero(keep)[0]
    K = Kfull[free][:, free].tocsr()
    K.sort_indices()
    G = Gfull[free].tocsr()
    G.sort_indices()
    return Elastic(n=len(free), rowptr=K.indptr.astype(np.int64), col=K.indices.astype(np.int32),
                   K=K.data.copy(), g_rowptr=G.indptr.astype(np.int64),
                   g_col=G.indices.astype(np.int32), G=G.data.copy(), free=free, n_nodes=n,
                   T_ref=T_ref, E=E, nu=nu, alpha=alpha)
