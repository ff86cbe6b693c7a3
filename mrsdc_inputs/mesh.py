"""Structured-box Q1 (trilinear) finite element operators.

Seeded input generation only: these arrays are what a caller hands to the
time stepper (the library and the oracle alike).  Nothing here belongs to the
time-stepping method itself.

Discretisation (paper §2, eq. femDiscr and the definitions that follow it):
  * stiffness  K_ij = k * int grad(phi_i) . grad(phi_j) dx   (K = -A_X)
  * unit Robin boundary mass R_ij = int_{Gamma_Robin} phi_i phi_j dS
    (B_X,env = -h R), and the Robin load r_i = int_{Gamma_Robin} phi_i dS
    (b_X,env = h T_env r)
  * row-sum lumped mass m_i = rho*c * sum_j int phi_i phi_j dx (paper §2,
    the sentence after eq. coupledFEM)

On an axis-aligned box with a tensor grid every one of these integrals
factorises into 1D integrals of products of hat functions, so the global
operators are sums of Kronecker products of 1D matrices:
  K = k (Mz (x) My (x) Kx + Mz (x) Ky (x) Mx + Kz (x) My (x) Mx)
with the 1D stiffness Kx = int psi_a' psi_b' and mass Mx = int psi_a psi_b.
Nodes are numbered x fastest: idx = ix + nx*(iy + ny*iz).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

# face name -> (axis, side)
FACES = {"x0": (0, 0), "x1": (0, 1), "y0": (1, 0), "y1": (1, 1), "z0": (2, 0), "z1": (2, 1)}


def _one_d(n: int, L: float, x=None):
    """Dense 1D stiffness, consistent mass and lumped mass on n nodes (uniform
    on [0, L] unless the sorted node coordinates x are given)."""
    uniform = x is None
    x = np.linspace(0.0, L, n) if uniform else np.asarray(x, dtype=np.float64)
    assert len(x) == n and np.all(np.diff(x) > 0)
    Kd = np.zeros((n, n))
    Md = np.zeros((n, n))
    for e in range(n - 1):
        # one spacing for a uniform grid: every cell's entries the same numbers
        h = L / (n - 1) if uniform else x[e + 1] - x[e]
        i = np.array([e, e + 1])
        Kd[np.ix_(i, i)] += np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
        Md[np.ix_(i, i)] += np.array([[2.0, 1.0], [1.0, 2.0]]) * h / 6.0
    return Kd, Md, Md.sum(axis=1), x


def jittered_nodes(n: int, L: float, rng, amp: float = 0.2):
    """n sorted node coordinates on [0, L]: the uniform ones with every interior
    node moved by U[-amp, amp] times the spacing (a graded, irregular 1D mesh;
    amp < 0.5 keeps the order)."""
    x = np.linspace(0.0, L, n)
    if n > 2:
        x[1:-1] += rng.uniform(-amp, amp, size=n - 2) * (L / (n - 1))
    return x


@dataclass
class Face:
    """A tensor grid of face nodes.

    u, v: sorted 1D node coordinates along the face's two in-plane axes (the
    lower-numbered box axis is u).  ids[a*nv + b] is the body-local node index
    of grid point (u[a], v[b]).
    """

    u: np.ndarray
    v: np.ndarray
    ids: np.ndarray  # int32, length nu*nv

    @property
    def nu(self) -> int:
        return len(self.u)

    @property
    def nv(self) -> int:
        return len(self.v)


@dataclass
class Body:
    n: int
    rowptr: np.ndarray  # int64 [n+1]
    col: np.ndarray  # int32 [nnz], sorted within a row
    K: np.ndarray  # float64 [nnz]
    R: np.ndarray  # float64 [nnz], unit-coefficient Robin mass on K's pattern
    mass: np.ndarray  # float64 [n], lumped
    rload: np.ndarray  # float64 [n], int_{Robin} phi_i
    coords: np.ndarray  # float64 [n,3]
    faces: dict = field(default_factory=dict)  # name -> Face
    dims: tuple = ()  # (nx, ny, nz)
    lengths: tuple = ()  # (Lx, Ly, Lz)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def csr(self, which: str = "K") -> sp.csr_matrix:
        vals = {"K": self.K, "R": self.R}[which]
        return sp.csr_matrix((vals, self.col, self.rowptr), shape=(self.n, self.n))


def box(L, nodes, k: float, rho_c: float, robin_faces=(), axes=None) -> Body:
    """Q1 operators of the box [0,Lx]x[0,Ly]x[0,Lz] on nx*ny*nz nodes (a tensor
    grid: uniform, or the sorted per-axis coordinates in axes).

    robin_faces: names from FACES on which the unit Robin mass is assembled.
    The stored pattern is the full structural 27-point pattern (explicit zeros
    kept: on cubic cells the face-neighbour stiffness entries vanish).
    """
    Lx, Ly, Lz = L
    nx, ny, nz = nodes
    axes = axes or (None, None, None)
    one = [_one_d(nx, Lx, axes[0]), _one_d(ny, Ly, axes[1]), _one_d(nz, Lz, axes[2])]
    n = nx * ny * nz

    tri = [sp.diags([np.ones(m - 1), np.ones(m), np.ones(m - 1)], [-1, 0, 1]) for m in (nx, ny, nz)]
    # CSR throughout: scipy's default block (BSR) path for small factors would
    # store explicit zeros beyond the 27-point pattern
    P = sp.kron(tri[2], sp.kron(tri[1], tri[0], format="csr"), format="csr")
    P.sort_indices()
    rowptr = P.indptr.astype(np.int64)
    col = P.indices.astype(np.int32)
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(rowptr))
    cols = col.astype(np.int64)

    def split(idx):
        ix = idx % nx
        r = idx // nx
        return ix, r % ny, r // ny

    ri = split(rows)
    ci = split(cols)
    Kd = [o[0] for o in one]
    Md = [o[1] for o in one]
    kx = Kd[0][ri[0], ci[0]]
    ky = Kd[1][ri[1], ci[1]]
    kz = Kd[2][ri[2], ci[2]]
    mx = Md[0][ri[0], ci[0]]
    my = Md[1][ri[1], ci[1]]
    mz = Md[2][ri[2], ci[2]]
    Kv = k * (kx * my * mz + mx * ky * mz + mx * my * kz)
    del kx, ky, kz

    Rv = np.zeros_like(Kv)
    mfac = (mx, my, mz)
    for name in robin_faces:
        axis, side = FACES[name]
        last = (nx, ny, nz)[axis] - 1
        target = 0 if side == 0 else last
        sel = (ri[axis] == target) & (ci[axis] == target)
        f = np.ones_like(Kv)
        for d in range(3):
            if d != axis:
                f = f * mfac[d]
        Rv += np.where(sel, f, 0.0)
    del mx, my, mz

    ml = [o[2] for o in one]
    idx = np.arange(n)
    ix, iy, iz = split(idx)
    mass = rho_c * ml[0][ix] * ml[1][iy] * ml[2][iz]
    Rm = sp.csr_matrix((Rv, col, rowptr), shape=(n, n))
    rload = np.asarray(Rm @ np.ones(n)).ravel()
    xs = [o[3] for o in one]
    coords = np.stack([xs[0][ix], xs[1][iy], xs[2][iz]], axis=1)

    faces = {}
    for name, (axis, side) in FACES.items():
        other = [d for d in range(3) if d != axis]
        dims = (nx, ny, nz)
        fixed = 0 if side == 0 else dims[axis] - 1
        nu, nv = dims[other[0]], dims[other[1]]
        a = np.arange(nu)[:, None]
        b = np.arange(nv)[None, :]
        ijk = [None, None, None]
        ijk[axis] = np.full((nu, nv), fixed)
        ijk[other[0]] = np.broadcast_to(a, (nu, nv))
        ijk[other[1]] = np.broadcast_to(b, (nu, nv))
        ids = (ijk[0] + nx * (ijk[1] + ny * ijk[2])).astype(np.int32).ravel()
        faces[name] = Face(u=xs[other[0]].copy(), v=xs[other[1]].copy(), ids=ids)

    return Body(n=n, rowptr=rowptr, col=col, K=Kv, R=Rv, mass=mass, rload=rload,
                coords=coords, faces=faces, dims=(nx, ny, nz), lengths=(Lx, Ly, Lz))


def permute(b: Body, perm) -> Body:
    """The same body with its nodes renumbered: new node i is old node perm[i]
    (a caller's own numbering; the operators are the same up to that
    relabelling).  Rows keep their columns sorted."""
    perm = np.asarray(perm, dtype=np.int64)
    n = b.n
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)
    A = sp.csr_matrix((np.arange(b.nnz, dtype=np.float64) + 1.0, b.col, b.rowptr), shape=(n, n))
    Ap = A[perm][:, perm].tocsr()
    Ap.sort_indices()
    src = Ap.data.astype(np.int64) - 1  # old entry index of each new entry
    faces = {name: Face(u=f.u.copy(), v=f.v.copy(), ids=inv[f.ids].astype(np.int32))
             for name, f in b.faces.items()}
    return Body(n=n, rowptr=Ap.indptr.astype(np.int64), col=Ap.indices.astype(np.int32),
                K=b.K[src].copy(), R=b.R[src].copy(), mass=b.mass[perm].copy(),
                rload=b.rload[perm].copy(), coords=b.coords[perm].copy(), faces=faces,
                dims=(), lengths=b.lengths)
