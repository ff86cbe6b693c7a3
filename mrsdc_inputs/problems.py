"""Seeded synthetic workloads: box machines, couplings, motion and schemes.

Input generation only.  A Problem is a plain bundle of arrays and numbers
that both the GPU library and the CPU oracle receive; the time stepping, the
coupling integrals and the linear solves are implemented independently on
each side.

Geometry readings (the paper's own machine model is not available, boxes
stand in for it):
  * single box with a moving rectangular heat-flux patch on one face;
  * stand box + stock box: the stock's x0 face slides along the stand's x1
    face (the rail, paper §2 Fig. 1 red surface) in z; its position is
    v_offset(t) = s0 + a sin(2 pi t / period + phase) (paper §5, motion law).
  * Robin exchange on every face except the rail face of the stand and the
    contact face of the stock, which are insulated where not in contact
    (paper §2, the boundary conditions on the rail).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

from .mesh import FACES, Body, Face, box, jittered_nodes, permute

K_STEEL = 15.0  # W/(m K)
RHO_C_STEEL = 3.6e6  # J/(m^3 K)

LOBATTO = 0
EQUI_NOLEFT = 1
FP64 = 0
FP32_REFINE = 1
MULTIRATE = 0  # the method of section 3
SINGLE_RATE = 1  # single-rate SDC with the coupling implicit (section 5 comparison)


@dataclass
class Motion:
    s0: float = 0.0
    a: float = 0.0
    period: float = 1.0
    phase: float = 0.0

    def s(self, t: float) -> float:
        return self.s0 + self.a * math.sin(2.0 * math.pi * t / self.period + self.phase)


@dataclass
class Contact:
    """Stand/stock coupling on the overlap of two faces (paper §2, Gamma_R(t)).

    The moving face's coordinates are given in the fixed face's (u, v) frame at
    zero offset; at time t its v coordinates are shifted by motion.s(t).
    """

    fix_body: int
    fix_face: str
    mov_body: int
    mov_face: str
    mov_u: np.ndarray
    mov_v: np.ndarray
    alpha: float
    friction_W: float
    split: float = 0.5


@dataclass
class Patch:
    """Rigid rectangle sliding over one face: flux q0 + alpha (T_fixed - T).

    Centre (u_center, motion.s(t)); sides width_u x width_v.
    """

    body: int
    face: str
    width_u: float
    width_v: float
    u_center: float
    q0: float
    alpha: float = 0.0
    T_fixed: float = 0.0


@dataclass
class Scheme:
    M: int = 3
    family: int = LOBATTO
    P: int = 10
    K: int = 3
    dt: float = 1.0
    pcg_rtol: float = 1e-13
    pcg_maxit: int = 500
    precision: int = FP64
    refine_rtol: float = 1e-10
    refine_maxit: int = 20
    inner_rtol: float = 1e-6
    sweep_tol: float = 0.0  # > 0: residual-controlled number of sweeps (at most K)
    method: int = MULTIRATE


@dataclass
class Problem:
    name: str
    bodies: list
    h: list  # Robin coefficient per body
    T_amb: list  # ambient temperature per body
    coupling: object  # Contact | Patch | None
    motion: Motion
    scheme: Scheme
    T0: np.ndarray  # concatenated [body0, body1]
    nsteps: int
    t0: float = 0.0
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(sum(b.n for b in self.bodies))

    @property
    def nnz(self) -> int:
        return int(sum(b.nnz for b in self.bodies))

    @property
    def offsets(self):
        off = [0]
        for b in self.bodies:
            off.append(off[-1] + b.n)
        return off

    def with_scheme(self, **kw) -> "Problem":
        return replace(self, scheme=replace(self.scheme, **kw))


def noise_T0(n: int, seed: int, base: float = 20.0, amp: float = 0.5) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return base + rng.uniform(-amp, amp, size=n)


def _robin_except(*skip):
    return tuple(f for f in FACES if f not in skip)


def patch_box(L=(0.2, 0.2, 0.8), nodes=(9, 9, 33), h=10.0, T_amb=20.0, q0=2000.0,
              width=0.05, u_center=0.1, motion=Motion(0.4, 0.3, 2.0, 0.0), alpha=0.0,
              T_fixed=0.0, robin=True, scheme=None, nsteps=60, seed=0, name="patch_box") -> Problem:
    """Single box with a rigid moving patch on face x1 (Robin everywhere if robin)."""
    faces = tuple(FACES) if robin else ()
    b = box(L, nodes, K_STEEL, RHO_C_STEEL, faces)
    sc = scheme or Scheme(M=3, family=LOBATTO, P=10, K=3, dt=1.0)
    cpl = Patch(body=0, face="x1", width_u=width, width_v=width, u_center=u_center, q0=q0,
                alpha=alpha, T_fixed=T_fixed)
    return Problem(name=name, bodies=[b], h=[h], T_amb=[T_amb], coupling=cpl, motion=motion,
                   scheme=sc, T0=noise_T0(b.n, seed), nsteps=nsteps)


def machine(stand_nodes=(41, 41, 161), stock_nodes=(31, 31, 41), stand_L=(0.4, 0.4, 1.6),
            stock_L=(0.3, 0.3, 0.4), y_offset=0.05, h=10.0, T_amb=20.0, alpha=1000.0,
            friction_W=200.0, period=4.0, stroke=1.0, scheme=None, nsteps=120, seed=0,
            robin=True, jitter=0.0, mesh_seed=7, renumber=False,
            name="machine") -> Problem:
    """Stand + sliding stock.  Stock centre z_c(t) = Lz_stand/2 + stroke/2 sin(2 pi t/period).

    jitter > 0: irregular tensor meshes, every interior node coordinate moved
    by U[-jitter, jitter] grid spacings (default_rng(mesh_seed)), so the
    operators hold a different value in nearly every entry.  renumber: each
    body's nodes in a seeded random order (default_rng(mesh_seed + 1)), as
    an unstructured mesh generator may number them."""
    stand_faces = _robin_except("x1") if robin else ()
    stock_faces = _robin_except("x0") if robin else ()
    mrng = np.random.default_rng(mesh_seed)
    axes = [None, None]
    if jitter > 0:
        axes = [tuple(jittered_nodes(n, L, mrng, jitter) for n, L in zip(nodes, Ls))
                for nodes, Ls in ((stand_nodes, stand_L), (stock_nodes, stock_L))]
    stand = box(stand_L, stand_nodes, K_STEEL, RHO_C_STEEL, stand_faces, axes=axes[0])
    stock = box(stock_L, stock_nodes, K_STEEL, RHO_C_STEEL, stock_faces, axes=axes[1])
    if renumber:
        prng = np.random.default_rng(mesh_seed + 1)
        stand = permute(stand, prng.permutation(stand.n))
        stock = permute(stock, prng.permutation(stock.n))
    f = stock.faces["x0"]
    cpl = Contact(fix_body=0, fix_face="x1", mov_body=1, mov_face="x0",
                  mov_u=f.u + y_offset, mov_v=f.v.copy(), alpha=alpha, friction_W=friction_W)
    s0 = stand_L[2] / 2.0 - stock_L[2] / 2.0
    motion = Motion(s0=s0, a=stroke / 2.0, period=period, phase=0.0)
    # "20 fast substeps" per 5 s step over the 4 non-degenerate Lobatto
    # intervals: P = 5 embedded nodes per interval.  (P = 20 per interval makes
    # the equidistant no-left embedded quadrature diverge under the sweeps.)
    sc = scheme or Scheme(M=5, family=LOBATTO, P=5, K=4, dt=5.0)
    T0 = noise_T0(stand.n + stock.n, seed)
    return Problem(name=name, bodies=[stand, stock], h=[h, h], T_amb=[T_amb, T_amb],
                   coupling=cpl, motion=motion, scheme=sc, T0=T0, nsteps=nsteps)


# ---------------------------------------------------------------------------
# The workloads.  Mesh counts: the single box counts elements (8x8x32 ->
# 9x9x33 nodes); the machine meshes count nodes.
# ---------------------------------------------------------------------------

def box_patch_2673() -> Problem:
    """FP64 single steel box, 2,673 nodes, moving 2 kW/m^2 patch, 60 s horizon."""
    return patch_box(name="box-patch-2673")


def machine_310k(nsteps=120) -> Problem:
    """FP64 two-body machine, stand 41x41x161 + stock 31x31x41 (310,042 nodes)."""
    return machine(nsteps=nsteps, name="machine-310k")


def machine_310k_irregular(nsteps=120, renumber=False) -> Problem:
    """The 310,042-node machine on irregular tensor meshes (interior node
    coordinates moved by up to 0.2 grid spacings); with renumber, every
    body's nodes in a seeded random order."""
    return machine(nsteps=nsteps, jitter=0.2, renumber=renumber,
                   name="machine-310k-irregular" + ("-renumbered" if renumber else ""))


def machine_310k_fp32(nsteps=120) -> Problem:
    """The two-body machine with the FP32 inner solves + FP64 refinement."""
    p = machine(nsteps=nsteps, name="machine-310k-fp32refine")
    p.scheme.precision = FP32_REFINE
    return p


def scenario_params(s: int):
    """Per-scenario draws of the batched ensemble: (h, alpha, P_f, period, T0-seed rng)."""
    rng = np.random.default_rng(1000 + s)
    h = rng.uniform(5.0, 25.0)
    alpha = rng.uniform(500.0, 2000.0)
    pf = rng.uniform(50.0, 400.0)
    period = rng.uniform(2.0, 8.0)
    return h, alpha, pf, period, rng


def ensemble_member(s: int, stand_nodes=(54, 54, 214), stock_nodes=(41, 41, 54), nsteps=120,
                    precision=FP32_REFINE) -> Problem:
    """Scenario s of the 64-member ensemble on the 7.5 mm machine mesh."""
    h, alpha, pf, period, rng = scenario_params(s)
    p = machine(stand_nodes=stand_nodes, stock_nodes=stock_nodes, h=h, alpha=alpha,
                friction_W=pf, period=period, nsteps=nsteps, name=f"ensemble-7.5mm-s{s}")
    p.T0 = 20.0 + rng.uniform(-0.5, 0.5, size=p.N)
    p.scheme.precision = precision
    p.meta = dict(scenario=s, h=h, alpha=alpha, friction_W=pf, period=period)
    return p


MESH_LEVELS = {
    "2cm": ((21, 21, 81), (16, 16, 21)),
    "1cm": ((41, 41, 161), (31, 31, 41)),
    "5mm": ((81, 81, 321), (61, 61, 81)),
}


def serving_trace(n_requests=64, rate=20.0, seed=4, dt=5.0):
    """Poisson arrivals; each request: mesh level, horizon, scenario parameters."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    levels = list(MESH_LEVELS)
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        level = levels[int(rng.integers(0, len(levels)))]
        horizon = float(rng.uniform(60.0, 1800.0))
        nsteps = max(1, int(round(horizon / dt)))
        r = np.random.default_rng(10000 + i)
        reqs.append(dict(id=i, arrival=t, level=level, nsteps=nsteps,
                         h=r.uniform(5.0, 25.0), alpha=r.uniform(500.0, 2000.0),
                         friction_W=r.uniform(50.0, 400.0), period=r.uniform(2.0, 8.0),
                         seed=10000 + i))
    return reqs
