"""CPU FP64 oracle of the MRSDC time stepper (ctypes wrapper around plain C).

TEST INFRASTRUCTURE, NOT THE PRODUCT.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the GPU library; the only thing both receive is the same seeded Problem from
mrsdc_inputs.

See mrsdc_oracle.c for the passages of the paper each piece follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mrsdc_oracle.c")
LIB = os.path.join(HERE, "liborc.so")

NONE, CONTACT, PATCH = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C + OpenMP, libquadmath for weights)."""
    if force or not os.path.exists(LIB):
        tmp = LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-o", tmp, SRC,
               "-lquadmath", "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, LIB)
    return LIB


class _Body(C.Structure):
    _fields_ = [("n", C.c_int64), ("rowptr", C.c_void_p), ("col", C.c_void_p), ("K", C.c_void_p),
                ("R", C.c_void_p), ("mass", C.c_void_p), ("rload", C.c_void_p), ("h", C.c_double),
                ("Tamb", C.c_double)]


class _Face(C.Structure):
    _fields_ = [("body", C.c_int), ("nu", C.c_int), ("nv", C.c_int), ("u", C.c_void_p),
                ("v", C.c_void_p), ("ids", C.c_void_p)]


class _Coupling(C.Structure):
    _fields_ = [("kind", C.c_int), ("fix", _Face), ("mov", _Face), ("alpha", C.c_double),
                ("Pf", C.c_double), ("split", C.c_double), ("face", _Face), ("wu", C.c_double),
                ("wv", C.c_double), ("uc", C.c_double), ("q0", C.c_double), ("Tfix", C.c_double),
                ("s0", C.c_double), ("a", C.c_double), ("period", C.c_double),
                ("phase", C.c_double)]


class _Problem(C.Structure):
    _fields_ = [("nbody", C.c_int), ("body", _Body * 2), ("cpl", _Coupling)]


class _Scheme(C.Structure):
    _fields_ = [("M", C.c_int), ("family", C.c_int), ("P", C.c_int), ("K", C.c_int),
                ("dt", C.c_double), ("pcg_rtol", C.c_double), ("pcg_maxit", C.c_int), ("sweep_tol", C.c_double),
                ("method", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("solves", C.c_int64), ("pcg_iters", C.c_int64), ("fE_evals", C.c_int64),
                ("max_iters", C.c_int), ("t_pcg", C.c_double), ("t_embedded", C.c_double),
                ("t_total", C.c_double), ("threads", C.c_int), ("sweeps", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.orc_weights.argtypes = [C.c_int, C.c_int, C.c_int, C.c_double, P, P, P, P, P]
        L.orc_fE.argtypes = [P, C.c_double, P, P]
        L.orc_solve.argtypes = [P, C.c_double, P, P, C.c_double, C.c_int]
        L.orc_run.argtypes = [P, P, C.c_double, C.c_int, P, P, P]
        L.orc_stationary.argtypes = [P, P, C.c_double, C.c_int]
        L.orc_max_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class _Keep:
    """Holds the numpy arrays a ctypes struct points into."""

    def __init__(self):
        self.arrays = []

    def __call__(self, a, dtype):
        a = np.ascontiguousarray(a, dtype=dtype)
        self.arrays.append(a)
        return _ptr(a)


def _face(keep, body, face_obj=None, u=None, v=None):
    f = _Face()
    f.body = body
    u = face_obj.u if u is None else u
    v = face_obj.v if v is None else v
    f.nu, f.nv = len(u), len(v)
    f.u = keep(u, np.float64)
    f.v = keep(v, np.float64)
    f.ids = keep(face_obj.ids, np.int32)
    return f


def make_problem(pb, keep=None, h=None, alpha=None, friction_W=None, period=None):
    """Translate an mrsdc_inputs.Problem into the oracle's C struct."""
    keep = keep or _Keep()
    s = _Problem()
    s.nbody = len(pb.bodies)
    for i, b in enumerate(pb.bodies):
        cb = s.body[i]
        cb.n = b.n
        cb.rowptr = keep(b.rowptr, np.int64)
        cb.col = keep(b.col, np.int32)
        cb.K = keep(b.K, np.float64)
        cb.R = keep(b.R, np.float64)
        cb.mass = keep(b.mass, np.float64)
        cb.rload = keep(b.rload, np.float64)
        cb.h = pb.h[i] if h is None else h
        cb.Tamb = pb.T_amb[i]
    c = pb.coupling
    m = pb.motion
    s.cpl.s0, s.cpl.a, s.cpl.phase = m.s0, m.a, m.phase
    s.cpl.period = m.period if period is None else period
    if c is None:
        s.cpl.kind = NONE
        s.cpl.period = 1.0
    elif type(c).__name__ == "Contact":
        s.cpl.kind = CONTACT
        s.cpl.fix = _face(keep, c.fix_body, pb.bodies[c.fix_body].faces[c.fix_face])
        s.cpl.mov = _face(keep, c.mov_body, pb.bodies[c.mov_body].faces[c.mov_face],
                          u=c.mov_u, v=c.mov_v)
        s.cpl.alpha = c.alpha if alpha is None else alpha
        s.cpl.Pf = c.friction_W if friction_W is None else friction_W
        s.cpl.split = c.split
    else:
        s.cpl.kind = PATCH
        s.cpl.face = _face(keep, c.body, pb.bodies[c.body].faces[c.face])
        s.cpl.wu, s.cpl.wv, s.cpl.uc = c.width_u, c.width_v, c.u_center
        s.cpl.q0, s.cpl.alpha, s.cpl.Tfix = c.q0, c.alpha, c.T_fixed
    return s, keep


def _scheme(sc):
    s = _Scheme()
    s.M, s.family, s.P, s.K = sc.M, sc.family, sc.P, sc.K
    s.dt, s.pcg_rtol, s.pcg_maxit = sc.dt, sc.pcg_rtol, sc.pcg_maxit
    s.sweep_tol = getattr(sc, "sweep_tol", 0.0)
    s.method = getattr(sc, "method", 0)
    return s


def weights(M, family, P, dt=1.0):
    """(tau[0..M], s[M+1,M+1], shat[M+1,P+1], stil[M+1,P+1,M+1], spq[M+1,P+1,P+1])."""
    tau = np.zeros(M + 1)
    s = np.zeros((M + 1, M + 1))
    shat = np.zeros((M + 1, P + 1))
    stil = np.zeros((M + 1, P + 1, M + 1))
    spq = np.zeros((M + 1, P + 1, P + 1))
    rc = lib().orc_weights(M, family, P, dt, _ptr(tau), _ptr(s), _ptr(shat), _ptr(stil), _ptr(spq))
    if rc:
        raise ValueError("bad quadrature arguments")
    return tau, s, shat, stil, spq


def fE(pb, t, T, **over):
    s, keep = make_problem(pb, **over)
    out = np.zeros(pb.N)
    T = np.ascontiguousarray(T, dtype=np.float64)
    lib().orc_fE(C.byref(s), t, _ptr(T), _ptr(out))
    return out


def solve(pb, dtau, b, x0=None, rtol=1e-13, maxit=1000):
    s, keep = make_problem(pb)
    x = np.zeros(pb.N) if x0 is None else np.array(x0, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    it = lib().orc_solve(C.byref(s), dtau, _ptr(b), _ptr(x), rtol, maxit)
    if it < 0:
        raise RuntimeError("oracle PCG did not converge")
    return x, it


def stationary(pb, T0=None, rtol=1e-13, maxit=100000, **over):
    """Stationary field (K + h R) T = g of pb's conduction and Robin part
    (no mass term), warm-started from T0 (default zeros); returns (T, iters)."""
    s, keep = make_problem(pb, **over)
    T = np.zeros(pb.N) if T0 is None else np.array(T0, dtype=np.float64)
    it = lib().orc_stationary(C.byref(s), _ptr(T), rtol, maxit)
    if it < 0:
        raise RuntimeError("oracle stationary PCG did not converge")
    return T, it


def run(pb, nsteps=None, T0=None, t0=None, residuals=False, scheme=None, **over):
    """Advance pb.T0 (or T0) by nsteps steps; returns (T, stats[, residuals])."""
    s, keep = make_problem(pb, **over)
    sc = _scheme(scheme or pb.scheme)
    n = pb.nsteps if nsteps is None else nsteps
    T = np.array(pb.T0 if T0 is None else T0, dtype=np.float64)
    res = np.zeros(n * (sc.K + 1)) if residuals else None
    st = Stats()
    rc = lib().orc_run(C.byref(s), C.byref(sc), pb.t0 if t0 is None else t0, n, _ptr(T),
                       _ptr(res) if residuals else None, C.byref(st))
    if rc:
        raise RuntimeError(f"oracle run failed ({rc})")
    if residuals:
        return T, st.as_dict(), res.reshape(n, sc.K + 1)
    return T, st.as_dict()


def max_threads() -> int:
    return lib().orc_max_threads()


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's later calls."""
    lib().orc_set_threads(int(n))
