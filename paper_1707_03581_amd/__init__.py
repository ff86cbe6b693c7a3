"""MI355X MRSDC heat-conduction stepper: Python binding of the C-ABI (mrsdc.h).

Argument marshalling only: every step of the time stepper runs in the HIP
kernels of libmrsdc.so.  Importing this package fails loudly when the library
has not been built (python -m paper_1707_03581_amd.build).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmrsdc.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, ESTATE = 0, -1, -2, -3, -4, -5
FP64, FP32_REFINE = 0, 1
LOBATTO, EQUI_NOLEFT = 0, 1
MULTIRATE, SINGLE_RATE = 0, 1
OP_AUTO, OP_VALUES, OP_DICT, OP_PACKED, OP_PATTERNS, OP_COL32 = 0, 1, 2, 3, 4, 0x100
FACE_TAGS = {"x0": 0, "x1": 1, "y0": 2, "y1": 3, "z0": 4, "z1": 5}
_NAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ENOCONV: "ENOCONV",
          ESTATE: "ESTATE"}


class MrsdcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_NAMES.get(status, status)}: {msg}")
        self.status = status


class Config(C.Structure):
    _fields_ = [("device", C.c_int), ("precision", C.c_int), ("M", C.c_int),
                ("node_family", C.c_int), ("P", C.c_int), ("K", C.c_int), ("dt", C.c_double),
                ("pcg_rtol", C.c_double), ("pcg_maxit", C.c_int), ("refine_rtol", C.c_double),
                ("refine_maxit", C.c_int), ("inner_rtol", C.c_double),
                ("final_residual", C.c_int), ("use_graph", C.c_int), ("sweep_tol", C.c_double),
                ("method", C.c_int), ("stream", C.c_void_p), ("op_form", C.c_int),
                ("alloc", C.c_void_p), ("autotune", C.c_int)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("release", RELEASE_FN), ("user", C.c_void_p)]


def torch_allocator(device=0):
    """An mrsdc_allocator over torch's caching allocator: the library's device
    buffers are then torch's (counted by torch.cuda.memory_allocated).  Keep
    the returned object alive as long as any context created with it."""
    import torch

    def _alloc(nbytes, stream, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream or 0)
        except RuntimeError:
            return None

    def _release(ptr, stream, user):
        torch.cuda.caching_allocator_delete(ptr)

    a = Allocator(ALLOC_FN(_alloc), RELEASE_FN(_release), None)
    a._keep = (_alloc, _release)
    return a


class Stats(C.Structure):
    _fields_ = [("steps", C.c_int64), ("solves", C.c_int64), ("pcg_iters", C.c_int64),
                ("refine_steps", C.c_int64), ("max_iters", C.c_int32),
                ("redone_steps", C.c_int32), ("residual", C.c_double * 17),
                ("wall_s", C.c_double), ("bytes_moved", C.c_int64), ("sweeps", C.c_int64),
                ("op_form", C.c_int32), ("col_bytes", C.c_int32),
                ("graph_captures", C.c_int32), ("graph_launches", C.c_int32),
                ("col_depth", C.c_int32), ("groups_b", C.c_int32), ("groups_c", C.c_int32),
                ("autotuned", C.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "residual"}
        d["residual"] = list(self.residual)
        return d


class KernelTimes(C.Structure):
    _fields_ = [("cg_spmv_launches", C.c_int64), ("cg_spmv_ms", C.c_double),
                ("cg_spmv_bytes", C.c_int64), ("iface_launches", C.c_int64),
                ("iface_ms", C.c_double), ("nnz", C.c_int64), ("n", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None

_SIGS = {
    "mrsdc_config_init": (None, [C.c_void_p]),
    "mrsdc_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_void_p]),
    "mrsdc_set_body": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                                 C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "mrsdc_set_robin": (C.c_int, [C.c_void_p, C.c_int, C.c_double, C.c_double]),
    "mrsdc_set_face": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p,
                                 C.c_void_p, C.c_void_p]),
    "mrsdc_set_motion": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double]),
    "mrsdc_set_contact": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double,
                                    C.c_double, C.c_double, C.c_double, C.c_double]),
    "mrsdc_set_patch": (C.c_int, [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_double,
                                  C.c_double, C.c_double, C.c_double, C.c_double]),
    "mrsdc_set_temperature": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int64]),
    "mrsdc_set_time": (C.c_int, [C.c_void_p, C.c_double]),
    "mrsdc_set_stationary": (C.c_int, [C.c_void_p, C.c_double, C.c_int, C.POINTER(C.c_int)]),
    "mrsdc_set_stationary_noalloc": (C.c_int, [C.c_void_p, C.c_double, C.c_int,
                                               C.POINTER(C.c_int)]),
    "mrsdc_get_time": (C.c_int, [C.c_void_p, C.POINTER(C.c_double)]),
    "mrsdc_advance": (C.c_int, [C.c_void_p, C.c_double, C.c_void_p]),
    "mrsdc_get_temperature": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int64]),
    "mrsdc_get_temperature_device": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int64,
                                               C.c_void_p]),
    "mrsdc_footprint_bytes": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    "mrsdc_batch_slot_bytes": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64),
                                         C.POINTER(C.c_int64)]),
    "mrsdc_last_error": (C.c_char_p, [C.c_void_p]),
    "mrsdc_destroy": (C.c_int, [C.c_void_p]),
    "mrsdc_quadrature": (C.c_int, [C.c_int, C.c_int, C.c_int, C.c_double, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p]),
    "mrsdc_version": (C.c_char_p, []),
    "mrsdc_profile": (C.c_int, [C.c_void_p, C.c_int]),
    "mrsdc_batch_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_void_p, C.c_int]),
    "mrsdc_batch_set_scenario": (C.c_int, [C.c_void_p, C.c_int, C.c_double, C.c_double,
                                           C.c_double, C.c_double]),
    "mrsdc_batch_set_temperature": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int64]),
    "mrsdc_batch_set_time": (C.c_int, [C.c_void_p, C.c_int, C.c_double]),
    "mrsdc_batch_get_time": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double)]),
    "mrsdc_batch_set_active": (C.c_int, [C.c_void_p, C.c_int, C.c_int]),
    "mrsdc_batch_advance": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p]),
    "mrsdc_batch_get_temperature": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int64]),
    "mrsdc_batch_get_temperature_device": (C.c_int, [C.c_void_p, C.c_int, C.c_void_p, C.c_int64,
                                                     C.c_void_p]),
    "mrsdc_batch_advance_horizons": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "mrsdc_profile_read": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mrsdc_time_operator": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double),
                                      C.POINTER(C.c_int64)]),
    "mrsdc_deform_setup": (C.c_int, [C.c_void_p, C.c_int, C.c_int64, C.c_int64, C.c_void_p,
                                     C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_double]),
    "mrsdc_deform": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64]),
    "mrsdc_deform_device": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]),
    "mrsdc_deform_get_info": (C.c_int, [C.c_void_p, C.c_void_p]),
    "mrsdc_deform_time": (C.c_int, [C.c_void_p, C.c_int, C.POINTER(C.c_double),
                                    C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
}


class DeformInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("block", C.c_int64), ("padded_block", C.c_int64),
                ("nblocks", C.c_int64), ("factor_bytes", C.c_int64), ("factor_ms", C.c_double),
                ("factor_launches", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def lib():
    """The loaded libmrsdc.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        # torch brings its own HIP runtime (same soname as the system one);
        # loading torch first makes libmrsdc.so bind to that single copy
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1707_03581_amd.build` (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def quadrature(M, family, P, dt=1.0):
    """(tau, s, shat, stil, spq) as computed by the library (host only)."""
    tau = np.zeros(M + 1)
    s = np.zeros((M + 1, M + 1))
    shat = np.zeros((M + 1, P + 1))
    stil = np.zeros((M + 1, P + 1, M + 1))
    spq = np.zeros((M + 1, P + 1, P + 1))
    rc = lib().mrsdc_quadrature(M, family, P, dt, _p(tau), _p(s), _p(shat), _p(stil), _p(spq))
    if rc:
        raise MrsdcError(rc, "bad quadrature arguments")
    return tau, s, shat, stil, spq


def default_config(**kw) -> Config:
    cfg = Config()
    lib().mrsdc_config_init(C.byref(cfg))
    for k, v in kw.items():
        if k == "alloc" and isinstance(v, Allocator):
            cfg._allocator = v  # the config (and the caller) keep it alive
            v = C.cast(C.pointer(v), C.c_void_p).value
        setattr(cfg, k, v)
    return cfg


class Context:
    """One simulation on one GPU; methods mirror the C entry points."""

    def __init__(self, cfg: Config):
        self._L = lib()
        self._h = C.c_void_p()
        self.cfg = cfg
        rc = self._L.mrsdc_create(C.byref(self._h), C.byref(cfg))
        if rc:
            raise MrsdcError(rc, "mrsdc_create failed (scheme or device)")

    def _chk(self, rc):
        if rc:
            raise MrsdcError(rc, self._L.mrsdc_last_error(self._h).decode())
        return rc

    def set_body(self, body, rowptr, col, K, R, mass, robin_load):
        rowptr = np.ascontiguousarray(rowptr, np.int64)
        col = np.ascontiguousarray(col, np.int32)
        K = np.ascontiguousarray(K, np.float64)
        mass = np.ascontiguousarray(mass, np.float64)
        R = None if R is None else np.ascontiguousarray(R, np.float64)
        rl = None if robin_load is None else np.ascontiguousarray(robin_load, np.float64)
        n = len(mass)
        return self._chk(self._L.mrsdc_set_body(self._h, body, n, int(rowptr[-1]), _p(rowptr),
                                                _p(col), _p(K), None if R is None else _p(R),
                                                _p(mass), None if rl is None else _p(rl)))

    def set_robin(self, body, h, T_env):
        return self._chk(self._L.mrsdc_set_robin(self._h, body, h, T_env))

    def set_face(self, body, face, u, v, node_ids):
        u = np.ascontiguousarray(u, np.float64)
        v = np.ascontiguousarray(v, np.float64)
        ids = np.ascontiguousarray(node_ids, np.int32)
        return self._chk(self._L.mrsdc_set_face(self._h, body, face, len(u), len(v), _p(u), _p(v),
                                                _p(ids)))

    def set_motion(self, s0, a, period, phase=0.0):
        return self._chk(self._L.mrsdc_set_motion(self._h, s0, a, period, phase))

    def set_contact(self, fix_body, fix_face, mov_body, mov_face, du, dv, alpha, friction_W,
                    split=0.5):
        return self._chk(self._L.mrsdc_set_contact(self._h, fix_body, fix_face, mov_body, mov_face,
                                                   du, dv, alpha, friction_W, split))

    def set_patch(self, body, face, width_u, width_v, u_center, q0, alpha=0.0, T_fixed=0.0):
        return self._chk(self._L.mrsdc_set_patch(self._h, body, face, width_u, width_v, u_center,
                                                 q0, alpha, T_fixed))

    def set_temperature(self, body, T):
        T = np.ascontiguousarray(T, np.float64)
        return self._chk(self._L.mrsdc_set_temperature(self._h, body, _p(T), len(T)))

    def set_time(self, t):
        return self._chk(self._L.mrsdc_set_time(self._h, t))

    def set_stationary(self, rtol=1e-13, maxit=100000):
        """Replace the field by the stationary one, (K + h R) T = g; returns
        the CG iteration count."""
        it = C.c_int(0)
        self._chk(self._L.mrsdc_set_stationary(self._h, rtol, maxit, C.byref(it)))
        return it.value

    def set_stationary_noalloc(self, rtol=1e-13, maxit=100000):
        """set_stationary without any device allocation (fixed library
        scratch; the context's device state must exist)."""
        it = C.c_int(0)
        self._chk(self._L.mrsdc_set_stationary_noalloc(self._h, rtol, maxit, C.byref(it)))
        return it.value

    def get_time(self):
        t = C.c_double()
        self._chk(self._L.mrsdc_get_time(self._h, C.byref(t)))
        return t.value

    def advance(self, horizon):
        st = Stats()
        self._chk(self._L.mrsdc_advance(self._h, horizon, C.byref(st)))
        return st.as_dict()

    def get_temperature(self, body, n):
        out = np.empty(n)
        self._chk(self._L.mrsdc_get_temperature(self._h, body, _p(out), n))
        return out

    def get_temperature_device(self, body, tensor, stream=None):
        """Copy into a contiguous float64 device tensor (torch) on `stream`."""
        ptr = tensor.data_ptr()
        s = None if stream is None else C.c_void_p(stream)
        return self._chk(self._L.mrsdc_get_temperature_device(self._h, body, C.c_void_p(ptr),
                                                              tensor.numel(), s))

    def footprint_bytes(self):
        b = C.c_int64()
        self._chk(self._L.mrsdc_footprint_bytes(self._h, C.byref(b)))
        return b.value

    def profile(self, on=True):
        return self._chk(self._L.mrsdc_profile(self._h, 1 if on else 0))

    def profile_read(self):
        kt = KernelTimes()
        self._chk(self._L.mrsdc_profile_read(self._h, C.byref(kt)))
        return kt.as_dict()

    def deform_setup(self, el, body=0):
        """Register and factorise the thermo-elastic problem of a body (an
        object with n, rowptr, col, K, g_rowptr, g_col, G, T_ref)."""
        rp = np.ascontiguousarray(el.rowptr, dtype=np.int64)
        col = np.ascontiguousarray(el.col, dtype=np.int32)
        K = np.ascontiguousarray(el.K, dtype=np.float64)
        grp = np.ascontiguousarray(el.g_rowptr, dtype=np.int64)
        gcol = np.ascontiguousarray(el.g_col, dtype=np.int32)
        G = np.ascontiguousarray(el.G, dtype=np.float64)
        self._chk(self._L.mrsdc_deform_setup(self._h, body, int(el.n), int(rp[-1]), _p(rp), _p(col),
                                             _p(K), int(grp[-1]), _p(grp), _p(gcol), _p(G),
                                             float(el.T_ref)))
        self._df_n = int(el.n)
        return self.deform_info()

    def deform(self):
        """Displacement of the registered body for the current temperature."""
        out = np.empty(self._df_n)
        self._chk(self._L.mrsdc_deform(self._h, _p(out), self._df_n))
        return out

    def deform_info(self):
        info = DeformInfo()
        self._chk(self._L.mrsdc_deform_get_info(self._h, C.byref(info)))
        return info.as_dict()

    def deform_time(self, reps=5):
        """(microseconds per solve, microseconds per symmetric block product,
        algorithmic bytes per block product)."""
        a, b, n = C.c_double(), C.c_double(), C.c_int64()
        self._chk(self._L.mrsdc_deform_time(self._h, reps, C.byref(a), C.byref(b), C.byref(n)))
        return a.value, b.value, n.value

    def time_operator(self, reps=200):
        """(average microseconds per launch, algorithmic bytes per launch)."""
        us = C.c_double()
        by = C.c_int64()
        self._chk(self._L.mrsdc_time_operator(self._h, reps, C.byref(us), C.byref(by)))
        return us.value, by.value

    def last_error(self):
        return self._L.mrsdc_last_error(self._h).decode()

    def destroy(self):
        if self._h:
            self._L.mrsdc_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class BatchContext(Context):
    """S scenarios of one machine on one GPU (shared operators, per-scenario
    h, alpha, friction power, motion period, time and temperature)."""

    def __init__(self, cfg: Config, S: int):
        self._L = lib()
        self._h = C.c_void_p()
        self.cfg = cfg
        self.S = S
        rc = self._L.mrsdc_batch_create(C.byref(self._h), C.byref(cfg), S)
        if rc:
            raise MrsdcError(rc, "mrsdc_batch_create failed (scheme, S or device)")

    def set_scenario(self, s, h, alpha, friction_W, period):
        return self._chk(self._L.mrsdc_batch_set_scenario(self._h, s, h, alpha, friction_W, period))

    def set_scenario_temperature(self, s, T):
        T = np.ascontiguousarray(T, np.float64)
        return self._chk(self._L.mrsdc_batch_set_temperature(self._h, s, _p(T), len(T)))

    def set_scenario_time(self, s, t):
        return self._chk(self._L.mrsdc_batch_set_time(self._h, s, t))

    def get_scenario_time(self, s):
        t = C.c_double()
        self._chk(self._L.mrsdc_batch_get_time(self._h, s, C.byref(t)))
        return t.value

    def set_active(self, s, active=True):
        return self._chk(self._L.mrsdc_batch_set_active(self._h, s, 1 if active else 0))

    def advance_steps(self, nsteps):
        st = Stats()
        self._chk(self._L.mrsdc_batch_advance(self._h, nsteps, C.byref(st)))
        return st.as_dict()

    def slot_bytes(self):
        """(device bytes per scenario slot, shared device bytes) of the
        prepared context."""
        a, b = C.c_int64(), C.c_int64()
        self._chk(self._L.mrsdc_batch_slot_bytes(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def advance_horizons(self, horizons):
        """Advance each scenario by its own horizon (seconds; one per scenario)."""
        h = np.ascontiguousarray(horizons, np.float64)
        if len(h) != self.S:
            raise ValueError("one horizon per scenario")
        st = Stats()
        self._chk(self._L.mrsdc_batch_advance_horizons(self._h, _p(h), C.byref(st)))
        return st.as_dict()

    def get_scenario_temperature_device(self, s, tensor, stream=None):
        """Copy scenario s's field into a contiguous float64 device tensor."""
        st = None if stream is None else C.c_void_p(stream)
        return self._chk(self._L.mrsdc_batch_get_temperature_device(
            self._h, s, C.c_void_p(tensor.data_ptr()), tensor.numel(), st))

    def get_scenario_temperature(self, s, n):
        out = np.empty(n)
        self._chk(self._L.mrsdc_batch_get_temperature(self._h, s, _p(out), n))
        return out


def config_from_scheme(scheme, device=0, **over) -> Config:
    """Config from an object with M, family, P, K, dt, pcg_rtol, pcg_maxit, precision..."""
    kw = dict(device=device, precision=scheme.precision, M=scheme.M, node_family=scheme.family,
              P=scheme.P, K=scheme.K, dt=scheme.dt, pcg_rtol=scheme.pcg_rtol,
              pcg_maxit=scheme.pcg_maxit, refine_rtol=scheme.refine_rtol,
              refine_maxit=scheme.refine_maxit, inner_rtol=scheme.inner_rtol,
              sweep_tol=getattr(scheme, "sweep_tol", 0.0),
              method=getattr(scheme, "method", MULTIRATE))
    kw.update(over)
    return default_config(**kw)


def load_problem(ctx: Context, pb, h=None, alpha=None, friction_W=None, period=None, T0=None,
                 temperature=True):
    """Pass a problem description (bodies, faces, coupling, motion, T0) to ctx."""
    for i, b in enumerate(pb.bodies):
        ctx.set_body(i, b.rowptr, b.col, b.K, b.R, b.mass, b.rload)
        ctx.set_robin(i, pb.h[i] if h is None else h, pb.T_amb[i])
    m = pb.motion
    ctx.set_motion(m.s0, m.a, m.period if period is None else period, m.phase)
    c = pb.coupling
    if c is not None and type(c).__name__ == "Contact":
        F = pb.bodies[c.fix_body].faces[c.fix_face]
        G = pb.bodies[c.mov_body].faces[c.mov_face]
        ctx.set_face(c.fix_body, FACE_TAGS[c.fix_face], F.u, F.v, F.ids)
        ctx.set_face(c.mov_body, FACE_TAGS[c.mov_face], c.mov_u, c.mov_v, G.ids)
        ctx.set_contact(c.fix_body, FACE_TAGS[c.fix_face], c.mov_body, FACE_TAGS[c.mov_face],
                        0.0, 0.0, c.alpha if alpha is None else alpha,
                        c.friction_W if friction_W is None else friction_W, c.split)
    elif c is not None:
        F = pb.bodies[c.body].faces[c.face]
        ctx.set_face(c.body, FACE_TAGS[c.face], F.u, F.v, F.ids)
        ctx.set_patch(c.body, FACE_TAGS[c.face], c.width_u, c.width_v, c.u_center, c.q0, c.alpha,
                      c.T_fixed)
    if not temperature:
        return
    T = pb.T0 if T0 is None else T0
    off = pb.offsets
    for i in range(len(pb.bodies)):
        ctx.set_temperature(i, T[off[i]:off[i + 1]])
    ctx.set_time(pb.t0)


def batch_simulation(pb, members, device=0, **cfg_over) -> BatchContext:
    """Batch over a shared machine pb; members: list of dicts with h, alpha,
    friction_W, period, T0 (and optionally t0)."""
    ctx = BatchContext(config_from_scheme(pb.scheme, device=device, **cfg_over), len(members))
    load_problem(ctx, pb, temperature=False)
    for s, mb in enumerate(members):
        ctx.set_scenario(s, mb["h"], mb["alpha"], mb["friction_W"], mb["period"])
        ctx.set_scenario_temperature(s, mb["T0"])
        ctx.set_scenario_time(s, mb.get("t0", 0.0))
    return ctx


def simulation(pb, device=0, **cfg_over) -> Context:
    """Context for a problem description, ready to advance."""
    ctx = Context(config_from_scheme(pb.scheme, device=device, **cfg_over))
    load_problem(ctx, pb)
    return ctx


def get_state(ctx: Context, pb):
    return np.concatenate([ctx.get_temperature(i, b.n) for i, b in enumerate(pb.bodies)])
