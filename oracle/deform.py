"""Oracle of the thermo-elastic deformation solve -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU leg use it; the
GPU library shares nothing with it.

The deformation of §5 is the solution of the linear elasticity system with
the temperature field as load: K_u u = G (T - T_ref) over the free
displacement DOFs.  That result has a plain definition, so the oracle is that
definition: one sparse direct solve (SuperLU through scipy) in FP64.  The
paper's "factorise once, forward/backward solve per output" is how the
library reaches the same u; here the factorisation is kept too, so several
temperature fields reuse it.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spl


class Deformation:
    """Factorised K_u of one body (an object with csr(), gcsr(), T_ref)."""

    def __init__(self, el):
        self.el = el
        self.lu = spl.splu(el.csr().tocsc())
        self.G = el.gcsr()

    def load(self, T):
        return self.G @ (np.asarray(T, dtype=np.float64) - self.el.T_ref)

    def __call__(self, T):
        return self.lu.solve(self.load(T))


def deform(el, T):
    """u = K_u^{-1} G (T - T_ref)."""
    return Deformation(el)(T)
