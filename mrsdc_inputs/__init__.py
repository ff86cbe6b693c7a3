"""Seeded synthetic inputs shared by the GPU library's tests and the CPU oracle.

Holds meshes, assembled finite element operators, couplings, motion laws and
seeded initial fields: the arrays a caller passes to the time stepper.  It
contains none of the time-stepping method's arithmetic.
"""
from .mesh import FACES, Body, Face, box, jittered_nodes, permute  # noqa: F401
from .problems import (  # noqa: F401
    EQUI_NOLEFT, FP32_REFINE, FP64, LOBATTO, MESH_LEVELS, MULTIRATE, SINGLE_RATE, Contact, Motion,
    Patch, Problem,
    Scheme, box_patch_2673, machine_310k, machine_310k_fp32, machine_310k_irregular, ensemble_member, machine, noise_T0, patch_box,
    scenario_params, serving_trace,
)
