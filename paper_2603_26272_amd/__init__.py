"""WENO-ZA6 (arXiv 2603.26272) on AMD MI355X.

The numerical work runs in libza (HIP kernels for gfx950) behind the C ABI
of include/za.h; ``za`` is its ctypes binding, ``Problem`` the problem
description and ``workloads`` the seeded initial-data generators.
"""
from .problem import (ADVECTION, BUCKLEY, BURGERS, DT_CFL, DT_CFL_H2, EULER, FP32_RECON, FP64,
                      LF_PER_FIELD, LF_SCALAR, PERIODIC, TRANSMISSIVE, Problem)

__all__ = ["Problem", "ADVECTION", "EULER", "BURGERS", "BUCKLEY", "PERIODIC", "TRANSMISSIVE",
           "FP64", "FP32_RECON", "DT_CFL", "DT_CFL_H2", "LF_PER_FIELD", "LF_SCALAR"]
