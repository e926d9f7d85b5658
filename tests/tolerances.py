"""Parity bounds of the 2D GPU path against the FP64 oracle (shared by the 2D and serving
tests).

FP64: relative L2 <= 1e-12 per level (the parity bar).  Reduced precision (FP32 or split-BF16
transforms with one FP64 residual refinement): a bound per level index, about 100 x the largest
error measured for that level over the small 2D cases, the 1024^2 workload and the served
requests (FP32: 4.2e-15, 7.4e-16, 7.0e-16, 5.1e-16 for levels 0-3; split BF16: 1.5e-11,
2.7e-12, 3.2e-14, 3.1e-15), with level 3 -- the top level of RIDC4, the result -- capped at
1.5e-13 = 0.1 x the RIDC4 discretisation error of the 1024^2 workload, the bar at which a
reduced-precision result counts as matched.
"""

TOL64 = 1e-12
# per level index j = 0, 1, 2, 3 (index 3 also bounds any higher level)
TOL = {"fp32": (5e-13, 1e-13, 1e-13, 5e-14), "bf16x3": (1.5e-9, 3e-10, 5e-12, 1.5e-13)}


def tol_of(prec: str, j: int) -> float:
    """Bound of level j in precision prec."""
    return TOL64 if prec == "fp64" else TOL[prec][min(j, 3)]
