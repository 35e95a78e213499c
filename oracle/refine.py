"""Mixed precision: FP32-stored p(l)-CG inside FP64 iterative refinement
(test infrastructure only).

The inner solver is Alg. 1 with every vector it keeps (the bases Z^{(k)}, p and
the correction d) rounded to IEEE binary32 when stored; all arithmetic, the dot
products, G, T and the LU scalars stay in FP64 (values read from FP32 storage
are exact in FP64).  The outer loop is classical iterative refinement in FP64:

    r_k = b - A x_k  (FP64);  stop when ||r_k|| < tol ||r_0||
    solve A d = r_k with the inner solver from d = 0 to
        |zeta_t| < max(inner_tol ||r_k||, final_factor tol ||r_0||)
    (the last correction need not be more accurate than the outer goal; an inner
    breakdown ends that inner solve with its last iterate)
    x_{k+1} = x_k + d  (FP64)

The recursive residual of an FP32-stored solve drifts away from the true one
(Sec. 2.2, "Residual norm in p(l)-CG": |zeta| equals ||r|| only in exact
arithmetic), which is why the stopping test of the outer loop uses the
recomputed FP64 residual.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import plcg as _plcg


def round_fp32(v):
    """Store in binary32, read back exactly."""
    return v.astype(np.float32).astype(np.float64)


@dataclass
class RefineResult:
    x: np.ndarray
    outer: int
    inner_iters: int
    reason: str
    rnorm0: float
    true_relres: float
    inner: list = field(default_factory=list)


def refine(A, b, x0, l, sigma, tol, inner_tol, maxit, max_outer=50,
           final_factor=0.5) -> RefineResult:
    """FP64 iterative refinement around FP32-stored Alg. 1 (module docstring; the
    residual gap it repairs is the one of Sec. 2.2, 'Residual norm').
    final_factor None: every inner solve runs to inner_tol ||r_k||."""
    x = x0.copy()
    r = b - A(x)
    rnorm0 = math.sqrt(np.dot(r, r))
    total = 0
    outer = 0
    inner = []
    reason = "maxit"
    rn = rnorm0
    while True:
        if rn == 0 or rn < tol * rnorm0:
            reason = "converged"
            break
        if outer >= max_outer or total >= maxit:
            break
        abs_tol = inner_tol * rn
        if final_factor is not None:
            abs_tol = max(abs_tol, final_factor * tol * rnorm0)
        seg = _plcg.alg1(A, r, np.zeros_like(x), l, sigma, abs_tol, maxit - total,
                         store=round_fp32)
        inner.append((seg.t_done, seg.reason))
        total += seg.t_done
        x = x + seg.x
        outer += 1
        r = b - A(x)
        rn = math.sqrt(np.dot(r, r))
    return RefineResult(x=x, outer=outer, inner_iters=total, reason=reason, rnorm0=rnorm0,
                        true_relres=rn / rnorm0 if rnorm0 > 0 else 0.0, inner=inner)
