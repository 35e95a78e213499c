"""Classic Conjugate Gradients (test infrastructure only).

The Hestenes-Stiefel method the paper compares against (Sec. 1; Table 1 row
"CG": two global reductions and one SpMV per iteration).  Written as the
textbook recurrence, one statement per step:

    r_0 = b - A x_0,  p_0 = r_0
    alpha_k = (r_k, r_k) / (p_k, A p_k)
    x_{k+1} = x_k + alpha_k p_k,   r_{k+1} = r_k - alpha_k A p_k
    beta_k  = (r_{k+1}, r_{k+1}) / (r_k, r_k),   p_{k+1} = r_{k+1} + beta_k p_k

Iteration count = number of x updates.  Stopping test: ||r_k|| < tol ||r_0||
on the recursively updated residual.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


def _sqrt(a):
    if isinstance(a, (float, np.floating)):
        return math.sqrt(a)
    import mpmath
    return mpmath.sqrt(a)


@dataclass
class CGResult:
    x: np.ndarray
    iters: int
    reason: str                  # "converged" | "maxit" | "breakdown"
    rnorm0: float
    rec_relres: float
    true_relres: float
    spmvs: int
    iterates: list = field(default_factory=list)     # x_1, x_2, ... when recorded
    resnorms: list = field(default_factory=list)     # ||r_k||, k = 0..iters


def cg(A, b, x0, tol, maxit, record_iterates=False) -> CGResult:
    """Classic CG (Sec. 1; Table 1, row CG) from x0, at most maxit x updates, stopping
    when the recursive ||r_k|| < tol ||r_0||; the recurrence in the module docstring."""
    x = x0.copy()
    r = b - A(x)
    spmvs = 1
    rho = np.dot(r, r)
    rnorm0 = _sqrt(rho)
    resnorms = [rnorm0]
    iterates = []
    reason = "maxit"
    k = 0
    if rnorm0 == 0:
        reason = "converged"
    else:
        p = r.copy()
        while k < maxit:
            q = A(p)
            spmvs += 1
            pq = np.dot(p, q)
            if not (pq > 0):
                reason = "breakdown"
                break
            alpha = rho / pq
            x = x + alpha * p
            r = r - alpha * q
            rho_new = np.dot(r, r)
            k += 1
            resnorms.append(_sqrt(rho_new))
            if record_iterates:
                iterates.append(x.copy())
            if _sqrt(rho_new) < tol * rnorm0:
                reason = "converged"
                break
            beta = rho_new / rho
            p = r + beta * p
            rho = rho_new
    true_res = b - A(x)
    spmvs += 1
    denom = rnorm0 if rnorm0 != 0 else 1.0
    return CGResult(x=x, iters=k, reason=reason, rnorm0=rnorm0,
                    rec_relres=resnorms[-1] / denom,
                    true_relres=_sqrt(np.dot(true_res, true_res)) / denom,
                    spmvs=spmvs, iterates=iterates, resnorms=resnorms)
