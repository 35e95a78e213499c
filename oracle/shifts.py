"""Chebyshev shifts for the auxiliary basis (test infrastructure only).

Sec. 2.2 ("Choice of auxiliary basis shifts"), Eq. (chebyshev): for i = 0..l-1

    sigma_i = (lmax + lmin)/2 + (lmax - lmin)/2 * cos((2i + 1) pi / (2l)),

so sigma_0 is the largest shift.  They are the zeros of the degree-l Chebyshev
polynomial mapped from [-1, 1] onto [lmin, lmax], which minimise the 2-norm of
P_l(A) = prod_k (A - sigma_k I) over matrices with spectrum in that interval.
"""
from __future__ import annotations

import math


def chebyshev_shifts(l: int, lmin: float, lmax: float) -> list:
    """sigma_0 .. sigma_{l-1} of Eq. (chebyshev), Sec. 2.2, on [lmin, lmax]."""
    if l < 1:
        raise ValueError("pipeline length l must be >= 1")
    mid = 0.5 * (lmax + lmin)
    half = 0.5 * (lmax - lmin)
    return [mid + half * math.cos((2 * i + 1) * math.pi / (2 * l)) for i in range(l)]
