"""Deep pipelined CG, p(l)-CG, as the paper's Alg. 1 (test infrastructure only).

Scope: Alg. 1 with the identity preconditioner (M = I).  Then the unpreconditioned
auxiliary vector u_i coincides with z^{(l)}_i (Sec. 2.2, "Preconditioned p(l)-CG",
with M = I), so Alg. 1's u-update is the z^{(l)}-update and (u_0, r_0) = ||r_0||^2.

Everything is kept in dictionaries indexed exactly like the paper:
    z[k][j]  = z^{(k)}_j   (k = 0..l; z[0] is the orthonormal Lanczos basis V)
    G[j, c]  = g_{j,c}     (banded upper triangular, Z = V G; Sec. 2.1)
    gam[t], dlt[t]         (the tridiagonal T, Eq. Arnoldi_v2)
    eta[t], lam[t], zeta[t](LU factors of T and the vector q; Eqs. LU, x_a)
Iteration i of the loop updates column c = i - l + 1 of G and the Lanczos index
t = i - l, exactly as the algorithm is laid out; a step that the paper writes
for i >= l is skipped for smaller i.

Two forms of the dot products that start column i+1 of G (Alg. 1, "initiate
dot-products"):
  dots="full"       all 2l+1 products, (u_{i+1}, z^{(0)}_j) for
                    j = max(0, i-2l+1)..i-l+1 and (u_{i+1}, z^{(l)}_j) for
                    j = i-l+2..i+1, as printed in the algorithm;
  dots="symmetric"  only the l+1 products (u_{i+1}, z^{(l)}_j), j = i-l+2..i+1,
                    and (u_{i+1}, v_{i-l+1}); the remaining l entries of the
                    column are taken from Eq. (symmetry_G), g_{j,c} = g_{c-l,j+l},
                    when the column is finalised (Sec. 2.2, "Number of dot
                    products in p(l)-CG").

Readings of points the paper leaves open (each is listed with its reason in the
design notes of the repository):
  * indices below zero are dropped from every range and sum; delta_{-1} = 0;
  * the corrections of g_{j,c} (Eq. before haa1) run over increasing j, each
    using the already corrected entries g_{k,c}, k < j (forward substitution);
  * the convergence test uses |zeta_t| against tol times the norm of the
    residual of the caller's starting vector; after a restart this reference
    norm is kept, so the global criterion does not change;
  * breakdown = the square-root argument is not positive, or a non-finite
    value, or delta_t <= 0, or eta_t <= 0 (the last two cannot happen for an
    SPD matrix in exact arithmetic).  On breakdown Alg. 1 is restarted
    explicitly (Sec. 2.2, "Square root breakdowns") from the most recent
    iterate, x_{t-1}, with a freshly computed residual.
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


def _finite(a) -> bool:
    if isinstance(a, (float, np.floating)):
        return math.isfinite(a)
    import mpmath
    return bool(mpmath.isfinite(a))


class Breakdown(Exception):
    def __init__(self, t, where):
        super().__init__(f"breakdown at t={t} ({where})")
        self.t = t
        self.where = where


# ---------------------------------------------------------------------------
# Scalar steps (K2, K3 and the scalar half of K6 in the kernel table of Sec. 3.1)
# ---------------------------------------------------------------------------

def fill_symmetric(G, c, l):
    """Entries g_{j,c}, j = c-2l .. c-l-1, from Eq. (symmetry_G): g_{j,c} = g_{c-l, j+l}.

    Used only with the l+1 dot-product form.  Columns j+l < c are final by now.
    """
    for j in range(max(0, c - 2 * l), c - l):
        G[j, c] = G[c - l, j + l]


def finalize_column(G, c, l):
    """Turn the raw dot products of column c into g_{.,c} (Alg. 1, update of G).

    For j = c-l+1 .. c-1 (increasing):
        g_{j,c} <- (g_{j,c} - sum_{k=c-2l}^{j-1} g_{k,j} g_{k,c}) / g_{j,j}
    then g_{c,c} <- sqrt(g_{c,c} - sum_{k=c-2l}^{c-1} g_{k,c}^2).
    In iteration i of Alg. 1 the column is c = i-l+1, so c-2l = i-3l+1.
    Returns the square-root argument; raises Breakdown if it is not positive.
    """
    lo = max(0, c - 2 * l)
    for j in range(max(0, c - l + 1), c):
        s = G[j, c]
        for k in range(lo, j):
            s = s - G[k, j] * G[k, c]
        G[j, c] = s / G[j, j]
    arg = G[c, c]
    for k in range(lo, c):
        arg = arg - G[k, c] * G[k, c]
    if not (_finite(arg) and arg > 0):
        raise Breakdown(c - 1, "sqrt")
    G[c, c] = _sqrt(arg)
    return arg


def update_T(G, gam, dlt, sigma, t, l):
    """Add column t of the tridiagonal T (Eqs. haa1, haa3), t = i - l.

    t < l  (l <= i < 2l):
        gamma_t = (g_{t,t+1} + sigma_t g_{t,t} - g_{t-1,t} delta_{t-1}) / g_{t,t}
        delta_t = g_{t+1,t+1} / g_{t,t}
    t >= l (i >= 2l):
        gamma_t = (g_{t,t} gamma_{t-l} + g_{t,t+1} delta_{t-l} - g_{t-1,t} delta_{t-1}) / g_{t,t}
        delta_t = g_{t+1,t+1} delta_{t-l} / g_{t,t}
    The term g_{t-1,t} delta_{t-1} is zero for t = 0.
    """
    corr = G[t - 1, t] * dlt[t - 1] if t >= 1 else 0.0
    if t < l:
        gam[t] = (G[t, t + 1] + sigma[t] * G[t, t] - corr) / G[t, t]
        dlt[t] = G[t + 1, t + 1] / G[t, t]
    else:
        gam[t] = (G[t, t] * gam[t - l] + G[t, t + 1] * dlt[t - l] - corr) / G[t, t]
        dlt[t] = (G[t + 1, t + 1] * dlt[t - l]) / G[t, t]
    if not (_finite(gam[t]) and _finite(dlt[t]) and dlt[t] > 0):
        raise Breakdown(t, "T")


def update_LU(gam, dlt, eta, lam, zeta, t, beta):
    """LU factorisation of T and the recursive residual (Eq. LU and Sec. 2.1).

    t = 0: eta_0 = gamma_0, zeta_0 = ||r_0||.
    t >= 1: lambda_t = delta_{t-1}/eta_{t-1}, eta_t = gamma_t - lambda_t delta_{t-1},
            zeta_t = -lambda_t zeta_{t-1}.
    """
    if t == 0:
        eta[0] = gam[0]
        zeta[0] = beta
    else:
        lam[t] = dlt[t - 1] / eta[t - 1]
        eta[t] = gam[t] - lam[t] * dlt[t - 1]
        zeta[t] = -lam[t] * zeta[t - 1]
    if not (_finite(eta[t]) and eta[t] > 0):
        raise Breakdown(t, "eta")


# ---------------------------------------------------------------------------
# Vector steps (K1, K4, K5 and the vector half of K6)
# ---------------------------------------------------------------------------

def basis_updates(z, gam, dlt, sigma, t, l, i, store=None):
    """Three-term recurrences of all l+1 bases (Eqs. all_z_rec2, specific_z_rec).

    For k = 0..l-1:
        z^{(k)}_{t+k+1} = (z^{(k+1)}_{t+k+1} + (sigma_k - gamma_t) z^{(k)}_{t+k}
                           - delta_{t-1} z^{(k)}_{t+k-1}) / delta_t
    and z^{(l)}_{i+1} = (A z^{(l)}_i - gamma_t z^{(l)}_i - delta_{t-1} z^{(l)}_{i-1}) / delta_t,
    where z[l][i+1] holds A z^{(l)}_i on entry.  Each update reads only vectors
    that this iteration does not overwrite (basis k writes index t+k+1 and
    basis k-1 reads index t+k of basis k).
    """
    keep = store or (lambda v: v)
    dm1 = dlt[t - 1] if t >= 1 else 0.0
    for k in range(l):
        new = z[k + 1][t + k + 1] + (sigma[k] - gam[t]) * z[k][t + k]
        if t >= 1:
            new = new - dm1 * z[k][t + k - 1]
        z[k][t + k + 1] = keep(new / dlt[t])
    new = z[l][i + 1] - gam[t] * z[l][i]
    if t >= 1:
        new = new - dm1 * z[l][i - 1]
    z[l][i + 1] = keep(new / dlt[t])


def start_dots(G, z, i, l, dots, dot=np.dot, u=None):
    """Dot products that start column i+1 of G (Alg. 1, 'initiate dot-products'),
    with u = u_{i+1} (z^{(l)}_{i+1} when M = I)."""
    if u is None:
        u = z[l][i + 1]
    c = i + 1
    if dots == "full":
        for j in range(max(0, i - 2 * l + 1), i - l + 2):
            G[j, c] = dot(u, z[0][j])
    else:
        j = i - l + 1
        if j >= 0:
            G[j, c] = dot(u, z[0][j])
    for j in range(max(0, i - l + 2), i + 2):
        G[j, c] = dot(u, z[l][j])
    return 2 * l + 1 if dots == "full" else l + 1


@dataclass
class Segment:
    x: np.ndarray
    t_done: int            # number of x updates made (x_1 .. x_{t_done})
    reason: str            # "converged" | "maxit" | "breakdown"
    breakdown_t: int
    beta: float            # ||r_0|| of this segment
    zeta_last: float       # |zeta| of the last x update (beta if none)
    spmvs: int
    dots_per_iter: list
    diag: dict


def alg1(A, b, x0, l, sigma, abs_tol, m, dots="symmetric", keep_all=False, dot=np.dot,
         store=None, Minv=None):
    """One run of Alg. 1 (no restart) with M = I, from x0, at most m x-updates.

    ``dot`` is the inner product (default numpy's); tests pass a correctly
    rounded one to measure how much the results depend on summation order.
    ``store`` (default: none) is applied to every vector the algorithm keeps -
    z^{(k)}_0, each new basis vector, p and x - and models storing them in a
    narrower format (see oracle.refine); A z^{(l)}_i itself is not stored for
    i >= l, it is consumed by the recurrence at once.
    ``Minv`` (default: M = I) applies the preconditioner: Alg. 1 then keeps the
    unpreconditioned u_i = M z^{(l)}_i beside the bases (the u-lines of the
    algorithm, Sec. 2.2 'Preconditioned p(l)-CG'), the dot products are
    (u_{i+1}, z_j) - M-inner products of the z's - and the residual norm is the
    natural one, sqrt((u_0, r_0)).  u_0 is normalised with the z's.

    Stops when |zeta_t| < abs_tol.  Returns a Segment; ``diag`` holds G, gamma,
    delta, eta, lambda, zeta, and also the bases and the search directions when
    keep_all is set.
    """
    if dots not in ("full", "symmetric"):
        raise ValueError(dots)
    sigma = list(sigma)
    if len(sigma) != l:
        raise ValueError("need l shifts")
    x = x0.copy()
    u0 = b - A(x)                              # u_0 = b - A x_0, r_0 = M^{-1} u_0
    r0 = Minv(u0) if Minv is not None else u0
    spmvs = 1
    beta = _sqrt(dot(u0, r0))                  # sqrt((u_0, r_0))
    if beta == 0 or abs_tol >= beta:
        return Segment(x, 0, "converged", -1, beta, beta, spmvs, [], {})
    if not _finite(beta):
        return Segment(x, 0, "nonfinite", -1, beta, beta, spmvs, [], {})
    keep = store or (lambda v: v)
    z = [dict() for _ in range(l + 1)]
    v0 = keep(r0 / beta)
    U = {0: u0 / beta} if Minv is not None else None
    for k in range(l + 1):
        z[k][0] = v0                           # z^{(k)}_0 = r_0 / sqrt((u_0, r_0))
    G = {(0, 0): 1.0 if x0.dtype != object else type(beta)(1)}
    gam, dlt, eta, lam, zeta = {}, {}, {}, {}, {}
    p = None
    P = {}
    t_done = 0
    dots_per_iter = []
    reason = "maxit"
    bt = -1
    for i in range(0, m + l + 1):
        # line 3-4: u_{i+1} = A z^{(l)}_i - sigma_i u_i (i < l), z^{(l)}_{i+1} = u_{i+1}
        w = A(z[l][i])
        spmvs += 1
        if Minv is not None:
            # u_{i+1} = A z_i - sigma_i u_i (i < l), z^{(l)}_{i+1} = M^{-1} u_{i+1}
            if i < l:
                w = w - sigma[i] * U[i]
            U[i + 1] = w
            w = Minv(w)
            if i < l:
                w = keep(w)
        elif i < l:
            w = keep(w - sigma[i] * z[l][i])
        z[l][i + 1] = w
        # line 5-6: the first vectors of bases i+1 .. l-1 are copies
        if i < l - 1:
            for k in range(i + 1, l):
                z[k][i + 1] = z[l][i + 1]
        if i >= l:
            t = i - l
            c = t + 1
            try:
                if dots == "symmetric":
                    fill_symmetric(G, c, l)
                finalize_column(G, c, l)             # K2
                update_T(G, gam, dlt, sigma, t, l)   # K3
                if t >= 1 or i == l:
                    update_LU(gam, dlt, eta, lam, zeta, t, beta)
            except Breakdown as e:
                reason = "breakdown"
                bt = e.t
                break
            basis_updates(z, gam, dlt, sigma, t, l, i, store)   # K4
            if Minv is not None:
                # u_{i+1} = (u_{i+1} - gamma_t u_i - delta_{t-1} u_{i-1}) / delta_t
                un = U[i + 1] - gam[t] * U[i]
                if t >= 1:
                    un = un - dlt[t - 1] * U[i - 1]
                U[i + 1] = un / dlt[t]
        extra = {} if Minv is None else {"u": U[i + 1]}
        dots_per_iter.append(start_dots(G, z, i, l, dots, dot, **extra))   # K5
        # K6: search direction and iterate
        if i == l:
            p = keep(z[0][0] / eta[0])
            P[0] = p
        elif i >= l + 1:
            t = i - l
            p_new = keep((z[0][t] - dlt[t - 1] * p) / eta[t])
            x = keep(x + zeta[t - 1] * p)
            p = p_new
            P[t] = p
            t_done = t
            if abs(zeta[t]) < abs_tol:
                reason = "converged"
                break
        if not keep_all:
            _forget(z, i, l, dots)
            P.clear()
            if U is not None:
                for j in [j for j in U if j < i - 1]:
                    del U[j]
    zeta_last = abs(zeta[t_done]) if t_done in zeta else beta
    diag = dict(G=G, gam=gam, dlt=dlt, eta=eta, lam=lam, zeta=zeta)
    if keep_all:
        diag.update(z=z, P=P)
    return Segment(x, t_done, reason, bt, beta, zeta_last, spmvs, dots_per_iter, diag)


def _forget(z, i, l, dots):
    """Drop vectors no later iteration reads (the paper keeps the three most
    recent vectors of each basis and the l most recent of Z^{(l)}, Sec. 3.2)."""
    t = i - l
    for k in range(l):
        keep = t + k
        if k == 0 and dots == "full":
            keep = min(keep, i - 2 * l + 2)
        for j in [j for j in z[k] if j < keep]:
            del z[k][j]
    keep_l = min(i, i - l + 3)
    for j in [j for j in z[l] if j < keep_l]:
        del z[l][j]


@dataclass
class PLCGResult:
    x: np.ndarray
    iters: int
    reason: str
    restarts: int
    rnorm0: float
    rec_relres: float
    true_relres: float
    spmvs: int
    segments: list = field(default_factory=list)


def plcg(A, b, x0, l, sigma, tol, maxit, dots="symmetric", max_restarts=100,
         keep_all=False) -> PLCGResult:
    """p(l)-CG with explicit restarts after breakdown (Sec. 2.2).

    Stops when |zeta_t| < tol * ||b - A x0||; the reference norm is that of the
    caller's start and is kept across restarts.  Iteration count = number of
    x updates over all segments.
    """
    x = x0.copy()
    r = b - A(x)
    spmvs = 1
    rnorm0 = _sqrt(np.dot(r, r))
    abs_tol = tol * rnorm0
    total = 0
    restarts = 0
    segments = []
    reason = "maxit"
    rec = rnorm0
    while True:
        seg = alg1(A, b, x, l, sigma, abs_tol, maxit - total, dots=dots, keep_all=keep_all)
        segments.append(seg)
        spmvs += seg.spmvs
        x = seg.x
        total += seg.t_done
        rec = seg.zeta_last
        if seg.reason == "breakdown":
            restarts += 1
            if restarts > max_restarts:
                reason = "breakdown_limit"
                break
            if total >= maxit:
                reason = "maxit"
                break
            continue
        reason = seg.reason
        break
    true_res = b - A(x)
    spmvs += 1
    denom = rnorm0 if rnorm0 != 0 else 1.0
    return PLCGResult(x=x, iters=total, reason=reason, restarts=restarts, rnorm0=rnorm0,
                      rec_relres=rec / denom,
                      true_relres=_sqrt(np.dot(true_res, true_res)) / denom,
                      spmvs=spmvs, segments=segments)
