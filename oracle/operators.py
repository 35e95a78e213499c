"""Operators for the oracle (test infrastructure only).

The stencils are the unscaled integer Dirichlet Laplacians whose spectra lie in
(0, 8) in 2D and (0, 12) in 3D, the intervals on which the Chebyshev shifts of
Sec. 2.2 are placed for these problems.  Unknowns are ordered row-major with x
fastest; values outside the grid are zero (Dirichlet boundary eliminated).

  2D 5-point: (Au)[y,x] = 4 u[y,x] - u[y-1,x] - u[y+1,x] - u[y,x-1] - u[y,x+1]
  3D 7-point: (Au)[z,y,x] = 6 u[z,y,x] - (six face neighbours)
"""
from __future__ import annotations

import numpy as np


def _neighbour_sum(U: np.ndarray) -> np.ndarray:
    """Sum of the face neighbours of every grid point, zero outside the grid."""
    S = np.zeros_like(U)
    for ax in range(U.ndim):
        n = U.shape[ax]
        if n < 2:
            continue
        lo = [slice(None)] * U.ndim
        hi = [slice(None)] * U.ndim
        lo[ax] = slice(0, n - 1)
        hi[ax] = slice(1, n)
        S[tuple(lo)] += U[tuple(hi)]   # neighbour at +1 along ax
        S[tuple(hi)] += U[tuple(lo)]   # neighbour at -1 along ax
    return S


def laplacian(dims):
    """Return ``A(u)`` for the Dirichlet Laplacian on a grid of shape ``dims``: the
    finite-difference test problems of Sec. 4.2 (2D 5-point) and its 3D 7-point
    counterpart, unscaled.

    ``dims`` is (nx, ny) for the 5-point stencil or (nx, ny, nz) for the 7-point
    stencil; the operator acts on flat vectors of length prod(dims).
    """
    dims = tuple(int(d) for d in dims)
    shape = tuple(reversed(dims))          # numpy shape: (ny, nx) or (nz, ny, nx)
    diag = 2 * len(dims)

    def apply(u: np.ndarray) -> np.ndarray:
        U = u.reshape(shape)
        return (diag * U - _neighbour_sum(U)).reshape(-1)

    apply.n = int(np.prod(dims))
    apply.dims = dims
    return apply


def dense(M: np.ndarray):
    """Operator from an explicit matrix."""
    def apply(u):
        return M @ u
    apply.n = M.shape[0]
    return apply


def diagonal(d):
    """The diagonal operator (A u)_p = d_p u_p (the one-point stencil, Sec. 4.2)."""
    d = np.asarray(d, dtype=float)

    def apply(u):
        return d * u
    apply.n = d.shape[0]
    return apply


def csr(rowptr, colind, vals):
    """A sparse matrix given in compressed sparse rows, applied with scipy (the
    assembled matrices of the paper's PETSc runs, Sec. 4)."""
    import scipy.sparse as sp
    n = len(rowptr) - 1
    M = sp.csr_matrix((np.asarray(vals, float), np.asarray(colind), np.asarray(rowptr)),
                      shape=(n, n))

    def apply(u):
        return M @ u
    apply.n = n
    return apply


def assemble(apply) -> np.ndarray:
    """Dense matrix of a (small) operator, column by column."""
    n = apply.n
    M = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[j] = 1.0
        M[:, j] = apply(e)
        e[j] = 0.0
    return M


def laplacian_eigenvalues(dims) -> np.ndarray:
    """Closed-form spectrum of the Dirichlet Laplacian on ``dims``.

    For each axis of length n the 1D factor contributes 4 sin^2(k pi / (2(n+1))),
    k = 1..n (textbook result for the tridiagonal matrix tridiag(-1, 2, -1));
    the d-dimensional spectrum is the set of all sums of one factor per axis.
    """
    lam = np.zeros(1)
    for n in dims:
        k = np.arange(1, n + 1)
        f = 4.0 * np.sin(k * np.pi / (2.0 * (n + 1))) ** 2
        lam = (lam[:, None] + f[None, :]).reshape(-1)
    return np.sort(lam)


def laplacian_mode(dims, ks) -> np.ndarray:
    """Eigenvector of the Dirichlet Laplacian for wave numbers ``ks`` (flat, x fastest)."""
    vec = np.ones(1)
    for n, k in zip(dims, ks):
        j = np.arange(1, n + 1)
        f = np.sin(j * k * np.pi / (n + 1))
        vec = (f[:, None] * vec[None, :]).reshape(-1)   # later axes vary slower
    return vec


def laplacian_extremes(dims):
    """(lambda_min, lambda_max) in closed form."""
    lmin = sum(4.0 * np.sin(np.pi / (2.0 * (n + 1))) ** 2 for n in dims)
    lmax = sum(4.0 * np.cos(np.pi / (2.0 * (n + 1))) ** 2 for n in dims)
    return lmin, lmax


def variable_laplacian(dims, cx, cy, cz=None):
    """Variable-coefficient Dirichlet Laplacian and its Jacobi scaling (the
    operator of the batched workloads; scaling = Alg. 1 with M = diag(A) in its
    symmetric form, Sec. 2.2 on preconditioning).

    (A u)_p = sum over the grid edges (p, q) incident to p of c_pq (u_p - u_q),
    with u = 0 outside the grid, so the diagonal d_p is the sum of all edges at
    p (boundary edges included) and A is an SPD M-matrix.  Returns (A, As, dis)
    where As = D^{-1/2} A D^{-1/2} and dis = D^{-1/2} (diagonal of As is 1).
    Edge layouts as in synth.edge_coefficients.
    """
    dims = tuple(int(d) for d in dims)
    d3 = len(dims) == 3
    nx, ny = dims[0], dims[1]
    nz = dims[2] if d3 else 1
    CX = np.asarray(cx, dtype=float).reshape(nz, ny, nx + 1)
    CY = np.asarray(cy, dtype=float).reshape(nz, ny + 1, nx)
    CZ = np.asarray(cz, dtype=float).reshape(nz + 1, ny, nx) if d3 else None
    diag = CX[:, :, :-1] + CX[:, :, 1:] + CY[:, :-1, :] + CY[:, 1:, :]
    if d3:
        diag = diag + CZ[:-1] + CZ[1:]
    W = CX[:, :, 1:-1]          # interior x-edges between (x, x+1)
    N = CY[:, 1:-1, :]          # interior y-edges
    T = CZ[1:-1] if d3 else None

    def apply(u):
        U = u.reshape(nz, ny, nx)
        out = diag * U
        out[:, :, :-1] -= W * U[:, :, 1:]
        out[:, :, 1:] -= W * U[:, :, :-1]
        out[:, :-1, :] -= N * U[:, 1:, :]
        out[:, 1:, :] -= N * U[:, :-1, :]
        if d3:
            out[:-1] -= T * U[1:]
            out[1:] -= T * U[:-1]
        return out.reshape(-1)

    dis = (1.0 / np.sqrt(diag)).reshape(-1)

    def apply_scaled(u):
        return dis * apply(dis * u)

    n = nx * ny * nz
    apply.n = n
    apply_scaled.n = n
    return apply, apply_scaled, dis
