"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle's callers.

This module holds no arithmetic of the solver: it only draws numbers and names
workloads.  Every random vector is a counter-based SplitMix64 stream (Steele,
Lea and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
element ``i`` of a stream with seed ``s`` is ``mix64(s + (i + 1) * GOLDEN)``
with the published SplitMix64 finaliser, mapped to a double in ``[-1, 1)`` from
its top 53 bits.  Because element ``i`` depends only on ``(s, i)``, any slice of
a vector can be regenerated without the rest of it.

Workloads (grid ordering is row-major with x fastest; Dirichlet boundary values
are eliminated, so an ``nx*ny`` grid has ``nx*ny`` unknowns):

* ``poisson64_manufactured`` - 2D 5-point, 64x64, x* uniform[-1,1) from the seed,
  b = A x* (b is formed by the caller with its own operator), x0 = 0.
* ``poisson2048`` - 2D 5-point, 2048x2048, b uniform[-1,1) from the seed, x0 = 0.
* ``poisson3d256`` - 3D 7-point, 256^3, b uniform[-1,1) from the seed, x0 = 0.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Raw 64-bit outputs ``start .. start+count-1`` of the SplitMix64 stream ``seed``."""
    idx = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + idx * GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform(n: int, seed: int, start: int = 0) -> np.ndarray:
    """``n`` float64 values uniform on [-1, 1): top 53 bits of SplitMix64, scaled."""
    z = splitmix64(seed, start, n)
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0


# Named workloads: (operator kind, grid dims, right-hand side kind, Chebyshev interval).
WORKLOADS = {
    "poisson64_manufactured": dict(kind="2d5", dims=(64, 64), rhs="manufactured",
                                   interval=(0.0, 8.0), tol=1e-8),
    "poisson2048": dict(kind="2d5", dims=(2048, 2048), rhs="uniform",
                        interval=(0.0, 8.0), tol=1e-8),
    "poisson3d256": dict(kind="3d7", dims=(256, 256, 256), rhs="uniform",
                         interval=(0.0, 12.0), tol=1e-10),
    # the latency- to bandwidth-bound transition: 2D Poisson from 128^2 to 1024^2
    "poisson128": dict(kind="2d5", dims=(128, 128), rhs="uniform", interval=(0.0, 8.0), tol=1e-8),
    "poisson256": dict(kind="2d5", dims=(256, 256), rhs="uniform", interval=(0.0, 8.0), tol=1e-8),
    "poisson512": dict(kind="2d5", dims=(512, 512), rhs="uniform", interval=(0.0, 8.0), tol=1e-8),
    "poisson1024": dict(kind="2d5", dims=(1024, 1024), rhs="uniform", interval=(0.0, 8.0),
                        tol=1e-8),
    # the 2048^2 Poisson problem assembled in CSR (a general sparse matrix, as
    # the paper's PETSc runs store it)
    "csr2048": dict(kind="csr", dims=(2048, 2048), rhs="uniform",
                    interval=(0.0, 8.0), tol=1e-8),
    # the one-point-stencil toy: diagonal with the 2048^2 Laplacian's spectrum,
    # the same right-hand side as poisson2048
    "diag2048": dict(kind="diag", dims=(2048, 2048), rhs="uniform",
                     interval=(0.0, 8.0), tol=1e-8),
    "diag64": dict(kind="diag", dims=(64, 64), rhs="uniform",
                   interval=(0.0, 8.0), tol=1e-8),
    # 2D variable-coefficient 5-point operator (lognormal(0, 1) edge coefficients
    # from seed 7), solved Jacobi-scaled with shifts on [0, 2]; b uniform, seed 0
    "varcoef2048": dict(kind="2d5var", dims=(2048, 2048), rhs="uniform",
                        interval=(0.0, 2.0), tol=1e-8, coef_seed=7),
}


def grid_size(dims) -> int:
    n = 1
    for d in dims:
        n *= int(d)
    return n


def spectrum_diagonal(dims) -> np.ndarray:
    """Diagonal of the one-point-stencil toy problem on the grid ``dims``: entry
    p = x + nx*(y + ny*z) is the eigenvalue of the Dirichlet Laplacian's sine mode
    with wave numbers (x+1, y+1, z+1), i.e. the sum over the axes of
    4 sin^2(k pi / (2 (n + 1))).  An operator definition (input data), in the
    order of the grid's unknowns."""
    d = np.zeros(1)
    for n in dims:          # x varies fastest: later axes are the slower index
        k = np.arange(1, int(n) + 1)
        f = 4.0 * np.sin(k * np.pi / (2.0 * (int(n) + 1))) ** 2
        d = (f[:, None] + d[None, :]).reshape(-1)
    return d


def _csr(n, rows, cols, vals):
    """CSR arrays (rowptr int64, colind int32, vals float64) from coordinate
    triplets, columns ascending within each row."""
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rowptr[1:])
    return rowptr, cols.astype(np.int32), vals.astype(np.float64)


def csr_variable_laplacian(dims, cx=None, cy=None, cz=None):
    """The grid operator (A u)_p = sum over the edges (p, q) at p of c_pq (u_p - u_q),
    u = 0 outside (boundary edges add to the diagonal), assembled in CSR.  Edge
    layouts as in edge_coefficients; None means all coefficients 1, which gives
    the unscaled 5-point (7-point) Dirichlet Laplacian.  An operator definition
    (input data)."""
    dims = tuple(int(d) for d in dims)
    d3 = len(dims) == 3
    nx, ny = dims[0], dims[1]
    nz = dims[2] if d3 else 1
    n = nx * ny * nz
    CX = np.ones((nz, ny, nx + 1)) if cx is None else np.asarray(cx, float).reshape(nz, ny, nx + 1)
    CY = np.ones((nz, ny + 1, nx)) if cy is None else np.asarray(cy, float).reshape(nz, ny + 1, nx)
    if d3:
        CZ = (np.ones((nz + 1, ny, nx)) if cz is None
              else np.asarray(cz, float).reshape(nz + 1, ny, nx))
    idx = np.arange(n).reshape(nz, ny, nx)
    diag = CX[:, :, :-1] + CX[:, :, 1:] + CY[:, :-1, :] + CY[:, 1:, :]
    if d3:
        diag = diag + CZ[:-1] + CZ[1:]
    rows = [idx.reshape(-1)]
    cols = [idx.reshape(-1)]
    vals = [diag.reshape(-1)]

    def couple(a, b, c):          # symmetric entries -c between unknowns a and b
        rows.extend([a.reshape(-1), b.reshape(-1)])
        cols.extend([b.reshape(-1), a.reshape(-1)])
        vals.extend([-c.reshape(-1), -c.reshape(-1)])

    couple(idx[:, :, :-1], idx[:, :, 1:], CX[:, :, 1:-1])
    couple(idx[:, :-1, :], idx[:, 1:, :], CY[:, 1:-1, :])
    if d3:
        couple(idx[:-1], idx[1:], CZ[1:-1])
    return _csr(n, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def sample_indices(n: int, count: int = 512, seed: int = 12345) -> np.ndarray:
    """Sorted distinct indices for spot checks: the first and last 32, plus
    SplitMix64 draws spread over [0, n)."""
    edge = min(32, n)
    head = np.arange(edge, dtype=np.int64)
    tail = np.arange(max(0, n - edge), n, dtype=np.int64)
    draws = (splitmix64(seed, 0, count) % np.uint64(max(n, 1))).astype(np.int64)
    return np.unique(np.concatenate([head, tail, draws]))


def dense_sample_indices(dims) -> np.ndarray:
    """Whole grid rows for dense spot checks of full-size results, where a
    parallel split of the grid into eighths puts its seams.  2D (nx, ny): the
    first and last row and rows k*ny/8 - 1 and k*ny/8 for k = 1..7.  3D
    (nx, ny, nz): in planes 0, nz/8 - 1, nz/8, nz/2 - 1, nz/2 and nz - 1, rows 0,
    15, 16, 31, 32, ny/2 - 1, ny/2 and ny - 1.  Sorted, distinct, in range."""
    dims = tuple(int(d) for d in dims)
    nx, ny = dims[0], dims[1]
    if len(dims) == 2:
        rows = {0, ny - 1}
        for k in range(1, 8):
            rows |= {k * ny // 8 - 1, k * ny // 8}
        cells = [(0, y) for y in rows]
    else:
        nz = dims[2]
        planes = {0, nz // 8 - 1, nz // 8, nz // 2 - 1, nz // 2, nz - 1}
        rows = {0, 15, 16, 31, 32, ny // 2 - 1, ny // 2, ny - 1}
        cells = [(z, y) for z in planes for y in rows]
    ny_, nz_ = ny, dims[2] if len(dims) == 3 else 1
    starts = sorted({(z * ny_ + y) * nx for z, y in cells if 0 <= y < ny_ and 0 <= z < nz_})
    return np.concatenate([np.arange(s0, s0 + nx, dtype=np.int64) for s0 in starts])


def lognormal(n: int, seed: int, start: int = 0) -> np.ndarray:
    """``n`` lognormal(0, 1) values: exp of a standard normal from the Box-Muller
    transform of two SplitMix64 uniforms (u1 in (0, 1], u2 in [0, 1))."""
    z = splitmix64(seed, 2 * start, 2 * n)
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    u1 = 1.0 - u[0::2]
    u2 = u[1::2]
    g = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return np.exp(g)


def edge_coefficients(dims, seed: int):
    """Edge coefficients of a variable-coefficient grid operator, lognormal(0, 1).

    2D dims (nx, ny): cx has ny rows of nx+1 edges (x-edges, the first and last
    of a row touch the boundary), cy has ny+1 rows of nx (y-edges).  3D adds cz
    with nz+1 planes of ny*nx.  Flat arrays, x fastest; three independent
    streams derived from ``seed``.
    """
    dims = tuple(int(d) for d in dims)
    nx, ny = dims[0], dims[1]
    nz = dims[2] if len(dims) == 3 else 1
    cx = lognormal((nx + 1) * ny * nz, seed * 3 + 1)
    cy = lognormal(nx * (ny + 1) * nz, seed * 3 + 2)
    cz = lognormal(nx * ny * (nz + 1), seed * 3 + 3) if len(dims) == 3 else None
    return cx, cy, cz


def batch_recipe(count: int = 512, seed: int = 0, lo: int = 32, hi: int = 512):
    """The batched workload: `count` 2D systems with side uniform on [lo, hi]
    (square grids), edge coefficients lognormal(0, 1), b uniform[-1, 1).
    Returns a list of (dims, coefficient seed, rhs seed)."""
    sides = lo + (splitmix64(seed * 7 + 5, 0, count) % np.uint64(hi - lo + 1)).astype(np.int64)
    return [((int(s), int(s)), 1000 + 2 * k, 1001 + 2 * k) for k, s in enumerate(sides)]
