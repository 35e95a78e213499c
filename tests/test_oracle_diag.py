"""Pins for the one-point-stencil toy problem (Sec. 4.2): a diagonal matrix with
the 2D Laplacian's spectrum.  The diagonal comes from the input generator; the
oracle applies it as a plain diagonal operator."""
import numpy as np
import pytest
import scipy.fft

import synth
from oracle import cg as ocg
from oracle import operators, shifts
from oracle import plcg as oplcg


def _sine(dims, u):
    """Orthonormal sine transform (DST-I) along every axis of a flat grid vector."""
    shape = tuple(reversed(dims))
    return scipy.fft.dstn(u.reshape(shape), type=1, norm="ortho").reshape(-1)


@pytest.mark.parametrize("dims", [(7, 5), (16, 16), (4, 6, 3)])
def test_diagonal_is_the_laplacian_spectrum(dims):
    d = synth.spectrum_diagonal(dims)
    assert np.allclose(np.sort(d), operators.laplacian_eigenvalues(dims), rtol=0, atol=1e-13)


@pytest.mark.parametrize("dims", [(7, 5), (12, 9), (4, 6, 3)])
def test_sine_transform_diagonalises_the_laplacian_in_grid_order(dims):
    """S A u = diag(d) S u with S the orthonormal sine transform: entry p of the
    diagonal belongs to the sine mode that the transform puts at p."""
    A = operators.laplacian(dims)
    d = synth.spectrum_diagonal(dims)
    u = synth.uniform(A.n, 31)
    assert np.abs(_sine(dims, A(u)) - d * _sine(dims, u)).max() <= 1e-13 * np.abs(d * u).max() * 8


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_toy_iterates_are_the_rotated_laplacian_iterates(l):
    """Krylov iterates are invariant under an orthogonal change of basis: CG and
    p(l)-CG on diag(d) with rhs S b give S x_t, where x_t are the iterates on the
    Laplacian with rhs b (S = sine transform)."""
    dims = (24, 20)
    A = operators.laplacian(dims)
    D = operators.diagonal(synth.spectrum_diagonal(dims))
    b = synth.uniform(A.n, 41)
    bh = _sine(dims, b)
    x0 = np.zeros(A.n)
    for t in (1, 5, 20):
        if l == 0:
            xa = ocg.cg(A, b, x0, 1e-30, t).x
            xd = ocg.cg(D, bh, x0, 1e-30, t).x
        else:
            sig = shifts.chebyshev_shifts(l, 0.0, 8.0)
            xa = oplcg.alg1(A, b, x0, l, sig, 0.0, t).x
            xd = oplcg.alg1(D, bh, x0, l, sig, 0.0, t).x
        assert np.linalg.norm(xd - _sine(dims, xa)) <= 1e-12 * np.linalg.norm(xd)


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_toy_terminates_after_the_number_of_distinct_eigenvalues(l):
    """On a diagonal matrix with m distinct entries CG reaches the solution in m
    steps (finite termination); p(l)-CG has the same x_t in exact arithmetic.  In
    FP64 the deeper pipeline propagates more rounding (Sec. 2.2), so l = 3 gets a
    looser bound; a wrong term would leave an O(1) residual."""
    dims = (6, 4)
    d = synth.spectrum_diagonal(dims)
    m = len(np.unique(np.round(d, 12)))
    D = operators.diagonal(d)
    b = synth.uniform(D.n, 42)
    x0 = np.zeros(D.n)
    if l == 0:
        x = ocg.cg(D, b, x0, 1e-30, m).x
    else:
        x = oplcg.alg1(D, b, x0, l, shifts.chebyshev_shifts(l, 0.0, 8.0), 0.0, m).x
    assert np.linalg.norm(d * x - b) <= (1e-9 if l <= 2 else 1e-6) * np.linalg.norm(b)
