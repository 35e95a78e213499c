"""Pins of the variable-coefficient operator and its Jacobi scaling."""
import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import operators, shifts
from oracle import cg as ocg
from oracle import plcg as oplcg


@pytest.mark.parametrize("dims", [(7, 5), (4, 3, 5), (1, 6), (6, 1, 2)])
def test_unit_coefficients_give_the_laplacian(dims):
    n = int(np.prod(dims))
    nx, ny = dims[0], dims[1]
    nz = dims[2] if len(dims) == 3 else 1
    A, As, dis = operators.variable_laplacian(dims, np.ones((nx + 1) * ny * nz),
                                              np.ones(nx * (ny + 1) * nz),
                                              np.ones(nx * ny * (nz + 1)) if len(dims) == 3 else None)
    L = operators.laplacian(dims)
    M = operators.assemble(A)
    assert np.array_equal(M, operators.assemble(L))
    assert np.allclose(dis, 1.0 / np.sqrt(2 * len(dims)))


@pytest.mark.parametrize("dims", [(9, 7), (5, 4, 3)])
def test_scaled_operator_spd_unit_diagonal_spectrum_in_0_2(dims):
    cx, cy, cz = synth.edge_coefficients(dims, 3)
    A, As, dis = operators.variable_laplacian(dims, cx, cy, cz)
    M = operators.assemble(A)
    Ms = operators.assemble(As)
    assert np.allclose(M, M.T, rtol=0, atol=1e-13)
    assert np.allclose(np.diag(Ms), 1.0)
    ev = scipy.linalg.eigvalsh(Ms)
    assert ev[0] > 0 and ev[-1] < 2          # Gershgorin on a unit-diagonal M-matrix
    assert np.allclose(Ms, np.diag(dis) @ M @ np.diag(dis), atol=1e-14)
    # an M-matrix: non-positive off-diagonal, weakly dominant rows
    off = M - np.diag(np.diag(M))
    assert np.all(off <= 0) and np.all(np.diag(M) >= -off.sum(axis=1) * (1 - 1e-14))


def test_lognormal_generator():
    v = synth.lognormal(200000, 7)
    g = np.log(v)
    assert abs(g.mean()) < 0.01 and abs(g.std() - 1.0) < 0.01
    assert np.array_equal(synth.lognormal(5, 7, start=3), synth.lognormal(8, 7)[3:])


def test_scaled_plcg_matches_jacobi_cg_count():
    """On the Jacobi-scaled operator with shifts on [0, 2] (the interval of the
    paper's block-Jacobi runs, Sec. 4.2), p(l)-CG needs the same iteration count
    as CG on the same operator."""
    dims = (32, 32)
    cx, cy, cz = synth.edge_coefficients(dims, 11)
    A, As, dis = operators.variable_laplacian(dims, cx, cy, cz)
    b = synth.uniform(1024, 12)
    bs = dis * b
    ref = ocg.cg(As, bs, np.zeros(1024), 1e-8, 5000)
    for l in (2, 3):
        r = oplcg.plcg(As, bs, np.zeros(1024), l, shifts.chebyshev_shifts(l, 0.0, 2.0), 1e-8, 5000)
        assert r.reason == "converged" and abs(r.iters - ref.iters) <= 2
        x = dis * r.x
        assert np.linalg.norm(b - A(x)) / np.linalg.norm(b) < 1e-6


def test_batch_recipe_sizes():
    rec = synth.batch_recipe()
    sides = np.array([d[0] for d, _, _ in rec])
    assert len(rec) == 512 and sides.min() >= 32 and sides.max() <= 512
    assert 4.0e7 < np.sum(sides.astype(float) ** 2) < 6.5e7


@pytest.mark.parametrize("l", [1, 2, 3])
def test_preconditioned_alg1_equals_scaled_system(l):
    """Alg. 1 with M = diag(A) (u != z, M-inner products, Sec. 2.2) on A x = b has
    the same iterates as Alg. 1 with M = I on D^{-1/2} A D^{-1/2} y = D^{-1/2} b,
    mapped back by x = D^{-1/2} y - the symmetric scaling the batched solver uses
    - and both equal Jacobi-preconditioned CG (here: CG on the scaled system)."""
    dims = (24, 20)
    cx, cy, cz = synth.edge_coefficients(dims, 4)
    A, As, dis = operators.variable_laplacian(dims, cx, cy, cz)
    n = A.n
    b = synth.uniform(n, 5)
    dinv = dis * dis                            # M^{-1} = D^{-1}
    sig = shifts.chebyshev_shifts(l, 0.0, 2.0)
    ref = ocg.cg(As, dis * b, np.zeros(n), 1e-30, 12, record_iterates=True)
    for t in (1, 4, 12):
        pre = oplcg.alg1(A, b, np.zeros(n), l, sig, 0.0, t, Minv=lambda u: dinv * u)
        sca = oplcg.alg1(As, dis * b, np.zeros(n), l, sig, 0.0, t)
        xs = dis * sca.x
        xc = dis * ref.iterates[t - 1]
        assert pre.t_done == sca.t_done == t
        assert np.linalg.norm(pre.x - xs) <= 1e-12 * np.linalg.norm(xs)
        assert np.linalg.norm(pre.x - xc) <= 1e-12 * np.linalg.norm(xc)
    # the natural residual norm sqrt((u_0, r_0)) is the scaled residual norm
    pre = oplcg.alg1(A, b, np.zeros(n), l, sig, 0.0, 3, Minv=lambda u: dinv * u)
    assert abs(pre.beta - np.linalg.norm(dis * b)) <= 1e-12 * pre.beta
