"""Pins for the CSR input generator and the oracle's CSR operator: the assembled
matrices equal the oracle's independently written grid operators."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import operators


@pytest.mark.parametrize("dims", [(7, 5), (1, 9), (4, 3, 6), (64, 64)])
def test_csr_laplacian_equals_stencil(dims):
    rp, ci, va = synth.csr_variable_laplacian(dims)
    A = operators.laplacian(dims)
    C = operators.csr(rp, ci, va)
    u = synth.uniform(A.n, 61)
    assert np.abs(C(u) - A(u)).max() <= 1e-14 * np.abs(A(u)).max() * 8
    assert rp[0] == 0 and rp[-1] == len(ci) and np.all(np.diff(rp) >= 0)
    assert ci.dtype == np.int32 and rp.dtype == np.int64
    # columns ascending within rows, matrix symmetric
    for p in range(min(A.n, 50)):
        assert np.all(np.diff(ci[rp[p]:rp[p + 1]]) > 0)
    M = sp.csr_matrix((va, ci, rp), shape=(A.n, A.n))
    assert abs(M - M.T).max() == 0


@pytest.mark.parametrize("dims", [(9, 6), (5, 4, 3)])
def test_csr_variable_laplacian_equals_oracle_operator(dims):
    cx, cy, cz = synth.edge_coefficients(dims, 62)
    rp, ci, va = synth.csr_variable_laplacian(dims, cx, cy, cz)
    A, As, dis = operators.variable_laplacian(dims, cx, cy, cz)
    C = operators.csr(rp, ci, va)
    u = synth.uniform(A.n, 63)
    assert np.abs(C(u) - A(u)).max() <= 1e-13 * np.abs(A(u)).max()
    # SPD: smallest eigenvalue of the dense matrix is positive
    assert np.linalg.eigvalsh(operators.assemble(C))[0] > 0
