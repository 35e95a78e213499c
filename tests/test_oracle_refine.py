"""Pins of the mixed-precision oracle (FP32-stored p(l)-CG inside FP64 refinement)."""
import numpy as np
import pytest

import synth
from oracle import operators, refine, shifts
from oracle import plcg as oplcg


def _problem(dims=(20, 18, 16), seed=0):
    A = operators.laplacian(dims)
    return A, synth.uniform(A.n, seed)


def test_stored_vectors_are_binary32():
    A, b = _problem()
    seg = oplcg.alg1(A, b, np.zeros(A.n), 3, shifts.chebyshev_shifts(3, 0, 12), 0.0, 12,
                     keep_all=True, store=refine.round_fp32)
    z = seg.diag["z"]
    for k in range(4):
        for j, v in z[k].items():
            assert np.array_equal(v, v.astype(np.float32).astype(np.float64)), (k, j)
    for v in seg.diag["P"].values():
        assert np.array_equal(v, v.astype(np.float32).astype(np.float64))


def test_fp32_storage_alone_has_a_residual_gap():
    """Without refinement the recursive |zeta_t| keeps falling while the true
    residual of the FP32-stored iterate stalls (|zeta| equals ||r|| only in exact
    arithmetic, Sec. 2.2 'Residual norm')."""
    A, b = _problem()
    seg = oplcg.alg1(A, b, np.zeros(A.n), 3, shifts.chebyshev_shifts(3, 0, 12),
                     1e-11 * np.linalg.norm(b), 5000, store=refine.round_fp32)
    true = np.linalg.norm(b - A(seg.x)) / np.linalg.norm(b)
    assert seg.reason == "converged" and seg.zeta_last / np.linalg.norm(b) < 1e-11
    assert true > 1e-9


def test_refinement_converges_and_contracts():
    A, b = _problem()
    sig = shifts.chebyshev_shifts(3, 0, 12)
    r = refine.refine(A, b, np.zeros(A.n), 3, sig, 1e-10, 1e-3, 10000)
    assert r.reason == "converged" and r.true_relres < 1e-10
    assert 2 <= r.outer <= 8
    # classical refinement: each step shrinks the true residual by about inner_tol
    rr = refine.refine(A, b, np.zeros(A.n), 3, sig, 1e-30, 1e-3, 10000, max_outer=3)
    assert rr.outer == 3 and rr.true_relres < 1e-7


def test_refinement_without_rounding_is_plain_plcg():
    A, b = _problem((16, 16))
    sig = shifts.chebyshev_shifts(2, 0, 8)
    x0 = np.zeros(A.n)
    seg = oplcg.alg1(A, b, x0, 2, sig, 1e-8 * np.linalg.norm(b), 1000)
    seg_id = oplcg.alg1(A, b, x0, 2, sig, 1e-8 * np.linalg.norm(b), 1000, store=lambda v: v)
    assert seg.t_done == seg_id.t_done and np.array_equal(seg.x, seg_id.x)


@pytest.mark.parametrize("inner_tol", [1e-3, 1e-5])
def test_refinement_matches_fp64_accuracy(inner_tol):
    A, b = _problem((24, 24, 24), seed=3)
    sig = shifts.chebyshev_shifts(3, 0, 12)
    r64 = oplcg.plcg(A, b, np.zeros(A.n), 3, sig, 1e-10, 5000)
    rm = refine.refine(A, b, np.zeros(A.n), 3, sig, 1e-10, inner_tol, 20000)
    assert rm.true_relres < 1e-10 and r64.true_relres < 1e-9
    lmin, lmax = operators.laplacian_extremes((24, 24, 24))
    assert np.linalg.norm(rm.x - r64.x) <= (lmax / lmin) * 2e-10 * np.linalg.norm(r64.x)


def test_last_correction_is_not_oversolved():
    """With the inner stop floored at tol ||r_0|| / 2 the refinement ends just
    below tol instead of inner_tol times below the previous residual, in fewer
    inner iterations; without the floor it overshoots by orders of magnitude."""
    A, b = _problem((24, 24, 24), seed=3)
    sig = shifts.chebyshev_shifts(3, 0, 12)
    tol = 1e-10
    floored = refine.refine(A, b, np.zeros(A.n), 3, sig, tol, 1e-4, 20000)
    plain = refine.refine(A, b, np.zeros(A.n), 3, sig, tol, 1e-4, 20000, final_factor=None)
    assert floored.reason == plain.reason == "converged"
    assert 1e-3 * tol < floored.true_relres < tol
    assert plain.true_relres < 0.1 * floored.true_relres
    assert floored.inner_iters < plain.inner_iters
