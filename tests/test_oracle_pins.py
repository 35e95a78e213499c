"""Pins of the oracle against facts fixed by the paper and by mathematics.

None of these compares the oracle with itself: each checks a closed form, a
library routine, an exact-arithmetic identity (p(l)-CG iterates equal CG
iterates, Sec. 2.1 via the D-Lanczos derivation), an invariant of the bases
(Z = V G, V orthonormal, G symmetric about its l-th upper diagonal), or a count
printed in Table 1.  test_oracle_mutations.py shows that plausible mistakes in
the oracle's steps fail these pins.
"""
import json
import math
import os

import mpmath
import numpy as np
import pytest
import scipy.linalg
import scipy.sparse
import scipy.sparse.linalg

import synth
from oracle import cg as ocg
from oracle import operators, shifts
from oracle import plcg as oplcg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- shifts ----

@pytest.mark.parametrize("l,lo,hi,expect", [
    (1, 0, 8, [4.0]),
    (2, 0, 8, [4 + 2 * math.sqrt(2), 4 - 2 * math.sqrt(2)]),
    (3, 0, 8, [4 + 2 * math.sqrt(3), 4.0, 4 - 2 * math.sqrt(3)]),
    (3, 0, 12, [6 + 3 * math.sqrt(3), 6.0, 6 - 3 * math.sqrt(3)]),
    (2, 0, 2, [1 + math.sqrt(2) / 2, 1 - math.sqrt(2) / 2]),
])
def test_shifts_closed_form(l, lo, hi, expect):
    got = shifts.chebyshev_shifts(l, lo, hi)
    assert np.allclose(got, expect, rtol=0, atol=1e-14)


@pytest.mark.parametrize("l", [1, 2, 3, 4, 5, 8])
def test_shifts_are_mapped_chebyshev_roots(l):
    # numpy's Chebyshev-series root finder on T_l, mapped to [lo, hi].
    lo, hi = 0.3, 7.7
    coef = np.zeros(l + 1)
    coef[l] = 1.0
    roots = np.polynomial.chebyshev.chebroots(coef).real
    mapped = np.sort(0.5 * (hi + lo) + 0.5 * (hi - lo) * roots)
    got = shifts.chebyshev_shifts(l, lo, hi)
    assert np.allclose(np.sort(got), mapped, atol=1e-12)
    assert all(got[i] > got[i + 1] for i in range(l - 1))   # sigma_0 is the largest


# ------------------------------------------------------------- operators ----

def _scipy_laplacian(dims):
    mats = []
    for n in dims:
        mats.append(scipy.sparse.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)],
                                       [-1, 0, 1]))
    A = None
    # Kronecker sum; x (dims[0]) is the fastest index.
    for ax, T in enumerate(mats):
        term = T
        for n in dims[:ax]:
            term = scipy.sparse.kron(term, scipy.sparse.identity(n))
        for n in dims[ax + 1:]:
            term = scipy.sparse.kron(scipy.sparse.identity(n), term)
        A = term if A is None else A + term
    return A.toarray()


@pytest.mark.parametrize("dims", [(5, 7), (1, 9), (6, 1), (4, 3, 5), (1, 1, 1), (3, 1, 2)])
def test_operator_matches_kronecker_sum(dims):
    A = operators.laplacian(dims)
    M = operators.assemble(A)
    assert np.array_equal(M, _scipy_laplacian(dims))


@pytest.mark.parametrize("dims,ks", [((64, 64), (1, 1)), ((64, 64), (17, 40)),
                                     ((33, 20), (3, 19)), ((12, 9, 7), (1, 5, 7))])
def test_operator_eigenpairs_closed_form(dims, ks):
    A = operators.laplacian(dims)
    v = operators.laplacian_mode(dims, ks)
    lam = sum(4 * math.sin(k * math.pi / (2 * (n + 1))) ** 2 for n, k in zip(dims, ks))
    # rounding of A v is relative to ||A|| ||v|| (||A|| < 4 * dimension)
    assert np.linalg.norm(A(v) - lam * v) <= 1e-14 * 4 * len(dims) * np.linalg.norm(v)


@pytest.mark.parametrize("dims", [(16, 16), (9, 5), (5, 4, 3)])
def test_spectrum_closed_form_vs_eigvalsh(dims):
    M = operators.assemble(operators.laplacian(dims))
    ev = scipy.linalg.eigvalsh(M)
    assert np.allclose(ev, operators.laplacian_eigenvalues(dims), atol=1e-12)
    lmin, lmax = operators.laplacian_extremes(dims)
    assert abs(ev[0] - lmin) < 1e-12 and abs(ev[-1] - lmax) < 1e-12


def test_spectral_bounds_configs():
    # 2D n: lmin = 8 sin^2(pi/(2(n+1))), lmax = 8 cos^2(pi/(2(n+1))); all inside [0, 8].
    lmin, lmax = operators.laplacian_extremes((64, 64))
    assert abs(lmin - 8 * math.sin(math.pi / 130) ** 2) < 1e-15
    assert 0 < lmin < lmax < 8
    lmin3, lmax3 = operators.laplacian_extremes((256, 256, 256))
    assert 0 < lmin3 < lmax3 < 12


# ---------------------------------------------------------------------- CG --

def _dense_spd(n, seed=0, lo=1.0, hi=10.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return Q @ np.diag(np.linspace(lo, hi, n)) @ Q.T


@pytest.mark.parametrize("n", [8, 16])
def test_cg_finite_termination(n):
    M = _dense_spd(n)
    b = synth.uniform(n, 11)
    r = ocg.cg(operators.dense(M), b, np.zeros(n), 1e-13, 10 * n)
    assert r.reason == "converged" and r.iters <= n
    assert r.true_relres < 1e-12


def test_cg_iterates_match_scipy():
    A = operators.laplacian((20, 20))
    M = scipy.sparse.csr_matrix(_scipy_laplacian((20, 20)))
    b = synth.uniform(400, 2)
    ours = ocg.cg(A, b, np.zeros(400), 1e-30, 12, record_iterates=True)
    theirs = []
    scipy.sparse.linalg.cg(M, b, x0=np.zeros(400), rtol=1e-30, maxiter=12,
                           callback=lambda xk: theirs.append(xk.copy()))
    assert len(theirs) == 12
    for a, c in zip(ours.iterates, theirs):
        assert np.linalg.norm(a - c) <= 1e-12 * np.linalg.norm(c)


# --------------------------------------------------------------- p(l)-CG --

def _poisson_manufactured(dims, seed=0):
    A = operators.laplacian(dims)
    xs = synth.uniform(A.n, seed)
    return A, xs, A(xs)


@pytest.mark.parametrize("l", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("dots", ["symmetric", "full"])
def test_plcg_early_iterates_equal_cg(l, dots):
    """x_t of p(l)-CG is the CG iterate x_t (D-Lanczos, Sec. 2.1): fp64 agreement."""
    A, xs, b = _poisson_manufactured((32, 32), seed=4)
    x0 = np.zeros(A.n)
    ref = ocg.cg(A, b, x0, 1e-30, 8, record_iterates=True)
    sig = shifts.chebyshev_shifts(l, 0.0, 8.0)
    for t in (1, 2, 3, 5, 8):
        r = oplcg.plcg(A, b, x0, l, sig, 1e-30, t, dots=dots)
        assert r.iters == t
        assert np.linalg.norm(r.x - ref.iterates[t - 1]) <= 1e-13 * np.linalg.norm(ref.iterates[t - 1])


@pytest.mark.parametrize("l", [1, 2, 3, 5])
def test_plcg_equals_cg_in_50_digit_arithmetic(l):
    """Same identity at 50 significant digits: any wrong term shows at O(1)."""
    mpmath.mp.dps = 50
    try:
        A = operators.laplacian((7, 5))
        n = A.n
        b = np.array([mpmath.mpf(float(v)) for v in synth.uniform(n, 3)], dtype=object)
        x0 = np.array([mpmath.mpf(0)] * n, dtype=object)
        ref = ocg.cg(A, b, x0, mpmath.mpf("1e-45"), 7, record_iterates=True)
        sig = [mpmath.mpf(4) + 4 * mpmath.cos((2 * i + 1) * mpmath.pi / (2 * l)) for i in range(l)]
        for t in (1, 3, 7):
            r = oplcg.plcg(A, b, x0, l, sig, mpmath.mpf("1e-48"), t)
            d = r.x - ref.iterates[t - 1]
            err = mpmath.sqrt(sum(v * v for v in d))
            scale = mpmath.sqrt(sum(v * v for v in ref.iterates[t - 1]))
            assert err <= mpmath.mpf("1e-40") * scale
    finally:
        mpmath.mp.dps = 15


@pytest.mark.parametrize("l", [1, 2, 3, 4, 5])
def test_plcg_iteration_count_equals_cg_64(l):
    """64x64 manufactured workload: same iteration count as CG, residuals agree."""
    A, xs, b = _poisson_manufactured((64, 64), seed=0)
    x0 = np.zeros(A.n)
    ref = ocg.cg(A, b, x0, 1e-8, 2000)
    r = oplcg.plcg(A, b, x0, l, shifts.chebyshev_shifts(l, 0.0, 8.0), 1e-8, 2000)
    assert r.reason == "converged" and r.restarts == 0
    assert abs(r.iters - ref.iters) <= 1
    # recursive |zeta_t| equals the true residual norm in exact arithmetic
    assert 0.1 < r.rec_relres / r.true_relres < 10
    assert r.true_relres < 1e-8 * 10
    # manufactured solution: ||x - x*|| / ||x*|| <= kappa * relres
    lmin, lmax = operators.laplacian_extremes((64, 64))
    err = np.linalg.norm(r.x - xs) / np.linalg.norm(xs)
    assert err <= (lmax / lmin) * r.true_relres
    assert np.linalg.norm(r.x - ref.x) <= 1e-12 * np.linalg.norm(ref.x)


@pytest.mark.parametrize("l", [1, 2, 3])
def test_full_history_invariants(l):
    """Z^{(0)} = V orthonormal, Z^{(l)} = V G, G banded and symmetric about its l-th
    upper diagonal (Eq. symmetry_G), T = V^T A V (Eq. v_ex), A-orthogonal search
    directions with p_j^T A p_j = 1/eta_j (from P = V U^{-1}, Eq. x_a)."""
    A, xs, b = _poisson_manufactured((12, 10), seed=7)
    x0 = np.zeros(A.n)
    sig = shifts.chebyshev_shifts(l, 0.0, 8.0)
    T = 14
    seg = oplcg.alg1(A, b, x0, l, sig, 0.0, T, dots="full", keep_all=True)
    d = seg.diag
    G, z, gam, dlt, eta, P = d["G"], d["z"], d["gam"], d["dlt"], d["eta"], d["P"]
    V = np.array([z[0][j] for j in range(T + 1)]).T
    assert np.abs(V.T @ V - np.eye(T + 1)).max() < 1e-12
    # Z^{(l)} = V G for the columns whose G entries are final
    for c in range(1, T + 1):
        rows = [j for j in range(max(0, c - 2 * l), c + 1)]
        rec = sum(G[j, c] * z[0][j] for j in rows)
        assert np.linalg.norm(rec - z[l][c]) <= 1e-10 * np.linalg.norm(z[l][c])
    # band symmetry g_{j,i} = g_{i-l, j+l}
    for c in range(l + 1, T + 1):
        for j in range(max(0, c - 2 * l), c - l):
            assert abs(G[j, c] - G[c - l, j + l]) <= 1e-10 * abs(G[c - l, c - l] + G[c, c])
    # T entries
    for t in range(T - 1):
        Av = A(z[0][t])
        assert abs(gam[t] - np.dot(Av, z[0][t])) < 1e-11
        assert abs(dlt[t] - np.dot(Av, z[0][t + 1])) < 1e-11
    # search directions
    keys = sorted(P)
    for a in keys:
        Apa = A(P[a])
        for c in keys:
            val = np.dot(P[c], Apa)
            if a == c:
                assert abs(val * eta[a] - 1.0) < 1e-11
            else:
                assert abs(val) < 1e-11 * math.sqrt(abs(np.dot(P[a], Apa) * np.dot(P[c], A(P[c]))))


def test_full_and_symmetric_forms_agree():
    A, xs, b = _poisson_manufactured((40, 30), seed=1)
    x0 = np.zeros(A.n)
    for l in (2, 4):
        sig = shifts.chebyshev_shifts(l, 0.0, 8.0)
        a = oplcg.plcg(A, b, x0, l, sig, 1e-8, 3000, dots="full")
        c = oplcg.plcg(A, b, x0, l, sig, 1e-8, 3000, dots="symmetric")
        assert a.iters == c.iters
        assert np.linalg.norm(a.x - c.x) <= 1e-12 * np.linalg.norm(a.x)


def test_scale_invariance():
    """A -> cA with shifts on c[lmin, lmax] gives the same iterates (Eq. chebyshev)."""
    A, xs, b = _poisson_manufactured((24, 24), seed=2)
    A10 = operators.laplacian((24, 24))
    A10 = (lambda f: (lambda u: 10.0 * f(u)))(A10)
    x0 = np.zeros(576)
    r1 = oplcg.plcg(A, b, x0, 2, shifts.chebyshev_shifts(2, 0, 8), 1e-8, 2000)
    r2 = oplcg.plcg(A10, 10.0 * b, x0, 2, shifts.chebyshev_shifts(2, 0, 80), 1e-8, 2000)
    assert r1.iters == r2.iters
    assert np.linalg.norm(r1.x - r2.x) <= 1e-11 * np.linalg.norm(r1.x)


def test_breakdown_restart_converges():
    """Shifts on a too-wide interval break down (Sec. 2.2); the explicit restart
    still reaches the tolerance on the true residual."""
    A = operators.laplacian((64, 64))
    b = synth.uniform(A.n, 1)
    x0 = np.zeros(A.n)
    r = oplcg.plcg(A, b, x0, 2, shifts.chebyshev_shifts(2, 0, 16), 1e-8, 20000)
    assert r.restarts >= 1
    assert r.reason == "converged" and r.true_relres < 1e-7
    # every restart resumes from the last iterate: x-updates of each segment add up
    assert r.iters == sum(s.t_done for s in r.segments)


def test_dense_lucky_breakdown_restarts():
    for n in (8, 16):
        M = _dense_spd(n)
        b = synth.uniform(n, 5)
        for l in (1, 2, 3):
            r = oplcg.plcg(operators.dense(M), b, np.zeros(n), l,
                           shifts.chebyshev_shifts(l, 1, 10), 1e-12, 500)
            assert r.reason == "converged" and r.true_relres < 1e-11


def test_zero_rhs_and_converged_start():
    A = operators.laplacian((6, 6))
    z = np.zeros(36)
    r = oplcg.plcg(A, z, z, 2, shifts.chebyshev_shifts(2, 0, 8), 1e-8, 100)
    assert r.iters == 0 and r.reason == "converged"
    xs = synth.uniform(36, 9)
    r = oplcg.plcg(A, A(xs), xs, 2, shifts.chebyshev_shifts(2, 0, 8), 1e-8, 100)
    assert r.iters == 0 and r.reason == "converged"


def test_maxit_stops_at_m():
    A, xs, b = _poisson_manufactured((16, 16))
    r = oplcg.plcg(A, b, np.zeros(256), 3, shifts.chebyshev_shifts(3, 0, 8), 1e-12, 9)
    assert r.iters == 9 and r.reason == "maxit"


@pytest.mark.parametrize("l", [1, 2, 3, 4, 5])
def test_table1_counts(l):
    with open(os.path.join(GOLDEN, "table1_costs.json")) as f:
        g = json.load(f)
    A, xs, b = _poisson_manufactured((16, 16))
    sig = shifts.chebyshev_shifts(l, 0, 8)
    m = 30
    for dots, key in (("symmetric", "dots_symmetric"), ("full", "dots_full")):
        seg = oplcg.alg1(A, b, np.zeros(256), l, sig, 0.0, m, dots=dots)
        steady = seg.dots_per_iter[2 * l + 1:]
        want = eval(g["plcg"][key], {"l": l})
        assert set(steady) == {want}
        # one SpMV per loop iteration plus the initial residual
        assert seg.spmvs == 1 + (m + l + 1)
    assert g["plcg"]["spmv"] == 1 and g["plcg"]["glred"] == 1


def test_diagonal_toy_matches_laplacian_count():
    """The diagonal system with the 2D Laplacian's eigenvalues (Sec. 4.2) needs about
    as many iterations as the Laplacian itself."""
    dims = (48, 48)
    lam = operators.laplacian_eigenvalues(dims)
    D = (lambda d: (lambda u: d * u))(lam)
    b = synth.uniform(lam.size, 3)
    ref = ocg.cg(D, b, np.zeros(lam.size), 1e-8, 5000)
    r = oplcg.plcg(D, b, np.zeros(lam.size), 2, shifts.chebyshev_shifts(2, 0, 8), 1e-8, 5000)
    A = operators.laplacian(dims)
    rl = ocg.cg(A, b, np.zeros(lam.size), 1e-8, 5000)
    assert abs(r.iters - ref.iters) <= 1
    assert abs(ref.iters - rl.iters) <= 0.1 * rl.iters


def test_synth_generator_known_values():
    # SplitMix64 reference outputs for seed 0 (published test vector of the generator)
    z = synth.splitmix64(0, 0, 3)
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    u = synth.uniform(1000, 0)
    assert u.min() >= -1 and u.max() < 1 and abs(u.mean()) < 0.1
    assert np.array_equal(synth.uniform(10, 5, start=7), synth.uniform(17, 5)[7:])
