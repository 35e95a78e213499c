"""GPU path (through the C ABI) against the oracle, on the same seeded inputs.

Bar: iteration counts equal (within 1), true relative residual within 10x of
the oracle's, ||x_gpu - x_oracle|| / ||x_oracle|| < 1e-8 (FP64), and, step by
step, early iterates and the recurrence coefficients gamma_t, delta_t, eta_t,
zeta_t within rounding of the oracle's.
"""
import math

import numpy as np
import pytest

import synth
from oracle import cg as ocg
from oracle import operators, shifts
from oracle import plcg as oplcg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _plcg():
    from paper_1905_06850_amd import plcg
    return plcg


def _kind(dims):
    return "2d5" if len(dims) == 2 else "3d7"


def _interval(dims):
    return (0.0, 8.0) if len(dims) == 2 else (0.0, 12.0)


LAUNCHES = ["streaming", "resident"]


def gpu_solve(dev, dims, method, l, b, x0, tol, maxit, launch="auto", **kw):
    """Solve on the GPU; launch "streaming" or "resident" forces that launch mode
    (skipping the case if the library does not offer it for this system) and
    checks that it is the one that ran."""
    plcg = _plcg()
    lo, hi = kw.pop("interval", _interval(dims))
    n = int(np.prod(dims))
    if launch == "resident" and not plcg.resident_supported(_kind(dims), n, method, l):
        pytest.skip(f"no resident kernel for {method} l={l} n={n}")
    print(f"[gpu] {method} l={l} dims={dims} tol={tol} maxit={maxit} launch={launch}",
          flush=True)
    s = plcg.Solver(_kind(dims), dims, method=method, l=l, lmin=lo, lmax=hi, launch=launch, **kw)
    bt = torch.from_numpy(np.ascontiguousarray(b)).to(dev)
    xt = torch.from_numpy(np.ascontiguousarray(x0)).to(dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    res = s.solve(bt.data_ptr(), xt.data_ptr(), tol, maxit, stream)
    if launch != "auto" and (res.iters > 0 or res.restarts > 0):
        assert res.launch_mode == plcg.LAUNCH_MODES[launch], res.as_dict()
    x = xt.cpu().numpy()
    return x, res, s


def oracle_solve(dims, method, l, b, x0, tol, maxit, interval=None, max_restarts=100):
    A = operators.laplacian(dims)
    if method == "cg":
        return ocg.cg(A, b, x0, tol, maxit)
    lo, hi = interval or _interval(dims)
    return oplcg.plcg(A, b, x0, l, shifts.chebyshev_shifts(l, lo, hi), tol, maxit,
                      max_restarts=max_restarts)


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


METHODS = [("cg", 1), ("plcg", 1), ("plcg", 2), ("plcg", 3), ("plcg", 4), ("plcg", 5)]


# ----------------------------------------------------------------- operator --

@pytest.mark.parametrize("dims", [(64, 64), (100, 37), (1, 513), (513, 1), (3, 3), (1, 1),
                                  (2048, 3), (20, 13, 7), (1, 1, 5), (33, 1, 2), (16, 16, 16),
                                  (1, 7, 1)])
def test_apply_matches_oracle(dev, dims):
    plcg = _plcg()
    A = operators.laplacian(dims)
    x = synth.uniform(A.n, 21)
    s = plcg.Solver(_kind(dims), dims, method="cg")
    xt = torch.from_numpy(x).to(dev)
    yt = torch.empty_like(xt)
    s.apply(xt.data_ptr(), yt.data_ptr(), torch.cuda.current_stream(dev).cuda_stream)
    y = yt.cpu().numpy()
    # same five or seven terms; only the summation order may differ
    assert np.abs(y - A(x)).max() <= 8 * np.finfo(float).eps * 2 * len(dims) * 2
    s.close()


def test_shifts_match_oracle(dev):
    plcg = _plcg()
    for l in range(1, 9):
        s = plcg.Solver("2d5", (8, 8), method="plcg", l=l, lmin=0.0, lmax=8.0)
        assert s.shifts() == shifts.chebyshev_shifts(l, 0.0, 8.0)
        s.close()


# --------------------------------------------------------------- full solves --

@pytest.mark.parametrize("launch", LAUNCHES)
@pytest.mark.parametrize("method,l", METHODS)
def test_solve_parity_64_manufactured(dev, method, l, launch):
    dims = (64, 64)
    A = operators.laplacian(dims)
    xs = synth.uniform(A.n, 0)
    b = A(xs)
    x0 = np.zeros(A.n)
    ref = oracle_solve(dims, method, l, b, x0, 1e-8, 5000)
    x, res, s = gpu_solve(dev, dims, method, l, b, x0, 1e-8, 5000, launch=launch)
    assert res.reason == 1, res.as_dict()
    assert abs(res.iters - ref.iters) <= 1
    assert res.true_relres <= 10 * ref.true_relres and ref.true_relres <= 10 * res.true_relres
    assert res.rec_relres <= 10 * ref.rec_relres
    assert _rel(x, ref.x) < 1e-8
    s.close()


# (32, 48, 5) and (64, 160, 6): planes of whole chunks, visited by column tiles
@pytest.mark.parametrize("dims,launch", [((64, 64), "streaming"), ((30, 32), "resident")])
@pytest.mark.parametrize("l", [6, 7, 8])
def test_deep_pipelines_solve_parity(dev, l, dims, launch):
    """The deepest pipelines the library offers, solved through at 64^2 with
    the streaming kernels and at 30 x 32 (one unknown per thread) resident."""
    A = operators.laplacian(dims)
    b = A(synth.uniform(A.n, 0))
    x0 = np.zeros(A.n)
    ref = oracle_solve(dims, "plcg", l, b, x0, 1e-8, 5000)
    x, res, s = gpu_solve(dev, dims, "plcg", l, b, x0, 1e-8, 5000, launch=launch)
    assert res.reason == 1 and ref.reason == "converged"
    assert abs(res.iters - ref.iters) <= 1 and res.restarts == ref.restarts == 0
    assert _rel(x, ref.x) < 1e-8
    s.close()


@pytest.mark.parametrize("dims", [(100, 37), (37, 100), (1, 700), (700, 1), (20, 13, 7),
                                  (5, 9, 11), (1, 1, 600), (32, 48, 5), (64, 160, 6),
                                  (102, 30)])
@pytest.mark.parametrize("method,l", [("cg", 1), ("plcg", 1), ("plcg", 2), ("plcg", 3)])
@pytest.mark.parametrize("launch", LAUNCHES)
def test_solve_parity_ragged(dev, dims, method, l, launch):
    A = operators.laplacian(dims)
    b = synth.uniform(A.n, 3)
    x0 = 0.1 * synth.uniform(A.n, 4)
    ref = oracle_solve(dims, method, l, b, x0, 1e-8, 5000)
    x, res, s = gpu_solve(dev, dims, method, l, b, x0, 1e-8, 5000, launch=launch)
    assert res.reason == 1 and ref.reason == "converged"
    assert abs(res.iters - ref.iters) <= 1
    assert res.true_relres <= 10 * max(ref.true_relres, 1e-15)
    assert _rel(x, ref.x) < 1e-8
    s.close()


@pytest.mark.parametrize("launch,x_update", [("streaming", "every"), ("streaming", "paired"),
                                             ("resident", "auto")])
@pytest.mark.parametrize("method,l", METHODS)
def test_early_iterates(dev, method, l, launch, x_update):
    """x after exactly m steps against the oracle's x_m.  Odd and even m; with
    x_update "paired" the streaming p(l)-CG sweeps write x on even t only (two
    steps at once) and add an odd last step after the run."""
    dims = (48, 40)
    A = operators.laplacian(dims)
    b = synth.uniform(A.n, 8)
    x0 = np.zeros(A.n)
    for m in (0, 1, 2, 3, 7, 20):
        ref = oracle_solve(dims, method, l, b, x0, 1e-30, m)
        x, res, s = gpu_solve(dev, dims, method, l, b, x0, 1e-30, m, launch=launch,
                              x_update=x_update)
        assert res.iters == m == ref.iters
        assert res.reason == 2
        assert m == 0 or res.x_update_every == (2 if x_update == "paired" else 1)
        if m == 0:
            assert np.array_equal(x, x0)
        else:
            assert _rel(x, ref.x) < 1e-13
        s.close()


@pytest.mark.parametrize("method,dims,l,precision,interval", [
    ("plcg", (64, 64), 1, "fp64", None), ("plcg", (100, 37), 2, "fp64", None),
    ("plcg", (20, 13, 7), 3, "fp64", None), ("plcg", (64, 64), 5, "fp64", None),
    ("plcg", (48, 48), 3, "fp64", (6.0, 8.0)), ("plcg", (96, 80), 1, "fp32", None),
    ("plcg", (60, 50), 2, "fp32", None), ("cg", (64, 64), 1, "fp64", None),
    ("cg", (100, 37), 1, "fp64", None), ("cg", (20, 13, 7), 1, "fp64", None),
    ("cg", (64, 160, 6), 1, "fp64", None)])
def test_paired_x_updates_bitwise_equal(dev, method, dims, l, precision, interval):
    """PLCG_X_PAIRED (x written every second iteration, two steps with the same
    two roundings) against PLCG_X_EVERY: x, iteration and restart counts and both
    residuals bit for bit equal, for runs that stop after an odd and an even
    number of steps and runs to convergence (the (6, 8) interval on 48^2
    breaks down and restarts; fp32: FP32-stored inner solves in refinement;
    CG: its sweep B, with p_{k-1} in its second p buffer)."""
    n = int(np.prod(dims))
    b = synth.uniform(n, 5)
    x0 = np.zeros(n)
    kw = {"precision": precision, "inner_tol": 1e-4 if precision == "fp32" else 0.0}
    if interval is not None:
        kw["interval"] = interval
    for tol, maxit in ((1e-30, 7), (1e-30, 8), (1e-9, 100000)):
        out = []
        for xu in ("every", "paired"):
            x, res, s = gpu_solve(dev, dims, method, l, b, x0, tol, maxit, launch="streaming",
                                  x_update=xu, **dict(kw))
            s.close()
            assert res.x_update_every == (2 if xu == "paired" else 1)
            out.append((x, res))
        (xe, re_), (xp, rp) = out
        assert np.array_equal(xe.view(np.uint64), xp.view(np.uint64))
        assert (re_.iters, re_.restarts, re_.outer, re_.reason) == \
            (rp.iters, rp.restarts, rp.outer, rp.reason)
        assert re_.rec_relres == rp.rec_relres and re_.true_relres == rp.true_relres
    if interval is not None:
        assert re_.restarts > 0


@pytest.mark.parametrize("l", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("x_update,precision", [("every", "fp64"), ("paired", "fp64"),
                                                ("paired", "fp32")])
def test_stop_near_end_of_check_group(dev, l, x_update, precision):
    """The host checks the device status after every `check_every` launches and
    stops enqueueing once a stop is published; x_t is complete only after sweep
    t + l, which may not have been enqueued by then.  With check_every = 1, 2, 3
    the stop lands in the last launches of a group: x, counts and residuals must
    be bit for bit those of check_every = 64 (convergence, and the breakdown +
    restart of a too-narrow interval), and x must match the oracle."""
    cases = [((128, 128), None, 1e-9)]
    if precision == "fp64" and l in (2, 3):
        cases.append(((64, 64), (0.0, 16.0), 1e-8) if l == 2 else ((48, 48), (6.0, 8.0), 1e-9))
    for dims, interval, tol in cases:
        n = int(np.prod(dims))
        b = synth.uniform(n, 31)
        x0 = np.zeros(n)
        kw = {"precision": precision, "inner_tol": 1e-4 if precision == "fp32" else 0.0,
              "x_update": x_update}
        if interval is not None:
            kw["interval"] = interval
        runs = {}
        for ce in (64, 1, 2, 3):
            x, res, s = gpu_solve(dev, dims, "plcg", l, b, x0, tol, 100000, launch="streaming",
                                  check_every=ce, **dict(kw))
            s.close()
            runs[ce] = (x, res)
        xr, rr = runs[64]
        assert rr.reason == 1, rr.as_dict()
        for ce in (1, 2, 3):
            x, res = runs[ce]
            assert np.array_equal(x.view(np.uint64), xr.view(np.uint64)), (ce, res.as_dict())
            assert (res.iters, res.restarts, res.outer, res.reason, res.spmvs) == \
                (rr.iters, rr.restarts, rr.outer, rr.reason, rr.spmvs)
            assert res.rec_relres == rr.rec_relres and res.true_relres == rr.true_relres
        if precision == "fp64" and interval is None:
            ref = oracle_solve(dims, "plcg", l, b, x0, tol, 100000)
            assert abs(rr.iters - ref.iters) <= 1 and rr.restarts == ref.restarts == 0
            assert _rel(xr, ref.x) < 1e-8
        if interval is not None:
            # restarts: the count depends on rounding; the solve must still reach tol
            assert rr.restarts > 0 and rr.true_relres < 10 * tol


@pytest.mark.parametrize("dims", [(64, 64, 256), (32, 48, 1100)])
def test_cg_3d_zmarch_iterates(dev, dims):
    """3D CG whose sweep A marches tiles through several planes (2 and 3 planes
    per workgroup here; the second grid ends with a shorter segment): early
    iterates against the oracle to rounding, and (64, 64, 256) solved through."""
    A = operators.laplacian(dims)
    b = synth.uniform(A.n, 12)
    x0 = np.zeros(A.n)
    for m in (1, 2, 5, 20):
        ref = oracle_solve(dims, "cg", 1, b, x0, 1e-30, m)
        x, res, s = gpu_solve(dev, dims, "cg", 1, b, x0, 1e-30, m)
        assert res.iters == m == ref.iters
        assert _rel(x, ref.x) < 1e-13
        s.close()
    if dims == (64, 64, 256):
        ref = oracle_solve(dims, "cg", 1, b, x0, 1e-8, 5000)
        x, res, s = gpu_solve(dev, dims, "cg", 1, b, x0, 1e-8, 5000)
        assert res.reason == 1 and abs(res.iters - ref.iters) <= 1
        assert _rel(x, ref.x) < 1e-8
        s.close()


def _fsum_dot(a, b):
    return math.fsum(a * b)


@pytest.mark.parametrize("launch", LAUNCHES)
@pytest.mark.parametrize("l", [1, 2, 3, 4, 5, 8])
def test_coefficients_match_oracle(dev, l, launch):
    """gamma_t, delta_t (Eqs. haa1, haa3), eta_t, zeta_t (Eq. LU) from the device
    scalar engine against the oracle's, t = 0..149.  The bound is ten times the
    oracle's own change when its dot products are rounded correctly instead of
    summed by BLAS (deep pipelines amplify local rounding, Sec. 2.2), and at
    least 1e-10."""
    dims = (64, 64)
    A = operators.laplacian(dims)
    b = synth.uniform(A.n, 5)
    x0 = np.zeros(A.n)
    sig = shifts.chebyshev_shifts(l, 0.0, 8.0)
    d = oplcg.alg1(A, b, x0, l, sig, 0.0, 150).diag
    d2 = oplcg.alg1(A, b, x0, l, sig, 0.0, 150, dot=_fsum_dot).diag
    x, res, s = gpu_solve(dev, dims, "plcg", l, b, x0, 1e-30, 150, history_cap=200,
                          launch=launch)
    hist = s.history(200)
    assert len(hist) >= 150
    for col, key in enumerate(("gam", "dlt", "eta", "zeta")):
        spread = max(abs(d[key][t] - d2[key][t]) / abs(d[key][t]) for t in range(150))
        dev_gpu = max(abs(hist[t][col] - d[key][t]) / abs(d[key][t]) for t in range(150))
        print(f"l={l} {key}: gpu deviation {dev_gpu:.2e}, oracle order spread {spread:.2e}")
        assert dev_gpu <= max(1e-10, 10 * spread)
    s.close()


# --------------------------------------------------------------- edge cases --

@pytest.mark.parametrize("launch", LAUNCHES)
@pytest.mark.parametrize("method,l", [("cg", 1), ("plcg", 2)])
def test_zero_rhs_and_tol_above_one(dev, method, l, launch):
    dims = (10, 10)
    z = np.zeros(100)
    x, res, s = gpu_solve(dev, dims, method, l, z, z, 1e-8, 100, launch=launch)
    assert res.iters == 0 and res.reason == 1 and np.all(x == 0)
    s.close()
    b = synth.uniform(100, 1)
    x, res, s = gpu_solve(dev, dims, method, l, b, z, 2.0, 100, launch=launch)
    assert res.iters == 0 and res.reason == 1
    s.close()


@pytest.mark.parametrize("method,l", [("cg", 1), ("plcg", 1), ("plcg", 3)])
def test_nonfinite_rhs(dev, method, l):
    plcg = _plcg()
    b = synth.uniform(64, 2)
    b[17] = np.nan
    with pytest.raises(plcg.PlcgError) as ei:
        gpu_solve(dev, (8, 8), method, l, b, np.zeros(64), 1e-8, 100)
    assert ei.value.status == plcg.PLCG_E_NONFINITE


@pytest.mark.parametrize("launch", LAUNCHES)
def test_breakdown_and_restart(dev, launch):
    """Shifts on a too-wide interval make the square root break down (Sec. 2.2);
    the library restarts from the latest iterate and still converges."""
    dims = (64, 64)
    A = operators.laplacian(dims)
    b = synth.uniform(A.n, 1)
    x0 = np.zeros(A.n)
    ref = oracle_solve(dims, "plcg", 2, b, x0, 1e-8, 20000, interval=(0.0, 16.0))
    x, res, s = gpu_solve(dev, dims, "plcg", 2, b, x0, 1e-8, 20000, interval=(0.0, 16.0),
                          launch=launch)
    assert ref.restarts >= 1 and res.restarts >= 1
    assert res.reason == 1
    assert res.true_relres < 1e-7
    assert abs(res.iters - ref.iters) <= 0.25 * ref.iters
    s.close()


@pytest.mark.parametrize("launch", LAUNCHES)
def test_single_unknown_breakdown_limit(dev, launch):
    """n = 1: the Krylov space is exhausted before x_1 is formed, so every
    segment breaks down at t = 0; both sides stop at the restart limit."""
    b = np.array([1.0])
    ref = oracle_solve((1, 1), "plcg", 1, b, np.zeros(1), 1e-8, 50, max_restarts=3)
    x, res, s = gpu_solve(dev, (1, 1), "plcg", 1, b, np.zeros(1), 1e-8, 50, max_restarts=3,
                          launch=launch)
    assert ref.reason == "breakdown_limit" and res.reason == 3
    assert res.restarts == ref.restarts == 4
    s.close()


def test_deterministic_and_submit_poll(dev):
    dims = (96, 80)
    A = operators.laplacian(dims)
    b = synth.uniform(A.n, 6)
    x1, r1, s = gpu_solve(dev, dims, "plcg", 3, b, np.zeros(A.n), 1e-9, 5000)
    bt = torch.from_numpy(b).to(dev)
    xt = torch.zeros(A.n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    r2 = s.solve(bt.data_ptr(), xt.data_ptr(), 1e-9, 5000, stream)
    assert np.array_equal(x1, xt.cpu().numpy()) and r1.iters == r2.iters
    xt.zero_()
    torch.cuda.synchronize()
    ticket = s.submit(bt.data_ptr(), xt.data_ptr(), 1e-9, 5000, stream)
    import time
    t0 = time.time()
    r3 = None
    while r3 is None and time.time() - t0 < 60:
        r3 = s.poll(ticket)
        time.sleep(0.001)
    assert r3 is not None and r3.iters == r1.iters
    assert np.array_equal(x1, xt.cpu().numpy())
    s.close()


@pytest.mark.parametrize("method,l,dims,launch", [("plcg", 2, (96, 80), "streaming"),
                                                  ("cg", 1, (96, 80), "streaming"),
                                                  ("plcg", 3, (64, 64, 80), "streaming"),
                                                  ("plcg", 2, (64, 64), "resident"),
                                                  ("cg", 1, (64, 64), "resident")])
def test_bitwise_reproducible_10_replays(dev, method, l, dims, launch):
    """Ten solves of the same system give the same bits (every reduction is a
    fixed-order sum; no atomics on values)."""
    plcg = _plcg()
    n = int(np.prod(dims))
    b = synth.uniform(n, 41)
    s = plcg.Solver(_kind(dims), dims, method=method, l=l, lmin=0.0,
                    lmax=8.0 if len(dims) == 2 else 12.0, launch=launch)
    bt = torch.from_numpy(b).to(dev)
    xt = torch.zeros(n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    first = None
    for rep in range(10):
        xt.zero_()
        r = s.solve(bt, xt, 1e-9, 20000, stream)
        assert r.reason == 1
        x = xt.cpu().numpy()
        if first is None:
            first = (r.iters, r.rec_relres, x)
        else:
            assert (r.iters, r.rec_relres) == first[:2] and np.array_equal(x, first[2]), rep
    s.close()


def test_timing_counts_sweeps(dev):
    dims = (64, 64)
    b = synth.uniform(4096, 2)
    plcg = _plcg()
    for method, l, per in (("plcg", 2, 1), ("cg", 1, 2)):
        s = plcg.Solver("2d5", dims, method=method, l=l, launch="streaming")
        s.set_timing(True)
        bt = torch.from_numpy(b).to(dev)
        xt = torch.zeros(4096, dtype=torch.float64, device=dev)
        r = s.solve(bt.data_ptr(), xt.data_ptr(), 1e-8, 5000,
                    torch.cuda.current_stream(dev).cuda_stream)
        # Launches that did work: for p(l)-CG every sweep of the segment
        # (iters + l + 1; spmvs also counts the two residuals), for CG sweeps A
        # and B of each iteration.  Timed in groups of 64 iterations; only the
        # groups in which every launch did work are summed.
        assert r.restarts == 0 and r.sweep_ms > 0
        work = r.spmvs - 2 if method == "plcg" else per * r.iters
        group = 64 * per
        assert work >= group
        assert r.sweeps == group * (work // group)
        # the host waits about once per group of 64 iterations, plus setup and end
        assert 1 <= r.host_waits <= work // group + 6
        s.close()


@pytest.mark.parametrize("launch", LAUNCHES)
@pytest.mark.parametrize("dims", [(2, 2), (3, 1, 1), (2, 1), (1, 1)])
@pytest.mark.parametrize("l", [1, 2, 3])
def test_tiny_systems_krylov_exhaustion(dev, dims, l, launch):
    """Systems with fewer distinct eigenvalues than the pipeline needs break down
    when the Krylov space is exhausted (Sec. 2.2).  Whether the square-root
    argument comes out as exactly zero or as a tiny positive number is decided by
    rounding, so either outcome is valid: converged with an accurate x, or the
    restart limit with x finite.  For n = 1 the argument is exactly zero and both
    sides must stop at the limit."""
    A = operators.laplacian(dims)
    b = synth.uniform(A.n, 3)
    x0 = 0.1 * synth.uniform(A.n, 4)
    ref = oracle_solve(dims, "plcg", l, b, x0, 1e-8, 500, max_restarts=20)
    x, res, s = gpu_solve(dev, dims, "plcg", l, b, x0, 1e-8, 500, max_restarts=20,
                          launch=launch)
    assert res.reason in (1, 3)
    assert np.all(np.isfinite(x))
    if res.reason == 1:
        assert res.true_relres < 1e-7
    else:
        assert res.restarts == 21
    if A.n == 1:
        assert ref.reason == "breakdown_limit" and res.reason == 3
    s.close()


# ------------------------------------------------------------ full-size cases --

def _dense_error(x, g, dims):
    """Relative error of x on the stored dense sample (whole grid rows at the
    seams of a split into eighths, synth.dense_sample_indices), or None when the
    stored result has none."""
    import os
    if "dense_file" not in g:
        return None
    path = os.path.join(os.path.dirname(__file__), "golden", g["dense_file"])
    if not os.path.exists(path):
        return None
    ref = np.load(path, allow_pickle=False)
    idx = synth.dense_sample_indices(dims)
    assert ref.shape == idx.shape
    return np.linalg.norm(x[idx] - ref) / np.linalg.norm(ref)


def _golden(name):
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name + ".json")
    if not os.path.exists(path):
        pytest.skip(f"no stored oracle result {name}")
    with open(path) as f:
        return json.load(f)


@pytest.mark.parametrize("name", ["poisson2048_cg", "poisson2048_p1", "poisson2048_p2",
                                  "poisson2048_p3", "poisson2048_p4", "poisson2048_p5",
                                  "poisson3d256_p1", "poisson3d256_p3", "poisson3d256_cg"])
def test_full_size_against_stored_oracle(dev, name):
    """The benchmark workloads at full size, in the launch configuration the
    benchmark times, against the oracle's stored result (tests/golden,
    written by make_golden.py from the oracle only): same iteration count within
    1, true residual within 10x, and ||x - x_oracle|| / ||x_oracle|| < 1e-8
    estimated from the stored sample of x and measured on the stored dense sample
    of whole rows at the seams of a split into eighths (plus ||x|| itself)."""
    g = _golden(name)
    dims = tuple(g["dims"])
    n = int(np.prod(dims))
    b = synth.uniform(n, g["seed"])
    method = g["method"]
    l = max(int(g["l"]), 1)
    x, res, s = gpu_solve(dev, dims, method, l, b, np.zeros(n), g["tol"], 100000,
                          interval=tuple(g["interval"]))
    assert res.reason == 1
    assert abs(res.iters - g["iters"]) <= 1
    # x on every second sweep, except p(2) at 2048^2, whose 8 vectors fill the
    # 256 MiB memory-side cache exactly (a second p buffer would not fit)
    assert res.x_update_every == (1 if name == "poisson2048_p2" else 2)
    assert res.true_relres <= 10 * g["true_relres"] and g["true_relres"] <= 10 * res.true_relres
    idx = np.array(g["sample_idx"])
    ref = np.array(g["sample_x"])
    est = np.sqrt(n / idx.size * np.sum((x[idx] - ref) ** 2)) / g["xnorm"]
    assert est < 1e-8
    dense = _dense_error(x, g, dims)
    assert dense is None or dense < 1e-8, dense
    assert abs(np.linalg.norm(x) - g["xnorm"]) <= 1e-8 * g["xnorm"]
    s.close()


# ------------------------------------------------------------ mixed precision --

def _mixed_oracle(dims, l, b, tol, inner_tol, maxit=20000, max_outer=50):
    from oracle import refine
    A = operators.laplacian(dims)
    lo, hi = _interval(dims)
    return refine.refine(A, b, np.zeros(A.n), l, shifts.chebyshev_shifts(l, lo, hi), tol,
                         inner_tol, maxit, max_outer=max_outer)


# FP32 storage: 4 unknowns per thread; (102, 30) takes the per-unknown stencil
# (nx not a multiple of 4), (64, 160, 6) the column-tiled chunk order
@pytest.mark.parametrize("dims,l,tol,inner_tol", [((48, 48, 48), 3, 1e-10, 1e-3),
                                                  ((48, 48, 48), 3, 1e-10, 1e-5),
                                                  ((64, 64), 1, 1e-10, 1e-3),
                                                  ((100, 37), 2, 1e-10, 1e-4),
                                                  ((102, 30), 2, 1e-10, 1e-4),
                                                  ((64, 160, 6), 3, 1e-10, 1e-4),
                                                  ((60, 50), 4, 1e-10, 1e-4),
                                                  ((60, 50), 5, 1e-10, 1e-4)])
def test_mixed_precision_against_oracle(dev, dims, l, tol, inner_tol):
    """FP32-stored inner p(l)-CG inside FP64 refinement against the oracle's
    model of the same arithmetic (oracle.refine): both reach the FP64 tolerance,
    with the same number of refinement steps (within 1) and inner iteration
    counts within 10 %; the solutions agree within kappa times the tolerance."""
    n = int(np.prod(dims))
    b = synth.uniform(n, 0)
    ref = _mixed_oracle(dims, l, b, tol, inner_tol)
    x, res, s = gpu_solve(dev, dims, "plcg", l, b, np.zeros(n), tol, 20000, precision="fp32",
                          inner_tol=inner_tol)
    assert ref.reason == "converged" and res.reason == 1
    assert res.true_relres < tol and ref.true_relres < tol
    assert abs(res.outer - ref.outer) <= 1
    assert abs(res.iters - ref.inner_iters) <= 0.1 * ref.inner_iters + 2
    lmin, lmax = operators.laplacian_extremes(dims)
    assert _rel(x, ref.x) <= (lmax / lmin) * 2 * tol
    s.close()


def test_mixed_precision_first_inner_steps(dev):
    """After a few inner iterations the FP32-stored GPU iterate equals the oracle's
    FP32-stored iterate to FP32 rounding."""
    dims = (40, 30)
    n = 1200
    b = synth.uniform(n, 2)
    for m in (1, 3, 8):
        ref = _mixed_oracle(dims, 2, b, 1e-30, 1e-30, maxit=m, max_outer=1)
        x, res, s = gpu_solve(dev, dims, "plcg", 2, b, np.zeros(n), 1e-30, m, precision="fp32",
                              inner_tol=1e-30)
        assert res.iters == m == ref.inner_iters and res.outer == 1 == ref.outer
        assert _rel(x, ref.x) < 1e-6
        s.close()


def test_full_size_mixed_against_stored_oracle(dev):
    """The 256^3 workload with FP32-stored p(3)-CG in FP64 refinement (inner tol
    1e-4), as the benchmark runs it, against the oracle's stored model of the same
    arithmetic: refinement steps within 1, inner iterations within 10 %, true
    residual below tol, and the sampled x within kappa * 2 * tol of the oracle's."""
    g = _golden("poisson3d256_m3")
    if g.get("final_factor") != 0.5:
        pytest.skip("stored result was written with an earlier refinement stopping rule")
    dims = tuple(g["dims"])
    n = int(np.prod(dims))
    b = synth.uniform(n, g["seed"])
    x, res, s = gpu_solve(dev, dims, "plcg", 3, b, np.zeros(n), g["tol"], 100000,
                          interval=tuple(g["interval"]), precision="fp32",
                          inner_tol=g["inner_tol"])
    assert res.reason == 1 and g["reason"] == "converged"
    assert abs(res.outer - g["outer"]) <= 1
    assert abs(res.iters - g["iters"]) <= 0.1 * g["iters"] + 2
    assert res.true_relres < g["tol"] and g["true_relres"] < g["tol"]
    lmin, lmax = operators.laplacian_extremes(dims)
    idx = np.array(g["sample_idx"])
    ref = np.array(g["sample_x"])
    est = np.sqrt(n / idx.size * np.sum((x[idx] - ref) ** 2)) / g["xnorm"]
    assert est <= (lmax / lmin) * 2 * g["tol"]
    dense = _dense_error(x, g, dims)
    assert dense is None or dense <= (lmax / lmin) * 2 * g["tol"], dense
    s.close()


def test_tensor_arguments(dev):
    """The binding also takes GPU tensors (and torch's current stream by default):
    same result as with device addresses; wrong dtype, device or length refused
    before any call into the library."""
    plcg = _plcg()
    dims = (64, 64)
    b = synth.uniform(4096, 7)
    s = plcg.Solver("2d5", dims, method="plcg", l=2)
    bt = torch.from_numpy(b).to(dev)
    x1 = torch.zeros(4096, dtype=torch.float64, device=dev)
    x2 = torch.zeros(4096, dtype=torch.float64, device=dev)
    r1 = s.solve(bt, x1, 1e-8, 5000)
    r2 = s.solve(bt.data_ptr(), x2.data_ptr(), 1e-8, 5000,
                 torch.cuda.current_stream(dev).cuda_stream)
    assert r1.iters == r2.iters and torch.equal(x1, x2)
    for bad in (bt.float(), bt.cpu(), bt[:100], bt[::2]):
        with pytest.raises(ValueError):
            s.solve(bad, x1, 1e-8, 10)
    s.close()


# ------------------------------------------------------------ resident solves --

@pytest.mark.parametrize("method,l", [("plcg", 2), ("plcg", 1), ("cg", 1)])
def test_resident_timing_and_waits(dev, method, l):
    """A resident solve is one launch per restart segment: the host waits a few
    times per solve, and the timing counts the iteration launches it replaces
    (p(l)-CG: every sweep of the segment; CG: sweeps A and B per iteration)."""
    plcg = _plcg()
    dims = (64, 64)
    b = synth.uniform(4096, 2)
    s = plcg.Solver("2d5", dims, method=method, l=l, launch="resident")
    s.set_timing(True)
    bt = torch.from_numpy(b).to(dev)
    xt = torch.zeros(4096, dtype=torch.float64, device=dev)
    r = s.solve(bt.data_ptr(), xt.data_ptr(), 1e-8, 5000,
                torch.cuda.current_stream(dev).cuda_stream)
    assert r.reason == 1 and r.restarts == 0 and r.launch_mode == plcg.PLCG_LAUNCH_RESIDENT
    assert r.sweeps == (r.spmvs - 2 if method == "plcg" else 2 * r.iters)
    assert r.sweep_ms > 0
    assert 1 <= r.host_waits <= 4
    s.close()


# widths: p(l)-CG spreads n over 960 threads, CG over 1024 (V = 1..5 each)
@pytest.mark.parametrize("dims,method,l", [((30, 32), "plcg", 1), ((31, 31), "plcg", 1),
                                           ((40, 48), "plcg", 2), ((17, 113), "plcg", 2),
                                           ((48, 60), "plcg", 3), ((60, 64), "plcg", 1),
                                           ((60, 80), "plcg", 2), ((32, 32), "cg", 1),
                                           ((25, 41), "cg", 1), ((60, 80), "cg", 1),
                                           ((12, 10, 8), "plcg", 4), ((12, 10, 8), "plcg", 6),
                                           ((19, 11, 23), "cg", 1)])
def test_resident_widths_against_oracle(dev, dims, method, l):
    """Resident solves at the boundaries of the unknowns-per-thread widths
    (960, 961, 1920, 1921, ..., 4800 unknowns) and in 3D, against the oracle.
    The deep 3D case is one whose stop is not decided by rounding: the oracle
    itself moves x by 5e-11 when its dot products are rounded correctly (on
    6 x 7 x 9 with l = 6 it moves by 1.6e-8 and stops one iteration later, so
    no implementation can meet a 1e-8 bar there)."""
    A = operators.laplacian(dims)
    b = synth.uniform(A.n, 31)
    x0 = 0.1 * synth.uniform(A.n, 32)
    ref = oracle_solve(dims, method, l, b, x0, 1e-8, 20000)
    x, res, s = gpu_solve(dev, dims, method, l, b, x0, 1e-8, 20000, launch="resident")
    assert res.reason == 1 and ref.reason == "converged"
    assert abs(res.iters - ref.iters) <= 1
    assert res.true_relres <= 10 * max(ref.true_relres, 1e-15)
    assert _rel(x, ref.x) < 1e-8
    s.close()


def test_resident_limits(dev):
    """Above PLCG_RESIDENT_MAX unknowns, or for a pipeline too deep for the
    registers, AUTO runs the streaming kernels and RESIDENT is refused; a
    resident solve allowed more than 2^20 iterations streams too."""
    plcg = _plcg()
    assert plcg.resident_supported("2d5", 4800, "plcg", 2)
    assert not plcg.resident_supported("2d5", 4801, "plcg", 1)
    assert not plcg.resident_supported("2d5", 4096, "plcg", 3)
    dims = (61, 80)
    A = operators.laplacian(dims)
    b = synth.uniform(A.n, 33)
    x, res, s = gpu_solve(dev, dims, "plcg", 1, b, np.zeros(A.n), 1e-8, 5000)
    assert res.reason == 1 and res.launch_mode == plcg.PLCG_LAUNCH_STREAMING
    s.close()
    with pytest.raises(plcg.PlcgError) as ei:
        plcg.Solver("2d5", dims, method="plcg", l=1, launch="resident")
    assert ei.value.status == plcg.PLCG_E_INVALID
    dims = (64, 64)
    b = synth.uniform(4096, 34)
    x, res, s = gpu_solve(dev, dims, "cg", 1, b, np.zeros(4096), 1e-8, (1 << 20) + 1,
                          launch="auto")
    assert res.reason == 1 and res.launch_mode == plcg.PLCG_LAUNCH_STREAMING
    s.close()


@pytest.mark.parametrize("method,l", [("plcg", 2), ("cg", 1)])
def test_resident_deterministic_and_submit_poll(dev, method, l):
    """Resident solves are bitwise reproducible (fixed reduction order inside the
    workgroup), also through plcg_submit / plcg_poll."""
    dims = (64, 64)
    A = operators.laplacian(dims)
    b = synth.uniform(A.n, 6)
    x1, r1, s = gpu_solve(dev, dims, method, l, b, np.zeros(A.n), 1e-9, 5000, launch="resident")
    bt = torch.from_numpy(b).to(dev)
    xt = torch.zeros(A.n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    r2 = s.solve(bt.data_ptr(), xt.data_ptr(), 1e-9, 5000, stream)
    assert np.array_equal(x1, xt.cpu().numpy()) and r1.iters == r2.iters
    xt.zero_()
    torch.cuda.synchronize()
    ticket = s.submit(bt.data_ptr(), xt.data_ptr(), 1e-9, 5000, stream)
    import time
    t0 = time.time()
    r3 = None
    while r3 is None and time.time() - t0 < 60:
        r3 = s.poll(ticket)
        time.sleep(0.001)
    assert r3 is not None and r3.iters == r1.iters
    assert np.array_equal(x1, xt.cpu().numpy())
    s.close()
