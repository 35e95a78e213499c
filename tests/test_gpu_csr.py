"""General sparse (CSR) operators through the C ABI against the oracle: the
assembled Poisson matrices, variable-coefficient matrices Jacobi-scaled by the
test, FP32-stored inner solves, and invalid matrices."""
import numpy as np
import pytest

import synth
from oracle import cg as ocg
from oracle import operators, refine, shifts
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


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


class Csr:
    """A CSR matrix copied to the device (kept alive while a solver is created)."""

    def __init__(self, dev, rp, ci, va):
        self.n = len(rp) - 1
        self.nnz = len(ci)
        self.t = (torch.from_numpy(np.ascontiguousarray(rp)).to(dev),
                  torch.from_numpy(np.ascontiguousarray(ci)).to(dev),
                  torch.from_numpy(np.ascontiguousarray(va)).to(dev))

    def arg(self):
        return (self.t[0].data_ptr(), self.t[1].data_ptr(), self.t[2].data_ptr(), self.nnz)


LAUNCHES = ["streaming", "resident"]


def gpu_solve(dev, csr, method, l, b, x0, tol, maxit, lo=0.0, hi=8.0, launch="auto", **kw):
    plcg = _plcg()
    if launch == "resident" and (kw.get("precision", "fp64") != "fp64" or
                                 not plcg.resident_supported("csr", csr.n, method, l)):
        pytest.skip(f"no resident kernel for {method} l={l} n={csr.n}")
    print(f"[gpu] csr {method} l={l} n={csr.n} nnz={csr.nnz} tol={tol} maxit={maxit} "
          f"launch={launch}", flush=True)
    s = plcg.Solver("csr", (csr.n,), method=method, l=l, lmin=lo, lmax=hi, csr=csr.arg(),
                    launch=launch, **kw)
    bt = torch.from_numpy(np.ascontiguousarray(b)).to(dev)
    xt = torch.from_numpy(np.ascontiguousarray(x0).copy()).to(dev)
    res = s.solve(bt.data_ptr(), xt.data_ptr(), tol, maxit,
                  torch.cuda.current_stream(dev).cuda_stream)
    if launch != "auto" and res.iters > 0:
        assert res.launch_mode == plcg.LAUNCH_MODES[launch]
    x = xt.cpu().numpy()
    s.close()
    return x, res


def oracle_solve(A, method, l, b, x0, tol, maxit, lo=0.0, hi=8.0):
    if method == "cg":
        return ocg.cg(A, b, x0, tol, maxit)
    return oplcg.plcg(A, b, x0, l, shifts.chebyshev_shifts(l, lo, hi), tol, maxit)


def scaled_variable(dims, seed):
    """D^{-1/2} A D^{-1/2} of a variable-coefficient operator, assembled here."""
    cx, cy, cz = synth.edge_coefficients(dims, seed)
    rp, ci, va = synth.csr_variable_laplacian(dims, cx, cy, cz)
    A, As, dis = operators.variable_laplacian(dims, cx, cy, cz)
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    return (rp, ci, va * dis[rows] * dis[ci]), As


@pytest.mark.parametrize("dims", [(64, 64), (37, 29), (9, 7, 5), (1, 1), (1, 300)])
def test_csr_apply_matches_oracle(dev, dims):
    plcg = _plcg()
    rp, ci, va = synth.csr_variable_laplacian(dims)
    csr = Csr(dev, rp, ci, va)
    s = plcg.Solver("csr", (csr.n,), method="cg", csr=csr.arg())
    x = synth.uniform(csr.n, 71)
    xt = torch.from_numpy(x).to(dev)
    yt = torch.empty_like(xt)
    s.apply(xt.data_ptr(), yt.data_ptr(), torch.cuda.current_stream(dev).cuda_stream)
    ref = operators.laplacian(dims)(x)
    assert np.abs(yt.cpu().numpy() - ref).max() <= 16 * np.finfo(float).eps * 8
    s.close()


@pytest.mark.parametrize("method,l", [("cg", 1), ("plcg", 1), ("plcg", 2), ("plcg", 3),
                                      ("plcg", 5)])
@pytest.mark.parametrize("launch", LAUNCHES)
def test_csr_poisson_solve_parity(dev, method, l, launch):
    dims = (64, 64)
    A = operators.laplacian(dims)
    csr = Csr(dev, *synth.csr_variable_laplacian(dims))
    xs = synth.uniform(A.n, 0)
    b = A(xs)
    x0 = np.zeros(A.n)
    ref = oracle_solve(A, method, l, b, x0, 1e-8, 5000)
    x, res = gpu_solve(dev, csr, method, l, b, x0, 1e-8, 5000, launch=launch)
    assert res.reason == 1 and abs(res.iters - ref.iters) <= 1
    assert res.true_relres <= 10 * ref.true_relres and ref.true_relres <= 10 * res.true_relres
    assert _rel(x, ref.x) < 1e-8


@pytest.mark.parametrize("dims", [(48, 40), (37, 29), (9, 7, 5)])
@pytest.mark.parametrize("method,l", [("cg", 1), ("plcg", 1), ("plcg", 2), ("plcg", 3)])
@pytest.mark.parametrize("launch", LAUNCHES)
def test_csr_scaled_variable_solve_parity(dev, dims, method, l, launch):
    """Jacobi-scaled variable-coefficient matrices (spectrum in (0, 2)): the
    preconditioned method of reading 15 on a general sparse matrix."""
    (rp, ci, va), As = scaled_variable(dims, 72)
    csr = Csr(dev, rp, ci, va)
    b = synth.uniform(As.n, 73)
    x0 = 0.1 * synth.uniform(As.n, 74)
    ref = oracle_solve(As, method, l, b, x0, 1e-8, 20000, 0.0, 2.0)
    x, res = gpu_solve(dev, csr, method, l, b, x0, 1e-8, 20000, 0.0, 2.0, launch=launch)
    assert res.reason == 1 and ref.reason == "converged"
    assert abs(res.iters - ref.iters) <= 1
    assert _rel(x, ref.x) < 1e-8


@pytest.mark.parametrize("method,l", [("cg", 1), ("plcg", 1), ("plcg", 2), ("plcg", 4)])
@pytest.mark.parametrize("launch,x_update", [("streaming", "every"), ("streaming", "paired"),
                                             ("resident", "auto")])
def test_csr_early_iterates(dev, method, l, launch, x_update):
    """x after m steps against the oracle's x_m; streaming with x updated in
    every iteration and paired (odd m end on the separate last step)."""
    (rp, ci, va), As = scaled_variable((40, 30), 75)
    csr = Csr(dev, rp, ci, va)
    b = synth.uniform(As.n, 76)
    x0 = np.zeros(As.n)
    for m in (1, 2, 5, 20):
        ref = oracle_solve(As, method, l, b, x0, 1e-30, m, 0.0, 2.0)
        x, res = gpu_solve(dev, csr, method, l, b, x0, 1e-30, m, 0.0, 2.0, launch=launch,
                           x_update=x_update)
        assert res.iters == m == ref.iters
        assert res.x_update_every == (2 if x_update == "paired" else 1)
        assert _rel(x, ref.x) < 1e-13


def test_csr_mixed_precision_against_oracle(dev):
    """FP32-stored inner p(2)-CG in FP64 refinement on a scaled CSR matrix."""
    (rp, ci, va), As = scaled_variable((60, 50), 77)
    csr = Csr(dev, rp, ci, va)
    b = synth.uniform(As.n, 78)
    tol, inner = 1e-10, 1e-4
    ref = refine.refine(As, b, np.zeros(As.n), 2, shifts.chebyshev_shifts(2, 0.0, 2.0), tol,
                        inner, 20000)
    x, res = gpu_solve(dev, csr, "plcg", 2, b, np.zeros(As.n), tol, 20000, 0.0, 2.0,
                       precision="fp32", inner_tol=inner)
    assert res.reason == 1 and ref.reason == "converged"
    assert abs(res.outer - ref.outer) <= 1
    assert abs(res.iters - ref.inner_iters) <= 0.1 * ref.inner_iters + 2
    assert res.true_relres < tol
    lam_min = np.linalg.eigvalsh(operators.assemble(As))[0]
    assert np.linalg.norm(x - ref.x) <= 2 * (res.true_relres + ref.true_relres) * ref.rnorm0 / lam_min


def test_csr_rejects_invalid_matrices(dev):
    plcg = _plcg()
    rp, ci, va = synth.csr_variable_laplacian((6, 5))
    bad = {
        "rowptr start": (rp + 1, ci, va),
        "rowptr decreasing": (np.where(np.arange(len(rp)) == 5, rp[3], rp), ci, va),
        "column range": (rp, np.where(np.arange(len(ci)) == 9, 30, ci).astype(np.int32), va),
        "negative column": (rp, np.where(np.arange(len(ci)) == 9, -1, ci).astype(np.int32), va),
        "nan value": (rp, ci, np.where(np.arange(len(va)) == 3, np.nan, va)),
    }
    for name, (r, c, v) in bad.items():
        print(f"[gpu] invalid CSR: {name}", flush=True)
        csr = Csr(dev, r.astype(np.int64), c, v)
        with pytest.raises(plcg.PlcgError) as ei:
            plcg.Solver("csr", (30,), method="plcg", l=2, csr=csr.arg())
        assert ei.value.status == plcg.PLCG_E_INVALID, name


def _arrow(n, seed):
    """SPD arrow matrix: diagonal d_p in [2, 4), row and column 0 coupled to every
    unknown with weight 1/n (diagonally dominant).  Its rows have very uneven
    lengths, so the library keeps the CSR layout instead of the ELL copy."""
    d = 3.0 + synth.uniform(n, seed)
    rows, cols, vals = [0], [0], [d[0] + 1.0]
    for p in range(1, n):
        rows += [0, p, p]
        cols += [p, 0, p]
        vals += [1.0 / n, 1.0 / n, d[p]]
    rows, cols, vals = np.array(rows), np.array(cols), np.array(vals)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n), out=rp[1:])
    return rp, cols.astype(np.int32), vals


@pytest.mark.parametrize("method,l", [("cg", 1), ("plcg", 1), ("plcg", 2), ("plcg", 3)])
@pytest.mark.parametrize("launch", LAUNCHES)
def test_csr_uneven_rows_parity(dev, method, l, launch):
    rp, ci, va = _arrow(3001, 79)
    A = operators.csr(rp, ci, va)
    csr = Csr(dev, rp, ci, va)
    b = synth.uniform(A.n, 80)
    x0 = np.zeros(A.n)
    ref = oracle_solve(A, method, l, b, x0, 1e-10, 2000, 1.9, 4.2)
    x, res = gpu_solve(dev, csr, method, l, b, x0, 1e-10, 2000, 1.9, 4.2, launch=launch)
    assert res.reason == 1 and ref.reason == "converged"
    assert abs(res.iters - ref.iters) <= 1
    assert _rel(x, ref.x) < 1e-8


@pytest.mark.parametrize("name", ["poisson2048_cg", "poisson2048_p1", "poisson2048_p2",
                                  "poisson2048_p3"])
def test_csr_full_size_against_stored_oracle(dev, name):
    """The 2048^2 Poisson matrix assembled in CSR (the csr2048 benchmark
    workload) against the oracle's stored result for the same problem
    (tests/golden, written from the oracle only): iterations within 1, true
    residual within 10x, sampled ||x - x_oracle|| / ||x_oracle|| < 1e-8."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name + ".json")
    if not os.path.exists(path):
        pytest.skip(f"no stored oracle result {name}")
    with open(path) as f:
        g = json.load(f)
    dims = tuple(g["dims"])
    csr = Csr(dev, *synth.csr_variable_laplacian(dims))
    n = csr.n
    b = synth.uniform(n, g["seed"])
    lo, hi = g["interval"]
    x, res = gpu_solve(dev, csr, g["method"], max(int(g["l"]), 1), b, np.zeros(n), g["tol"],
                       100000, lo, hi)
    assert res.reason == 1 and abs(res.iters - g["iters"]) <= 1
    assert res.true_relres <= 10 * g["true_relres"] and g["true_relres"] <= 10 * res.true_relres
    idx = np.array(g["sample_idx"])
    ref = np.array(g["sample_x"])
    est = np.sqrt(n / idx.size * np.sum((x[idx] - ref) ** 2)) / g["xnorm"]
    assert est < 1e-8
    dense = _dense_error(x, g, dims)
    assert dense is None or dense < 1e-8, dense


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


# ------------------------------------------------------- Jacobi-scaled CSR --

def _unscaled_variable(dims, seed):
    cx, cy, cz = synth.edge_coefficients(dims, seed)
    rp, ci, va = synth.csr_variable_laplacian(dims, cx, cy, cz)
    A, As, dis = operators.variable_laplacian(dims, cx, cy, cz)
    return (rp, ci, va), A, As, dis


def gpu_solve_jacobi(dev, csr, method, l, b, x0, tol, maxit, launch="auto", **kw):
    plcg = _plcg()
    if launch == "resident" and (kw.get("precision", "fp64") != "fp64" or
                                 not plcg.resident_supported("csr", csr.n, method, l)):
        pytest.skip(f"no resident kernel for {method} l={l} n={csr.n}")
    print(f"[gpu] csr jacobi {method} l={l} n={csr.n} tol={tol} maxit={maxit} launch={launch}",
          flush=True)
    s = plcg.Solver("csr", (csr.n,), method=method, l=l, lmin=0.0, lmax=2.0, csr=csr.arg(),
                    jacobi=True, launch=launch, **kw)
    bt = torch.from_numpy(np.ascontiguousarray(b)).to(dev)
    xt = torch.from_numpy(np.ascontiguousarray(x0).copy()).to(dev)
    res = s.solve(bt.data_ptr(), xt.data_ptr(), tol, maxit,
                  torch.cuda.current_stream(dev).cuda_stream)
    if launch != "auto" and res.iters > 0:
        assert res.launch_mode == plcg.LAUNCH_MODES[launch]
    x = xt.cpu().numpy()
    s.close()
    return x, res


@pytest.mark.parametrize("dims", [(48, 40), (9, 7, 5)])
@pytest.mark.parametrize("method,l", [("cg", 1), ("plcg", 1), ("plcg", 2), ("plcg", 3)])
@pytest.mark.parametrize("launch", LAUNCHES)
def test_csr_jacobi_parity(dev, dims, method, l, launch):
    """Jacobi-preconditioned solve of an unscaled variable-coefficient matrix
    against the oracle on the scaled system from the scaled x0 (the same method,
    reading 15): iterations within 1, x within 1e-8, both residual norms."""
    (rp, ci, va), A, As, dis = _unscaled_variable(dims, 81)
    csr = Csr(dev, rp, ci, va)
    b = synth.uniform(A.n, 82)
    x0 = 0.1 * synth.uniform(A.n, 83)
    ref = oracle_solve(As, method, l, dis * b, x0 / dis, 1e-8, 20000, 0.0, 2.0)
    x, res = gpu_solve_jacobi(dev, csr, method, l, b, x0, 1e-8, 20000, launch=launch)
    assert res.reason == 1 and ref.reason == "converged"
    assert abs(res.iters - ref.iters) <= 1
    xr = dis * ref.x
    assert _rel(x, xr) < 1e-8
    assert res.rec_relres <= 10 * ref.true_relres
    r0 = np.linalg.norm(b - A(x0))
    assert abs(res.rnorm0 - r0) <= 1e-12 * r0
    true = np.linalg.norm(b - A(x)) / r0
    assert abs(res.true_relres - true) <= 1e-3 * true + 1e-15


@pytest.mark.parametrize("l", [1, 2, 3])
@pytest.mark.parametrize("launch", LAUNCHES)
def test_csr_jacobi_is_preconditioned_alg1(dev, l, launch):
    """The first iterates equal those of Alg. 1 with M = diag(A) (u != z,
    M-inner products) run by the oracle on the unscaled matrix."""
    (rp, ci, va), A, As, dis = _unscaled_variable((40, 30), 84)
    csr = Csr(dev, rp, ci, va)
    b = synth.uniform(A.n, 85)
    x0 = np.zeros(A.n)
    dinv = dis * dis
    sig = shifts.chebyshev_shifts(l, 0.0, 2.0)
    for m in (1, 5, 20):
        ref = oplcg.alg1(A, b, x0, l, sig, 0.0, m, Minv=lambda u: dinv * u)
        x, res = gpu_solve_jacobi(dev, csr, "plcg", l, b, x0, 1e-30, m, launch=launch)
        assert res.iters == m == ref.t_done
        assert _rel(x, ref.x) < 1e-12


def test_csr_jacobi_mixed_precision(dev):
    (rp, ci, va), A, As, dis = _unscaled_variable((60, 50), 86)
    csr = Csr(dev, rp, ci, va)
    b = synth.uniform(A.n, 87)
    tol, inner = 1e-10, 1e-4
    ref = refine.refine(As, dis * b, np.zeros(A.n), 2, shifts.chebyshev_shifts(2, 0.0, 2.0), tol,
                        inner, 20000)
    x, res = gpu_solve_jacobi(dev, csr, "plcg", 2, b, np.zeros(A.n), tol, 20000,
                              precision="fp32", inner_tol=inner)
    assert res.reason == 1 and ref.reason == "converged"
    assert abs(res.outer - ref.outer) <= 1
    assert abs(res.iters - ref.inner_iters) <= 0.1 * ref.inner_iters + 2
    lam_min = np.linalg.eigvalsh(operators.assemble(As))[0]
    y, yref = x / dis, ref.x
    assert np.linalg.norm(y - yref) <= 2 * (res.rec_relres + ref.true_relres) * ref.rnorm0 / lam_min


def test_csr_jacobi_needs_a_positive_diagonal(dev):
    plcg = _plcg()
    rp, ci, va = synth.csr_variable_laplacian((6, 5))
    va = va.copy()
    diag_entry = [j for j in range(rp[3], rp[4]) if ci[j] == 3][0]
    va[diag_entry] = -1.0
    csr = Csr(dev, rp, ci, va)
    with pytest.raises(plcg.PlcgError) as ei:
        plcg.Solver("csr", (30,), method="plcg", l=2, csr=csr.arg(), jacobi=True)
    assert ei.value.status == plcg.PLCG_E_INVALID
