"""The one-point-stencil toy (Sec. 4.2) through the C ABI against the oracle:
diagonal operator d = the 2D Laplacian's spectrum (input generator), oracle
applying it as a plain diagonal."""
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


def _rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


LAUNCHES = ["streaming", "resident"]


def gpu_solve(dev, d, method, l, b, x0, tol, maxit, launch="auto", x_update="auto"):
    plcg = _plcg()
    if launch == "resident" and not plcg.resident_supported("diag", d.size, method, l):
        pytest.skip(f"no resident kernel for {method} l={l} n={d.size}")
    print(f"[gpu] diag {method} l={l} n={d.size} tol={tol} maxit={maxit} launch={launch}",
          flush=True)
    dt = torch.from_numpy(d).to(dev)
    s = plcg.Solver("diag", (d.size,), method=method, l=l, lmin=0.0, lmax=8.0,
                    diag=dt.data_ptr(), launch=launch, x_update=x_update)
    del dt                                       # copied by plcg_create
    bt = torch.from_numpy(b).to(dev)
    xt = torch.from_numpy(x0.copy()).to(dev)
    res = s.solve(bt.data_ptr(), xt.data_ptr(), tol, maxit,
                  torch.cuda.current_stream(dev).cuda_stream)
    if launch != "auto" and res.iters > 0:
        assert res.launch_mode == plcg.LAUNCH_MODES[launch]
    x = xt.cpu().numpy()
    s.close()
    return x, res


def oracle_solve(d, method, l, b, x0, tol, maxit):
    D = operators.diagonal(d)
    if method == "cg":
        return ocg.cg(D, b, x0, tol, maxit)
    return oplcg.plcg(D, b, x0, l, shifts.chebyshev_shifts(l, 0.0, 8.0), tol, maxit)


@pytest.mark.parametrize("n", [1, 2, 511, 512, 513, 4096, 70001])
def test_diag_apply_is_exact(dev, n):
    plcg = _plcg()
    d = 0.5 + (synth.uniform(n, 50) + 1.0) * 3.0
    x = synth.uniform(n, 51)
    dt = torch.from_numpy(d).to(dev)
    s = plcg.Solver("diag", (n,), method="cg", diag=dt.data_ptr())
    xt = torch.from_numpy(x).to(dev)
    yt = torch.empty_like(xt)
    s.apply(xt.data_ptr(), yt.data_ptr(), torch.cuda.current_stream(dev).cuda_stream)
    assert np.array_equal(yt.cpu().numpy(), d * x)      # one correctly rounded product
    s.close()


@pytest.mark.parametrize("dims", [(64, 64), (37, 29), (130, 7)])
@pytest.mark.parametrize("method,l", [("cg", 1), ("plcg", 1), ("plcg", 2), ("plcg", 3),
                                      ("plcg", 5)])
@pytest.mark.parametrize("launch", LAUNCHES)
def test_diag_solve_parity(dev, dims, method, l, launch):
    d = synth.spectrum_diagonal(dims)
    b = synth.uniform(d.size, 0)
    x0 = np.zeros(d.size)
    ref = oracle_solve(d, method, l, b, x0, 1e-8, 20000)
    x, res = gpu_solve(dev, d, method, l, b, x0, 1e-8, 20000, launch=launch)
    assert res.reason == 1 and ref.reason == "converged", res.as_dict()
    assert abs(res.iters - ref.iters) <= 1
    assert res.true_relres <= 10 * ref.true_relres and ref.true_relres <= 10 * res.true_relres
    assert _rel(x, ref.x) < 1e-8


@pytest.mark.parametrize("method,l", [("cg", 1), ("plcg", 1), ("plcg", 2), ("plcg", 4)])
@pytest.mark.parametrize("launch,x_update", [("streaming", "every"), ("streaming", "paired"),
                                             ("resident", "auto")])
def test_diag_early_iterates(dev, method, l, launch, x_update):
    """x after m steps against the oracle's x_m; streaming with x updated in
    every iteration and paired (odd m end on the separate last step)."""
    d = synth.spectrum_diagonal((48, 40))
    b = synth.uniform(d.size, 8)
    x0 = 0.1 * synth.uniform(d.size, 9)
    for m in (1, 2, 5, 20):
        ref = oracle_solve(d, method, l, b, x0, 1e-30, m)
        x, res = gpu_solve(dev, d, method, l, b, x0, 1e-30, m, launch=launch, x_update=x_update)
        assert res.iters == m == ref.iters
        assert res.x_update_every == (2 if x_update == "paired" else 1)
        assert _rel(x, ref.x) < 1e-13


def test_diag_rejects_nonpositive_entries(dev):
    plcg = _plcg()
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        d = np.ones(1000)
        d[777] = bad
        dt = torch.from_numpy(d).to(dev)
        with pytest.raises(plcg.PlcgError) as ei:
            plcg.Solver("diag", (1000,), method="plcg", l=2, diag=dt.data_ptr())
        assert ei.value.status == plcg.PLCG_E_INVALID


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


@pytest.mark.parametrize("name", ["diag2048_cg", "diag2048_p1", "diag2048_p2"])
def test_diag_full_size_against_stored_oracle(dev, name):
    """The 2048^2 toy as the benchmark runs it, against the oracle's stored result
    (tests/golden, written from the oracle only): iterations within 1, true
    residual within 10x, sampled ||x - x_oracle|| / ||x_oracle|| < 1e-8."""
    g = _golden(name)
    d = synth.spectrum_diagonal(tuple(g["dims"]))
    n = d.size
    b = synth.uniform(n, g["seed"])
    x, res = gpu_solve(dev, d, g["method"], max(int(g["l"]), 1), b, np.zeros(n), g["tol"],
                       100000)
    assert res.reason == 1 and g["reason"] == "converged"
    assert abs(res.iters - g["iters"]) <= 1
    assert res.true_relres <= 10 * g["true_relres"] and g["true_relres"] <= 10 * res.true_relres
    idx = np.array(g["sample_idx"])
    ref = np.array(g["sample_x"])
    est = np.sqrt(n / idx.size * np.sum((x[idx] - ref) ** 2)) / g["xnorm"]
    assert est < 1e-8
    dense = _dense_error(x, g, tuple(g["dims"]))
    assert dense is None or dense < 1e-8, dense
