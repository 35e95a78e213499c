"""plcg_solve_noalloc (workspace in a static device array, no allocation)
against plcg_create + plcg_solve on the same inputs: x, counts and residuals
bit for bit, on two calls in a row, the second on a smaller system (the array
keeps the first call's contents), and x against the oracle."""
import ctypes

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


def _interval(dims):
    return (0.0, 8.0) if len(dims) == 2 else (0.0, 12.0)


def _solve_both(dev, dims, method, l, precision, x_update, tol, maxit):
    """(x, result) from plcg_solve_noalloc, then from a handle, same inputs."""
    plcg = _plcg()
    n = int(np.prod(dims))
    b = synth.uniform(n, 17)
    lo, hi = _interval(dims)
    stream = torch.cuda.current_stream(dev).cuda_stream
    print(f"[gpu] noalloc {method} l={l} dims={dims} {precision} x_update={x_update}", flush=True)
    s = plcg.Solver("2d5" if len(dims) == 2 else "3d7", dims, method=method, l=l, lmin=lo,
                    lmax=hi, precision=precision, inner_tol=1e-4 if precision == "fp32" else 0.0,
                    x_update=x_update)
    bt = torch.from_numpy(b).to(dev)
    xa = torch.zeros(n, dtype=torch.float64, device=dev)
    ra = plcg.plcg_result()
    st = plcg.plcg_solve_noalloc(ctypes.byref(s.desc), ctypes.byref(s.cfg), bt.data_ptr(),
                                 xa.data_ptr(), tol, maxit, stream, ctypes.byref(ra))
    plcg.check(st, "plcg_solve_noalloc")
    xh = torch.zeros(n, dtype=torch.float64, device=dev)
    rh = s.solve(bt.data_ptr(), xh.data_ptr(), tol, maxit, stream)
    s.close()
    return b, xa.cpu().numpy(), ra, xh.cpu().numpy(), rh


@pytest.mark.parametrize("method,l,precision,x_update,big,small", [
    ("plcg", 2, "fp64", "auto", (300, 300), (64, 64)),       # streaming, then resident
    ("plcg", 1, "fp64", "paired", (500, 400), (120, 90)),
    ("plcg", 3, "fp32", "auto", (256, 200), (40, 40)),
    ("cg", 1, "fp64", "auto", (48, 40, 44), (20, 13, 7)),
    ("plcg", 3, "fp64", "auto", (48, 40, 44), (16, 16, 16)),
])
def test_noalloc_equals_solve(dev, method, l, precision, x_update, big, small):
    for dims in (big, small):
        b, xa, ra, xh, rh = _solve_both(dev, dims, method, l, precision, x_update, 1e-9, 100000)
        assert ra.reason == rh.reason == 1, (ra.as_dict(), rh.as_dict())
        assert np.array_equal(xa.view(np.uint64), xh.view(np.uint64)), dims
        assert (ra.iters, ra.restarts, ra.outer, ra.spmvs, ra.launch_mode, ra.x_update_every) == \
            (rh.iters, rh.restarts, rh.outer, rh.spmvs, rh.launch_mode, rh.x_update_every)
        assert ra.rec_relres == rh.rec_relres and ra.true_relres == rh.true_relres
        assert ra.rnorm0 == rh.rnorm0 and ra.sweep_ms == 0.0
        if precision == "fp64":
            A = operators.laplacian(dims)
            x0 = np.zeros(A.n)
            if method == "cg":
                ref = ocg.cg(A, b, x0, 1e-9, 100000)
            else:
                lo, hi = _interval(dims)
                ref = oplcg.plcg(A, b, x0, l, shifts.chebyshev_shifts(l, lo, hi), 1e-9, 100000)
            assert abs(ra.iters - ref.iters) <= 1
            assert np.linalg.norm(xa - ref.x) / np.linalg.norm(ref.x) < 1e-8


def test_noalloc_rejects_beyond_its_array(dev):
    """A system whose work vectors do not fit the static array is refused with
    the bytes it needs, and the next call still works."""
    plcg = _plcg()
    s = plcg.Solver("2d5", (8, 8), method="plcg", l=1)
    desc = plcg.plcg_operator_desc(plcg.PLCG_OP_STENCIL2D5, 2048, 2048, 1)
    res = plcg.plcg_result()
    bt = torch.zeros(2048 * 2048, dtype=torch.float64, device=dev)
    xt = torch.zeros_like(bt)
    st = plcg.plcg_solve_noalloc(ctypes.byref(desc), ctypes.byref(s.cfg), bt.data_ptr(),
                                 xt.data_ptr(), 1e-8, 10, 0, ctypes.byref(res))
    assert st == plcg.PLCG_E_INVALID
    assert b"bytes" in plcg.plcg_last_error()
    s.close()
    _, xa, ra, xh, rh = _solve_both(dev, (70, 70), "plcg", 2, "fp64", "auto", 1e-8, 1000)
    assert ra.reason == 1 and np.array_equal(xa, xh)
