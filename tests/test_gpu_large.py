"""Large sizes: a 1024^3 grid (2^30 unknowns, half the int32 index range,
8.6 GB per vector) through the C ABI.  The oracle cannot run Alg. 1 at this
size, so the check is what it can compute exactly: the first iterate of CG and
of p(l)-CG from x0 = 0 is x_1 = alpha b with alpha = (b, b) / (b, A b) (one
plane at a time on the CPU); after two iterations p(1)-CG and CG agree (same x_t
in exact arithmetic).  Sampled outputs include the first and last 32 unknowns."""
import time

import numpy as np
import pytest

import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _alpha(b, dims):
    """(b, b) / (b, A b) for the 3D 7-point Dirichlet Laplacian, plane by plane."""
    nx, ny, nz = dims
    B = b.reshape(nz, ny, nx)
    bb = bab = 0.0
    for z in range(nz):
        P = B[z]
        s = 6.0 * P
        s[:, 1:] -= P[:, :-1]
        s[:, :-1] -= P[:, 1:]
        s[1:, :] -= P[:-1, :]
        s[:-1, :] -= P[1:, :]
        if z > 0:
            s -= B[z - 1]
        if z < nz - 1:
            s -= B[z + 1]
        bb += float(np.dot(P.ravel(), P.ravel()))
        bab += float(np.dot(P.ravel(), s.ravel()))
    return bb / bab


def test_billion_unknowns_first_iterates(dev):
    from paper_1905_06850_amd import plcg
    dims = (1024, 1024, 1024)
    n = dims[0] * dims[1] * dims[2]
    t0 = time.time()
    b = np.empty(n)
    step = 1 << 26
    for s0 in range(0, n, step):
        b[s0:s0 + step] = synth.uniform(min(step, n - s0), 0, start=s0)
    print(f"[large] b generated ({time.time() - t0:.0f} s)", flush=True)
    alpha = _alpha(b, dims)
    print(f"[large] alpha = {alpha!r} ({time.time() - t0:.0f} s)", flush=True)
    idx = synth.sample_indices(n)
    ref1 = alpha * b[idx]
    bt = torch.from_numpy(b).to(dev)
    del b
    stream = torch.cuda.current_stream(dev).cuda_stream
    idx_t = torch.from_numpy(idx).to(dev)
    x2 = {}
    for method, l in (("cg", 1), ("plcg", 1), ("plcg", 3)):
        s = plcg.Solver("3d7", dims, method=method, l=l, lmin=0.0, lmax=12.0)
        for m in (1, 2):
            print(f"[large] {method} l={l} m={m}", flush=True)
            xt = torch.zeros(n, dtype=torch.float64, device=dev)
            r = s.solve(bt.data_ptr(), xt.data_ptr(), 1e-30, m, stream)
            assert r.iters == m
            xs = xt[idx_t].cpu().numpy()
            if m == 1:
                assert np.abs(xs - ref1).max() <= 1e-12 * np.abs(ref1).max()
            else:
                x2[(method, l)] = xs
            del xt
            torch.cuda.empty_cache()
        s.close()
    ref2 = x2[("cg", 1)]
    for key in (("plcg", 1), ("plcg", 3)):
        assert np.abs(x2[key] - ref2).max() <= 1e-10 * np.abs(ref2).max()
    print(f"[large] done ({time.time() - t0:.0f} s)", flush=True)
