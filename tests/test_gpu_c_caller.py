"""The C ABI from a plain C program (tests/c/solve_file.c, built by
__graft_entry__.build()): it reads b (and, for the variable-coefficient
operator, the edge coefficients), solves, writes x and checks two error paths;
x is compared with the oracle's."""
import os
import subprocess

import numpy as np
import pytest

import synth
from oracle import cg as ocg
from oracle import operators, shifts
from oracle import plcg as oplcg

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
BIN = os.path.join(HERE, "c", "solve_file")


@pytest.mark.parametrize("method,l", [("cg", 1), ("plcg", 1), ("plcg", 3)])
def test_c_caller_matches_oracle(tmp_path, method, l):
    assert os.path.exists(BIN), "tests/c/solve_file is not built (run __graft_entry__.build())"
    dims = (96, 80)
    A = operators.laplacian(dims)
    b = synth.uniform(A.n, 90)
    bpath, xpath = tmp_path / "b.bin", tmp_path / "x.bin"
    b.tofile(bpath)
    print(f"[gpu] C caller {method} l={l} dims={dims}", flush=True)
    out = subprocess.run([BIN, str(dims[0]), str(dims[1]), method, str(l), "1e-8", str(bpath),
                          str(xpath)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr + out.stdout
    fields = out.stdout.split()
    iters = int(fields[fields.index("iters") + 1])
    x = np.fromfile(xpath, dtype=np.float64)
    if method == "cg":
        ref = ocg.cg(A, b, np.zeros(A.n), 1e-8, 5000)
    else:
        ref = oplcg.plcg(A, b, np.zeros(A.n), l, shifts.chebyshev_shifts(l, 0.0, 8.0), 1e-8, 5000)
    assert abs(iters - ref.iters) <= 1
    assert np.linalg.norm(x - ref.x) <= 1e-8 * np.linalg.norm(ref.x)


@pytest.mark.parametrize("method,l", [("cg", 1), ("plcg", 2)])
def test_c_caller_variable_coefficients(tmp_path, method, l):
    """Edge coefficients from files, Jacobi-scaled solve on [0, 2], against the
    oracle on the scaled system."""
    assert os.path.exists(BIN), "tests/c/solve_file is not built (run __graft_entry__.build())"
    dims = (90, 70)
    cx, cy, _ = synth.edge_coefficients(dims, 91)
    A, As, dis = operators.variable_laplacian(dims, cx, cy)
    b = synth.uniform(A.n, 92)
    paths = [tmp_path / f for f in ("b.bin", "x.bin", "cx.bin", "cy.bin")]
    b.tofile(paths[0])
    cx.tofile(paths[2])
    cy.tofile(paths[3])
    print(f"[gpu] C caller variable coefficients {method} l={l} dims={dims}", flush=True)
    out = subprocess.run([BIN, str(dims[0]), str(dims[1]), method, str(l), "1e-8",
                          *[str(p) for p in paths]], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr + out.stdout
    fields = out.stdout.split()
    iters = int(fields[fields.index("iters") + 1])
    x = np.fromfile(paths[1], dtype=np.float64)
    if method == "cg":
        ref = ocg.cg(As, dis * b, np.zeros(A.n), 1e-8, 20000)
    else:
        ref = oplcg.plcg(As, dis * b, np.zeros(A.n), l, shifts.chebyshev_shifts(l, 0.0, 2.0),
                         1e-8, 20000)
    assert abs(iters - ref.iters) <= 1
    xr = dis * ref.x
    assert np.linalg.norm(x - xr) <= 1e-8 * np.linalg.norm(xr)
