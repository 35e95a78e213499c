"""The device scalar engine (update of G, Eqs. haa1/haa3, LU, breakdown and
stopping tests), compiled for the host and fed the dot products the oracle's
p(l)-CG forms: the general form and the compile-time-l form the kernels run
leave the same state byte for byte after every column, and both stop where the
oracle stops (same iteration, converged or broken down)."""
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import synth
from oracle import operators, shifts
from oracle import plcg as oplcg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _record(A, b, l, lo, hi, tol):
    """Run the oracle with a recording inner product; return the per-column raw
    products in the engine's layout and the oracle's segment."""
    sig = shifts.chebyshev_shifts(l, lo, hi)
    calls = []

    def rec(u, v):
        d = float(np.dot(u, v))
        calls.append(d)
        return d

    beta0 = float(np.linalg.norm(b))
    seg = oplcg.alg1(A, b, np.zeros(A.n), l, sig, tol * beta0, 4000, dot=rec)
    beta = float(np.sqrt(calls[0]))            # the first product is (r_0, r_0)
    cols, pos, i = [], 1, 0
    while pos < len(calls):
        c = i + 1
        raw = [float("nan")] * (l + 1)
        if c - l >= 0:
            raw[0] = calls[pos]
            pos += 1
        for j in range(max(0, c - l + 1), c + 1):
            raw[j - (c - l)] = calls[pos]
            pos += 1
        cols.append((c, raw))
        i += 1
    return [float(s) for s in sig], beta, float(tol * beta), cols, seg


def _cases():
    out = []
    for l in (1, 2, 3, 4, 5, 8):
        A = operators.laplacian((32, 32))
        out.append((f"poisson32_l{l}", l, A, synth.uniform(A.n, 5), 0.0, 8.0))
    for l in (1, 2, 3):                         # interval too wide: breakdowns
        A = operators.laplacian((24, 20))
        out.append((f"wide_l{l}", l, A, synth.uniform(A.n, 7), 0.0, 16.0))
    for l in (2, 4):
        dims = (20, 18)
        cx, cy, cz = synth.edge_coefficients(dims, 9)
        _, As, _ = operators.variable_laplacian(dims, cx, cy, cz)
        out.append((f"var_l{l}", l, As, synth.uniform(As.n, 10), 0.0, 2.0))
    A = operators.laplacian((9, 8, 7))
    out.append(("p3d_l6", 6, A, synth.uniform(A.n, 11), 0.0, 12.0))
    return out


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_engine_forms_agree_and_stop_where_the_oracle_stops(tmp_path):
    exe = str(tmp_path / "engine_replay")
    cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off",
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1905_06850_amd", "csrc"),
           os.path.join(ROOT, "tests", "c", "engine_replay.hip"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    lines, expect = [], {}
    cases = _cases()
    lines.append(str(len(cases)))
    for name, l, A, b, lo, hi in cases:
        sig, beta, abs_tol, cols, seg = _record(A, b, l, lo, hi, 1e-10)
        expect[name] = seg
        lines.append(f"{name} {l} {len(cols)} {beta!r} {abs_tol!r} " +
                     " ".join(repr(s) for s in sig))
        lines += [f"{c} " + " ".join(repr(r) for r in raw) for c, raw in cols]
    inp = tmp_path / "raw.txt"
    inp.write_text("\n".join(lines) + "\n")
    proc = subprocess.run([exe, str(inp)], capture_output=True, text=True)
    print(proc.stdout)
    assert proc.returncode == 0, proc.stdout + proc.stderr
    seen = 0
    for line in proc.stdout.splitlines():
        m = re.match(r"(\S+)\s+l=(\d+) columns=(\d+) status=(\d+) last_t=(-?\d+)", line)
        if not m:
            continue
        seen += 1
        name, status, last_t = m.group(1), int(m.group(4)), int(m.group(5))
        seg = expect[name]
        assert line.endswith("identical"), line
        if seg.reason == "converged":
            assert status == 1 and last_t == seg.t_done, (line, seg.reason, seg.t_done)
        else:
            # breakdown: the engine keeps x_{t-1}, the oracle's t_done
            assert seg.reason == "breakdown" and status == 2 and last_t == seg.t_done, \
                (line, seg.reason, seg.t_done)
    assert seen == len(cases)
