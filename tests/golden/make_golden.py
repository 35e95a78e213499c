"""Write the stored oracle results for the full-size workloads (calls only the oracle).

For each (workload, method) the oracle solves the seeded system once and the
script stores: iteration count, stop reason, restarts, recursive and true
relative residuals, ||x||_2, and x at the indices of synth.sample_indices.
GPU tests compare the library against these at the same sizes.

    python tests/golden/make_golden.py [name ...]     (names: see JOBS)
Runs single-threaded per job, jobs in parallel processes.
"""
import json
import os
import sys
import time
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

JOBS = {
    "poisson2048_cg": ("poisson2048", "cg", 0),
    "poisson2048_p1": ("poisson2048", "plcg", 1),
    "poisson2048_p2": ("poisson2048", "plcg", 2),
    "poisson2048_p3": ("poisson2048", "plcg", 3),
    "poisson2048_p4": ("poisson2048", "plcg", 4),
    "poisson2048_p5": ("poisson2048", "plcg", 5),
    "poisson3d256_p3": ("poisson3d256", "plcg", 3),
}


def run(name):
    import numpy as np

    import synth
    from oracle import cg as ocg
    from oracle import operators, shifts
    from oracle import plcg as oplcg

    wl_name, method, l = JOBS[name]
    wl = synth.WORKLOADS[wl_name]
    A = operators.laplacian(wl["dims"])
    b = synth.uniform(A.n, 0)
    x0 = np.zeros(A.n)
    t0 = time.time()
    if method == "cg":
        r = ocg.cg(A, b, x0, wl["tol"], 100000)
        extra = {}
    else:
        lo, hi = wl["interval"]
        r = oplcg.plcg(A, b, x0, l, shifts.chebyshev_shifts(l, lo, hi), wl["tol"], 100000)
        extra = {"restarts": r.restarts}
    idx = synth.sample_indices(A.n)
    out = {
        "workload": wl_name, "method": method, "l": l, "dims": list(wl["dims"]),
        "seed": 0, "tol": wl["tol"], "interval": list(wl["interval"]),
        "iters": int(r.iters), "reason": r.reason, "rec_relres": float(r.rec_relres),
        "true_relres": float(r.true_relres), "xnorm": float(np.linalg.norm(r.x)),
        "sample_idx": [int(i) for i in idx], "sample_x": [float(v) for v in r.x[idx]],
        "oracle_seconds": time.time() - t0, **extra,
        "writer": "tests/golden/make_golden.py (oracle only)",
    }
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f)
    return name, r.iters, time.time() - t0


if __name__ == "__main__":
    names = sys.argv[1:] or list(JOBS)
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    with Pool(min(len(names), 4)) as pool:
        for name, iters, dt in pool.imap_unordered(run, names):
            print(f"{name}: {iters} iterations, {dt:.0f} s", flush=True)
