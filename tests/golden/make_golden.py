"""Write the stored oracle results for the full-size workloads (calls only the oracle).

For each (workload, method) the oracle solves the seeded system once and the
script stores: iteration count, stop reason, restarts, recursive and true
relative residuals, ||x||_2, and x at the indices of synth.sample_indices; and,
in <name>_dense.npy (float64, no pickle), x at synth.dense_sample_indices (whole
grid rows at the seams of a split into eighths).
GPU tests compare the library against these at the same sizes.  "mixed" is
FP32-stored p(l)-CG in FP64 refinement (oracle.refine, inner tol 1e-4);
"batch" is system k of the batch512 recipe, solved alone on its Jacobi-scaled
form with p(2)-CG on [0, 2] (x stored in the original variables).

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
    "poisson3d256_p1": ("poisson3d256", "plcg", 1),
    "poisson3d256_p3": ("poisson3d256", "plcg", 3),
    "poisson3d256_cg": ("poisson3d256", "cg", 0),
    "poisson3d256_m3": ("poisson3d256", "mixed", 3),
    "diag2048_cg": ("diag2048", "cg", 0),
    "diag2048_p1": ("diag2048", "plcg", 1),
    "diag2048_p2": ("diag2048", "plcg", 2),
    "varcoef2048_p1": ("varcoef2048", "plcg", 1),
    "varcoef2048_p2": ("varcoef2048", "plcg", 2),
}
# batch512 systems: the smallest and the largest side of the recipe and two more
BATCH_SYSTEMS = (0, 1, 2, 3)
MIXED_INNER_TOL = 1e-4


def batch_system_index(k):
    """Index in the batch512 recipe of the k-th stored system."""
    import numpy as np

    import synth
    sides = np.array([d[0] for d, _, _ in synth.batch_recipe(512)])
    picks = [int(np.argmin(sides)), int(np.argmax(sides)), 100, 300]
    return picks[k]


def run_batch_system(name, k):
    import numpy as np

    import synth
    from oracle import operators, shifts
    from oracle import plcg as oplcg

    j = batch_system_index(k)
    dims, cseed, bseed = synth.batch_recipe(512)[j]
    cx, cy, cz = synth.edge_coefficients(dims, cseed)
    A, As, dis = operators.variable_laplacian(dims, cx, cy, cz)
    b = synth.uniform(A.n, bseed)
    t0 = time.time()
    r = oplcg.plcg(As, dis * b, np.zeros(A.n), 2, shifts.chebyshev_shifts(2, 0.0, 2.0), 1e-8,
                   100000)
    x = dis * r.x
    idx = synth.sample_indices(A.n)
    orig = float(np.linalg.norm(b - A(x)) / np.linalg.norm(b))
    return {
        "workload": "batch512", "method": "batch", "l": 2, "system": j, "dims": list(dims),
        "tol": 1e-8, "interval": [0.0, 2.0], "iters": int(r.iters), "reason": r.reason,
        "restarts": r.restarts, "rec_relres": float(r.rec_relres),
        "true_relres": float(r.true_relres), "orig_relres": orig,
        "xnorm": float(np.linalg.norm(x)),
        "sample_idx": [int(i) for i in idx], "sample_x": [float(v) for v in x[idx]],
        "oracle_seconds": time.time() - t0,
        "writer": "tests/golden/make_golden.py (oracle only)",
    }


def run(name):
    import numpy as np

    import synth
    from oracle import cg as ocg
    from oracle import operators, refine, shifts
    from oracle import plcg as oplcg

    if name.startswith("batch512_"):
        out = run_batch_system(name, int(name.split("_")[1]))
        with open(os.path.join(HERE, name + ".json"), "w") as f:
            json.dump(out, f)
        return name, out["iters"], out["oracle_seconds"]
    wl_name, method, l = JOBS[name]
    wl = synth.WORKLOADS[wl_name]
    dis = None
    if wl["kind"] == "diag":
        A = operators.diagonal(synth.spectrum_diagonal(wl["dims"]))
    elif wl["kind"] == "2d5var":
        # Jacobi-scaled: solve D^-1/2 A D^-1/2 y = D^-1/2 b, x = D^-1/2 y
        cx, cy, cz = synth.edge_coefficients(wl["dims"], wl["coef_seed"])
        A0, A, dis = operators.variable_laplacian(wl["dims"], cx, cy, cz)
    else:
        A = operators.laplacian(wl["dims"])
    b = synth.uniform(A.n, 0)
    x0 = np.zeros(A.n)
    lo, hi = wl["interval"]
    t0 = time.time()
    extra = {}
    if dis is not None:
        r = oplcg.plcg(A, dis * b, x0, l, shifts.chebyshev_shifts(l, lo, hi), wl["tol"], 100000)
        r.x = dis * r.x
        extra = {"restarts": r.restarts, "coef_seed": wl["coef_seed"], "jacobi": 1,
                 "orig_relres": float(np.linalg.norm(b - A0(r.x)) / np.linalg.norm(b))}
    elif method == "cg":
        r = ocg.cg(A, b, x0, wl["tol"], 100000)
        extra = {}
    elif method == "mixed":
        r = refine.refine(A, b, x0, l, shifts.chebyshev_shifts(l, lo, hi), wl["tol"],
                          MIXED_INNER_TOL, 100000)
        extra = {"outer": r.outer, "inner_tol": MIXED_INNER_TOL, "final_factor": 0.5}
        r.iters = r.inner_iters
        r.rec_relres = r.true_relres
    else:
        r = oplcg.plcg(A, b, x0, l, shifts.chebyshev_shifts(l, lo, hi), wl["tol"], 100000)
        extra = {"restarts": r.restarts}
    idx = synth.sample_indices(A.n)
    dense = synth.dense_sample_indices(wl["dims"])
    np.save(os.path.join(HERE, name + "_dense.npy"), r.x[dense], allow_pickle=False)
    out = {
        "workload": wl_name, "method": method, "l": l, "dims": list(wl["dims"]),
        "seed": 0, "tol": wl["tol"], "interval": list(wl["interval"]),
        "iters": int(r.iters), "reason": r.reason, "rec_relres": float(r.rec_relres),
        "true_relres": float(r.true_relres), "xnorm": float(np.linalg.norm(r.x)),
        "sample_idx": [int(i) for i in idx], "sample_x": [float(v) for v in r.x[idx]],
        "oracle_seconds": time.time() - t0, **extra,
        "dense_file": name + "_dense.npy", "dense_count": int(dense.size),
        "writer": "tests/golden/make_golden.py (oracle only)",
    }
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f)
    return name, r.iters, time.time() - t0


if __name__ == "__main__":
    names = sys.argv[1:] or list(JOBS) + [f"batch512_{k}" for k in BATCH_SYSTEMS]
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    with Pool(min(len(names), int(os.environ.get("GOLDEN_JOBS", "4")))) as pool:
        for name, iters, dt in pool.imap_unordered(run, names):
            print(f"{name}: {iters} iterations, {dt:.0f} s", flush=True)
