"""Benchmark: p(l)-CG and classic CG on the 2D 5-point Poisson problem, 2048x2048.

One step = one complete solve (setup residual, every iteration, the final true
residual) of A x = b with b uniform[-1, 1) from seed 0, x0 = 0, stopped at
relative residual 1e-8; b and x already live in GPU memory when the clock
starts.  `value` is the iteration rate (x updates per second) of the headline
method; the JSON line also carries every method's rate, the iteration kernel's
duration against the HBM roofline (with its working set and whether that fits
the 256 MiB memory-side cache), a block for the 256^3 3D problem at 1e-10
(CG, p(1), p(3), FP32-refined p(3): working sets beyond that cache), and the
oracle's rate on the host CPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--methods cg,1,2,3,4,5]
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "iters/s + HBM GB/s, p(l)-CG vs CG at 1e-8 rel res; batched solves/s, p99 lat"
HBM_PEAK_GBS = 8000.0


def vector_passes(method: str, l: int, x_update_every: int = 1) -> float:
    # (mixed methods run the same sweep on 4-byte values: see bytes_per_pass)
    """Algorithmic vector passes per iteration (each pass = N doubles read or written).

    p(l)-CG fused sweep: reads z^{(l)}_i (stencil input, once), z^{(l)}_{i-1},
    the current and previous vector of each basis k < l, max(0, l-3) older
    z^{(l)} vectors for the dot products and p_{t-1}; writes z^{(l)}_{i+1}, l new
    basis vectors and p_t: 3l + 5 + max(0, l - 3); plus reading and writing x:
    3l + 7 + max(0, l - 3) with x_update_every = 1, and with x_update_every = 2
    (x read and written with p_{t-2} on even t only) 1.5 instead of 2 more on
    average: 3l + 6.5 + max(0, l - 3).
    Classic CG: sweep A reads r, p_{k-1}, writes p_k, A p_k (4); sweep B reads
    x, p, r, A p and writes x, r (6): 10 per iteration; with x_update_every = 2
    sweep B reads r, A p and writes r (3), and every second one also reads x,
    p_k, p_{k-1} and writes x (7): 9 per iteration on average.
    """
    if method == "cg":
        return 9 if x_update_every == 2 else 10
    return 3 * l + 5 + max(0, l - 3) + (1.5 if x_update_every == 2 else 2)


_CPU_SCRIPT = """
import json, os, resource, sys, time
sys.path.insert(0, {root!r})
import numpy as np
import synth
from oracle import operators, shifts, plcg
from oracle import cg as ocg


def cpu_s():
    r = resource.getrusage(resource.RUSAGE_SELF)
    return r.ru_utime + r.ru_stime


def timed(fn, reps):
    walls, cpus = [], []
    for _ in range(reps):
        c0, t0 = cpu_s(), time.perf_counter()
        out = fn()
        walls.append(time.perf_counter() - t0)
        cpus.append(cpu_s() - c0)
    return out, walls, cpus


wl = synth.WORKLOADS[{workload!r}]
if wl["kind"] == "diag":
    A = operators.diagonal(synth.spectrum_diagonal(wl["dims"]))
elif wl["kind"] == "csr":
    A = operators.csr(*synth.csr_variable_laplacian(wl["dims"]))
else:
    A = operators.laplacian(wl["dims"])
b = synth.uniform(A.n, 0)
x0 = np.zeros(A.n)
l = {l}
sig = shifts.chebyshev_shifts(l, *wl["interval"])
plcg.plcg(A, b, x0, l, sig, 1e-30, 2)
r, walls, cpus = timed(lambda: plcg.plcg(A, b, x0, l, sig, 1e-30, {iters}), {reps})
# a whole solve of the 64 x 64 Poisson problem (b = A x*, x* uniform, seed 0), tol 1e-8
A64 = operators.laplacian((64, 64))
b64 = A64(synth.uniform(A64.n, 0))
s64 = shifts.chebyshev_shifts(l, 0.0, 8.0)
r64, w64, c64 = timed(lambda: plcg.plcg(A64, b64, np.zeros(A64.n), l, s64, 1e-8, 5000), {reps})
print(json.dumps(dict(iters=r.iters, walls=walls, cpus=cpus, iters64=r64.iters, walls64=w64,
                      cpus64=c64)))
"""


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


def cpu_baseline(workload: str, l: int, iters: int, reps: int = 5) -> dict:
    """Time the oracle (numpy, FP64) on the host CPU: `reps` runs of its first
    `iters` p(l)-CG iterations on `workload`, and `reps` whole solves of the
    64 x 64 Poisson problem, once with one thread and once with every usable
    host thread allowed (OMP / BLAS thread counts).  Best and median of the runs
    (the paper's protocol takes the best of 5).  numpy runs the oracle's vector
    updates and stencil on one core whatever the setting; only its BLAS dot
    products can use more, so `cores` is the average number of cores the run
    kept busy (CPU time / wall time), next to the threads allowed."""
    import statistics
    model, ncpu, usable = cpu_info()
    runs = {}
    for label, threads in (("one_thread", 1), ("all_threads", usable)):
        t = str(threads)
        env = dict(os.environ, OMP_NUM_THREADS=t, OPENBLAS_NUM_THREADS=t, MKL_NUM_THREADS=t)
        code = _CPU_SCRIPT.format(root=ROOT, workload=workload, l=l, iters=iters, reps=reps)
        out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True,
                             env=env, timeout=900)
        if out.returncode != 0:
            raise RuntimeError(out.stderr)
        r = json.loads(out.stdout.strip().splitlines()[-1])
        rates = [r["iters"] / w for w in r["walls"]]
        runs[label] = {
            "threads_allowed": threads,
            "cores_busy": sum(r["cpus"]) / sum(r["walls"]),
            "iters_per_s_best": max(rates), "iters_per_s_median": statistics.median(rates),
            "solve64_s_best": min(r["walls64"]), "solve64_s_median": statistics.median(r["walls64"]),
            "solve64_iters": r["iters64"],
        }
    best = max(runs.values(), key=lambda v: v["iters_per_s_best"])
    name = "CG" if l == 0 else f"p({l})-CG"
    return {"value": best["iters_per_s_best"], "unit": "iters/s",
            "cores": round(best["cores_busy"], 2), "kind": "oracle",
            "sample": f"{reps} runs of the first {iters} iterations of {name} on {workload}, "
                      f"best of {reps} (value) and median, with 1 and with {usable} threads "
                      f"allowed; {reps} whole solves of the 64x64 Poisson problem (b = A x*, "
                      f"tol 1e-8) likewise; numpy FP64 oracle",
            "cpu_model": model, "nproc": ncpu, "usable_cpus": usable, "runs": runs}


def code_only(text: str) -> str:
    """C++ source with its comments removed and every run of whitespace made one
    space: what the compiler sees, so that an edit of a comment or of the layout
    leaves the kernel source hash alone."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c in "\"'":                      # string or character literal, kept whole
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
            out.append(" ")
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash() -> str:
    """Hash of the code (comments and layout aside) of the iteration kernels: the
    device code of the single-system path."""
    import hashlib
    h = hashlib.sha256()
    for name in ("plcg_kernels.hip", "plcg_var_kernels.hip", "plcg_sweep.h", "plcg_device.h",
                 "plcg_internal.h"):
        with open(os.path.join(ROOT, "paper_1905_06850_amd", "csrc", name), encoding="utf-8") as f:
            h.update(code_only(f.read()).encode())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed counter
    summary, or None.

    profiles/traffic_<workload>.txt holds lines `key value`: the kernel source
    hash the counters were taken with, and `<kernel> <bytes>` per launch (FETCH_SIZE
    plus WRITE_SIZE, each scaled by the copy-kernel calibration factor), the kernel
    named without namespace, argument list or spaces, e.g.
    `plcg_sweep_kernel<1,false,double,0,true>`.  `kernel` may leave out the
    trailing template arguments (the streaming cache hints and the x update
    pairing the library picked for the workload), or all of them (a name ending
    in `<`): the one kernel of that family in the file is taken.  A different
    source hash means the kernel changed since: None.  Returns (name, bytes).
    """
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            parts = line.split()
            if len(parts) == 2 and not line.startswith("#"):
                vals[parts[0]] = parts[1]
    if vals.get("source_sha256_16") != kernel_source_hash():
        return None
    if kernel in vals:
        return kernel, float(vals[kernel])
    prefix = kernel if kernel.endswith("<") else kernel[:-1] + ","
    family = [k for k in vals if k.startswith(prefix)]
    return (family[0], float(vals[family[0]])) if len(family) == 1 else None


def hr_launch(rows, head_method):
    head = {"plcg": "p", "mixed": "m", "cg": "cg"}[head_method[0]]
    return rows.get(head + (str(head_method[1]) if head != "cg" else ""), {}).get("launch")


def profile_run(plcg, ctx, methods):
    import torch
    b, x, sp = ctx["b"], ctx["x"], ctx["sp"]
    n = b.numel()
    y = torch.empty_like(b)
    for _ in range(10):
        plcg.check(plcg.plcg_copy(b.data_ptr(), y.data_ptr(), n, sp), "plcg_copy")
    torch.cuda.synchronize()
    for m in methods.split(","):
        method, l = ("cg", 1) if m == "cg" else ("plcg", int(m.lstrip("m")))
        s = make_solver(plcg, ctx, method, l, precision="fp32" if m.startswith("m") else "fp64")
        x.zero_()
        s.solve(b.data_ptr(), x.data_ptr(), 1e-30, 100, sp)
        torch.cuda.synchronize()
        s.close()
    print("profile run done", flush=True)


def copy_probe(plcg, torch, dev, sp):
    """Streaming reference: a plain copy (the library's plcg_copy and torch's
    copy_) of 32 MiB .. 4 GiB, to place the sweeps against what one read and one
    write stream reach on this GPU below and above the 256 MB Infinity Cache."""
    out = []
    for mb in (32, 128, 256, 512, 1024, 4096):
        n = mb * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        row = {"MiB": mb}
        for name, fn in (("plcg_copy", lambda: plcg.check(
                plcg.plcg_copy(a.data_ptr(), b.data_ptr(), n, sp), "plcg_copy")),
                         ("torch_copy", lambda: b.copy_(a))):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(20):
                fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 20
            row[name + "_GBps"] = 2 * n * 8 / ms / 1e6
        out.append(row)
        print(json.dumps(row), flush=True)
        del a, b


def batch_bench(args, plcg, torch, dev, sp):
    """512 variable-coefficient systems (sides uniform on [32, 512], lognormal(0,1)
    edges, Jacobi-scaled, shifts on [0, 2]) solved together by the batch engine."""
    import numpy as np
    import synth
    recipe = synth.batch_recipe(args.batch_count)
    systems = []
    for dims, cseed, bseed in recipe:
        cx, cy, cz = synth.edge_coefficients(dims, cseed)
        n = dims[0] * dims[1]
        systems.append(dict(dims=dims, cx=cx, cy=cy, n=n,
                            b=torch.from_numpy(synth.uniform(n, bseed)).to(dev)))
    total_n = sum(s["n"] for s in systems)
    xs = [torch.zeros(s["n"], dtype=torch.float64, device=dev) for s in systems]
    l = args.batch_l
    prec = args.batch_precision

    def run(sched, autotune, timed, l=l):
        probe = plcg.Batch(l=l, max_slots=1, arena_bytes=1 << 20, precision=prec)
        need = sum(probe.footprint(s["dims"], s["cx"], s["cy"]) for s in systems)
        probe.close()
        batch = plcg.Batch(l=l, max_slots=len(systems), arena_bytes=need + (64 << 20),
                           use_graph=True, precision=prec, inner_tol=args.inner_tol)
        if sched is not None:
            batch.set_schedule(sched)
        for x in xs:
            x.zero_()
        tickets = {}
        for k, s in enumerate(systems):
            t = batch.add(s["dims"], s["b"].data_ptr(), xs[k].data_ptr(), 1e-8, 100000, sp,
                          s["cx"], s["cy"])
            tickets[t] = k
        if autotune:
            batch.autotune(8, sp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = {}
        ticks = 0
        while tickets:
            batch.step(args.batch_ticks, sp)
            ticks += args.batch_ticks
            torch.cuda.synchronize()
            now = time.perf_counter() - t0
            for t in list(tickets):
                r = batch.poll(t)
                if r is not None:
                    done[tickets.pop(t)] = (r, now)
        dt = time.perf_counter() - t0
        chosen = batch.schedule()
        batch.close()
        return dt, done, ticks, chosen

    # untimed: autotune the block-to-system schedule on the live batch; then time
    # a fresh batch with the default schedule (4 chunks per workgroup for every
    # size class) and one with the tuned schedule, and the tuned one at l + 1
    _, _, _, sched = run(None, True, False)
    dt_def, done_def, _, _ = run(None, False, True)
    dt, done, ticks, _ = run(sched, False, True)
    dt_l1, done_l1, _, _ = run(sched, False, True, l=l + 1) if l + 1 <= 5 else (None, {}, 0, 0)
    lat = np.array([v[1] for v in done.values()]) * 1e3
    iters = {k: v[0].iters for k, v in done.items()}
    outer = [v[0].outer for v in done.values()]
    ok = sum(1 for v in done.values() if v[0].reason == 1)
    # per unknown and (inner) iteration: the sweep's vector passes in the storage
    # precision plus the 2 FP64 edge-weight arrays of the 2D operator
    word = 4 if prec == "fp32" else 8
    # (a batch sweep updates x every iteration)
    per_unknown = (3 * l + 7 + max(0, l - 3)) * word + 2 * 8
    sweep_bytes = sum(systems[k]["n"] * iters[k] * per_unknown for k in iters)
    line = {
        "metric": "batched solves/s (" + METRIC + ")",
        "value": len(done) / dt, "unit": "solves/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": dt * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if prec == "fp64" else "f32-storage/f64-dots",
        "data": "synthetic",
        "config": {"workload": f"batch{len(systems)}: 2D variable-coefficient 5-point systems, "
                               f"side uniform on [32, 512] ({total_n} unknowns in all), "
                               "lognormal(0,1) edge coefficients, Jacobi-scaled, b uniform[-1,1), "
                               "tol 1e-8 on the scaled residual",
                   "method": (f"p({l})-CG, shifts on [0, 2]" if prec == "fp64" else
                              f"FP32-stored p({l})-CG in FP64 refinement (inner tol "
                              f"{args.inner_tol:g}), shifts on [0, 2]"),
                   "converged": ok, "outer_max": max(outer),
                   "schedule_chunks_per_workgroup": {"le8_chunks": sched[0], "le64_chunks": sched[1],
                                                     "larger": sched[2]},
                   "default_schedule_solves_per_s": len(done_def) / dt_def,
                   f"l{l + 1}_solves_per_s": (len(done_l1) / dt_l1) if dt_l1 else None,
                   "ticks": ticks,
                   "iters_min": min(iters.values()), "iters_max": max(iters.values()),
                   "latency_ms_p50": float(np.percentile(lat, 50)),
                   "latency_ms_p99": float(np.percentile(lat, 99)),
                   "alg_GBps": sweep_bytes / dt / 1e9},
    }
    print(json.dumps(line), flush=True)


def serve_bench(args, plcg, torch, dev, sp):
    """Serving stream: Poisson arrivals of solve requests, 70 % 2D 5-point (side
    uniform on 64..2048) and 30 % 3D 7-point (side 32..256), lognormal(0,1) edge
    coefficients, tol uniform in {1e-6, 1e-8, 1e-10}; requests draw their
    operator from a pool of registered operators."""
    import numpy as np
    import synth
    rng_u = synth.uniform(4 * args.serve_pool, 900)        # in [-1, 1)
    pool = []
    for k in range(args.serve_pool):
        u0, u1 = (rng_u[4 * k] + 1) / 2, (rng_u[4 * k + 1] + 1) / 2
        if u0 < 0.7:
            side = 64 + int(u1 * (2048 - 64 + 1))
            dims = (side, side)
        else:
            side = 32 + int(u1 * (256 - 32 + 1))
            dims = (side, side, side)
        pool.append(dims)
    batch = plcg.Batch(l=args.batch_l, max_slots=args.serve_slots,
                       arena_bytes=int(args.serve_arena_gb * (1 << 30)), use_graph=True,
                       precision=args.batch_precision, inner_tol=args.inner_tol)
    ops, bs = [], []
    for k, dims in enumerate(pool):
        cx, cy, cz = synth.edge_coefficients(dims, 5000 + k)
        ops.append(batch.register(dims, cx, cy, cz, sp))
        bs.append(torch.from_numpy(synth.uniform(int(np.prod(dims)), 6000 + k)).to(dev))
        del cx, cy, cz
    torch.cuda.synchronize()
    tols = (1e-6, 1e-8, 1e-10)
    results = {}
    for rate, window in ((args.serve_rate, args.serve_window),
                         (args.serve_sustain_rate, args.serve_sustain_window)):
        n = max(1, int(rate * window))
        gaps = -np.log(1.0 - (synth.uniform(n, 901 + int(rate)) + 1) / 2 * 0.999999) / rate
        arrivals = np.cumsum(gaps) - gaps[0]
        pick = ((synth.uniform(n, 902 + int(rate)) + 1) / 2 * len(pool)).astype(int) % len(pool)
        ptol = ((synth.uniform(n, 903 + int(rate)) + 1) / 2 * 3).astype(int) % 3
        # each request's solution goes to its own device buffer (allocated before the run)
        outs = [torch.empty(int(np.prod(pool[int(pick[k])])), dtype=torch.float64, device=dev)
                for k in range(n)]
        reqs = [(float(arrivals[k]), int(pick[k]), 200000, tols[ptol[k]], outs[k].data_ptr())
                for k in range(n)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = batch.serve(ops, [b.data_ptr() for b in bs], reqs, args.serve_ticks,
                          args.serve_time_limit, sp)
        wall = time.perf_counter() - t0
        done = [k for k, o in enumerate(out) if o.finish_s >= 0]
        lat = np.array([out[k].finish_s - reqs[k][0] for k in done]) * 1e3
        wait = np.array([out[k].admit_s - reqs[k][0] for k in done]) * 1e3
        ok = sum(1 for k in done if out[k].result.reason == 1)
        del outs
        last = max(out[k].finish_s for k in done) if done else wall
        results[f"{rate:g}/s"] = {
            "requests": n, "completed": len(done), "converged": ok,
            "solves_per_s": len(done) / last if last > 0 else 0.0,
            "latency_ms_p50": float(np.percentile(lat, 50)) if done else None,
            "latency_ms_p99": float(np.percentile(lat, 99)) if done else None,
            "queue_wait_ms_p50": float(np.percentile(wait, 50)) if done else None,
            "queue_wait_ms_p99": float(np.percentile(wait, 99)) if done else None,
            "makespan_s": last, "offered_window_s": window,
        }
        if not args.quiet:
            print(f"# serve {rate:g}/s: {json.dumps(results[f'{rate:g}/s'])}", file=sys.stderr,
                  flush=True)
    batch.close()
    head = results[f"{args.serve_rate:g}/s"]
    line = {
        "metric": "served solves/s and p99 latency (" + METRIC + ")",
        "value": head["solves_per_s"], "unit": "solves/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": head["makespan_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.batch_precision == "fp64" else "f32-storage/f64-dots",
        "data": "synthetic",
        "config": {"workload": "serving stream: Poisson arrivals, 70 % 2D 5-point side 64..2048, "
                               "30 % 3D 7-point side 32..256, lognormal(0,1) edge coefficients "
                               "(Jacobi-scaled), tol uniform in {1e-6, 1e-8, 1e-10}",
                   "method": (f"p({args.batch_l})-CG" if args.batch_precision == "fp64" else
                              f"FP32-stored p({args.batch_l})-CG in FP64 refinement (inner tol "
                              f"{args.inner_tol:g})")
                             + ", continuous batching, admission by HBM footprint, "
                               "solutions into per-request buffers",
                   "pool": [list(d) for d in pool], "slots": args.serve_slots,
                   "arena_gb": args.serve_arena_gb, "runs": results},
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="poisson2048")
    ap.add_argument("--methods", default="cg,1,2,3,4,5")
    ap.add_argument("--headline", default="1",
                    help="headline method: l of p(l)-CG, or m<l> for FP32-refined p(l)-CG")
    ap.add_argument("--inner-tol", type=float, default=1e-3,
                    help="inner tolerance of the FP32-refined methods (m<l>)")
    ap.add_argument("--cpu-iters", type=int, default=40,
                    help="oracle iterations per CPU-baseline run (5 runs per thread setting)")
    ap.add_argument("--no-3d", action="store_true",
                    help="poisson2048: leave out the 256^3 block")
    ap.add_argument("--inner-tol-3d", type=float, default=1e-4,
                    help="inner tolerance of the FP32-refined p(3)-CG in the 256^3 block")
    ap.add_argument("--steps-3d", type=int, default=5,
                    help="timed solves per method in the 256^3 block (at most --steps)")
    ap.add_argument("--launch", choices=("auto", "streaming", "resident"), default="auto",
                    help="single-system launch mode (resident: one workgroup, small systems)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--batch-l", type=int, default=2)
    ap.add_argument("--batch-ticks", type=int, default=64)
    ap.add_argument("--batch-precision", choices=("fp64", "fp32"), default="fp64",
                    help="batch512: FP64, or FP32-stored inner solves in FP64 refinement")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-window", type=float, default=1.0)
    ap.add_argument("--serve-sustain-rate", type=float, default=6.0)
    ap.add_argument("--serve-sustain-window", type=float, default=4.0)
    ap.add_argument("--serve-pool", type=int, default=16)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-arena-gb", type=float, default=48.0)
    ap.add_argument("--serve-ticks", type=int, default=16)
    ap.add_argument("--serve-time-limit", type=float, default=120.0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="plain copy bandwidth at 32 MiB .. 4 GiB (streaming reference)")
    ap.add_argument("--profile-run", action="store_true",
                    help="short fixed run for hardware-counter passes: 10 copies of "
                         "n doubles, then 100 iterations of each method")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: libplcg solves on one GPU; it has no multi-GPU path (a system "
              "would shard by slabs with one halo exchange and one small all-reduce per "
              "iteration, not implemented), so only --gpus 1 runs.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1905_06850_amd import plcg

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.copy_probe:
        copy_probe(plcg, torch, dev, torch.cuda.current_stream(dev).cuda_stream)
        return
    if args.workload == "batch512":
        batch_bench(args, plcg, torch, dev, torch.cuda.current_stream(dev).cuda_stream)
        return
    if args.workload == "serve":
        serve_bench(args, plcg, torch, dev, torch.cuda.current_stream(dev).cuda_stream)
        return
    if args.profile_run:
        ctx = setup_workload(plcg, torch, dev, args.workload)
        profile_run(plcg, ctx, args.methods)
        return

    methods = [parse_method(m) for m in args.methods.split(",")]
    head_method = parse_method(args.headline)
    if head_method not in methods:
        methods.append(head_method)
    ctx = setup_workload(plcg, torch, dev, args.workload)
    rows = run_methods(args, plcg, torch, ctx, methods, args.steps, args.warmup)
    kind, dims, n = ctx["kind"], ctx["dims"], ctx["n"]
    lo, hi = ctx["interval"]
    tol = ctx["tol"]
    del ctx
    torch.cuda.empty_cache()
    opname = {"2d5": "2D 5-point Dirichlet Poisson", "3d7": "3D 7-point Dirichlet Poisson",
              "diag": "diagonal one-point-stencil toy with the 2D Laplacian's spectrum on",
              "csr": "2D 5-point Dirichlet Poisson assembled in CSR,",
              "2d5var": "2D variable-coefficient 5-point operator (lognormal(0,1) edges, "
                        "Jacobi-scaled)"}[kind]
    head = {"plcg": "p", "mixed": "m"}[head_method[0]] + str(head_method[1])
    hl = head_method[1]
    hr = rows[head]
    line = {
        "metric": METRIC,
        "value": hr["iters_per_s"],
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": hr["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if head_method[0] != "mixed" else "f32-storage/f64-dots",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {opname} {'x'.join(str(d) for d in dims)} "
                        f"({n} unknowns), b uniform[-1,1) seed 0, x0 = 0, stop at relative "
                        f"residual {tol:g}; Chebyshev shifts on [{lo:g},{hi:g}]",
            "method": (f"p({hl})-CG" if head_method[0] == "plcg"
                       else f"FP32-stored p({hl})-CG in FP64 refinement"), "l": hl,
            "iters_per_solve": hr["iters"], "true_relres": hr["true_relres"],
            "alg_GBps": hr["alg_GBps"],
            "cg_iters_per_s": rows["cg"]["iters_per_s"] if "cg" in rows else None,
        },
        "roofline": roofline(args.workload, kind, head_method, hr),
        "methods": rows,
    }
    if args.workload == "poisson2048" and not args.no_3d:
        line["poisson3d256"] = block_3d(args, plcg, torch, dev)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.workload, hl, args.cpu_iters)
    print(json.dumps(line), flush=True)


def parse_method(tok):
    if tok == "cg":
        return ("cg", 0)
    if tok.startswith("m"):
        return ("mixed", int(tok[1:]))
    return ("plcg", int(tok))


def setup_workload(plcg, torch, dev, workload):
    """Device inputs of a single-system workload: b (seed 0, or b = A x* for a
    manufactured solution), x, and the operator data of the diagonal / CSR kinds."""
    import synth
    wl = synth.WORKLOADS[workload]
    dims = wl["dims"]
    kind = wl["kind"]
    n = synth.grid_size(dims)
    b = torch.from_numpy(synth.uniform(n, 0)).to(dev)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    sp = torch.cuda.current_stream(dev).cuda_stream
    # the one-point-stencil toy: diagonal operator holding the Laplacian's spectrum
    dg = (torch.from_numpy(synth.spectrum_diagonal(dims)).to(dev) if kind == "diag" else None)
    dptr = dg.data_ptr() if dg is not None else None
    # a general sparse matrix: the grid operator assembled in CSR
    csr_t, csr_arg, op_bytes = None, None, 0
    # variable-coefficient stencil: edge coefficients on the device, Jacobi-scaled solve
    coef_t, coef_arg = None, None
    if kind == "2d5var":
        cx, cy, _ = synth.edge_coefficients(dims, wl["coef_seed"])
        coef_t = [torch.from_numpy(cx).to(dev), torch.from_numpy(cy).to(dev)]
        coef_arg = (coef_t[0].data_ptr(), coef_t[1].data_ptr(), None)
        op_bytes = 8 * (len(cx) + len(cy))        # the scaled edge weights, read once per SpMV
        del cx, cy
    if kind == "csr":
        rp, ci, va = synth.csr_variable_laplacian(dims)
        csr_t = [torch.from_numpy(a).to(dev) for a in (rp, ci, va)]
        csr_arg = (csr_t[0].data_ptr(), csr_t[1].data_ptr(), csr_t[2].data_ptr(), len(ci))
        op_bytes = 12 * len(ci)                   # the entries: FP64 value + int32 column
        del rp, ci, va
    elif kind == "diag":
        op_bytes = 8 * n
    if wl["rhs"] == "manufactured":
        # b = A x*, x* uniform (seed 0), formed with the library's operator
        xs = b.clone()
        op = plcg.Solver(kind, dims, method="cg", diag=dptr, csr=csr_arg)
        op.apply(xs.data_ptr(), b.data_ptr(), sp)
        torch.cuda.synchronize()
        op.close()
    return dict(dims=dims, kind=kind, n=n, interval=wl["interval"], tol=wl["tol"], b=b, x=x,
                sp=sp, dg=dg, dptr=dptr, csr_t=csr_t, csr_arg=csr_arg, op_bytes=op_bytes,
                coef_t=coef_t, coef_arg=coef_arg)


def make_solver(plcg, ctx, method, l, launch="auto", precision="fp64", inner_tol=0.0):
    """A solver for the workload of ctx (the variable-coefficient stencil Jacobi-scaled)."""
    lo, hi = ctx["interval"]
    var = ctx["kind"] == "2d5var"
    return plcg.Solver("2d5" if var else ctx["kind"], ctx["dims"], method=method, l=max(l, 1),
                       lmin=lo, lmax=hi, precision=precision, inner_tol=inner_tol,
                       diag=ctx["dptr"], csr=ctx["csr_arg"], coef=ctx["coef_arg"], jacobi=var,
                       launch=launch)


CACHE_BYTES = 256 << 20     # MI355X memory-side (Infinity) cache


def working_set(method, l, x_update_every, n, word, op_bytes):
    """Bytes one iteration's sweeps touch: p(l)-CG: 2 vectors per basis k < l,
    max(2, l-1) ring slots of z^(l), p (two buffers when x is updated every
    second iteration) and x; CG: r, its two p buffers, A p and x; plus the
    operator's data."""
    if method == "cg":
        vecs = 5
    else:
        vecs = 2 * l + max(2, l - 1) + (2 if x_update_every == 2 else 1) + 1
    return vecs * n * word + op_bytes


def run_methods(args, plcg, torch, ctx, methods, steps, warmup, tol=None, inner_tol=None):
    """Each method: `warmup` untimed solves, `steps` timed solves (host clock
    around them, device synchronised on both sides), then one solve with HIP
    events around the iteration kernels for their average duration."""
    dims, kind, n = ctx["dims"], ctx["kind"], ctx["n"]
    lo, hi = ctx["interval"]
    tol = ctx["tol"] if tol is None else tol
    inner_tol = args.inner_tol if inner_tol is None else inner_tol
    b, x, sp = ctx["b"], ctx["x"], ctx["sp"]
    op_bytes = ctx["op_bytes"]
    rows = {}
    for method, l in methods:
        name = {"cg": "cg", "plcg": f"p{l}", "mixed": f"m{l}"}[method]
        launch = args.launch
        if launch == "resident" and (method == "mixed" or kind == "2d5var" or
                                     not plcg.resident_supported(
                                         kind, n, "cg" if method == "cg" else "plcg", max(l, 1))):
            launch = "auto"
        s = make_solver(plcg, ctx, "cg" if method == "cg" else "plcg", l, launch,
                        "fp32" if method == "mixed" else "fp64", inner_tol)
        for _ in range(warmup):
            x.zero_()
            s.solve(b.data_ptr(), x.data_ptr(), tol, 100000, sp)
        torch.cuda.synchronize()
        total_iters = 0
        results = []
        t0 = time.perf_counter()
        for _ in range(steps):
            x.zero_()
            r = s.solve(b.data_ptr(), x.data_ptr(), tol, 100000, sp)
            total_iters += r.iters
            results.append(r)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        # Per-kernel duration: one more solve with HIP events around every
        # iteration kernel (outside the timed steps).
        s.set_timing(True)
        x.zero_()
        rt = s.solve(b.data_ptr(), x.data_ptr(), tol, 100000, sp)
        s.set_timing(False)
        torch.cuda.synchronize()
        s.close()
        r = results[-1]
        its = total_iters / dt
        passes = vector_passes("cg" if method == "cg" else "plcg", l, r.x_update_every)
        word = 4 if method == "mixed" else 8
        # vector passes in the storage precision, plus the operator's own data
        # read once per SpMV (FP64 d, or the CSR arrays)
        bytes_iter = passes * word * n + op_bytes
        kernel_us = 1e3 * rt.sweep_ms / max(rt.sweeps, 1)
        kernels_per_iter = 2 if method == "cg" else 1
        resident = r.launch_mode == plcg.PLCG_LAUNCH_RESIDENT
        wset = working_set(method, l, r.x_update_every, n, word, op_bytes)
        rows[name] = {
            "iters": r.iters, "reason": plcg.REASONS[r.reason], "restarts": r.restarts,
            "true_relres": r.true_relres, "rec_relres": r.rec_relres,
            "ms_per_solve": 1e3 * dt / steps, "iters_per_s": its,
            "bytes_per_iter": bytes_iter,
            "us_per_iter": 1e6 / its, "vector_passes": passes, "operator_bytes": op_bytes,
            "x_update_every": r.x_update_every,
            "alg_GBps": bytes_iter * its / 1e9,
            "kernel_us": kernel_us, "kernels_per_iter": kernels_per_iter,
            "kernel_GBps": (bytes_iter / kernels_per_iter) / (kernel_us * 1e-6) / 1e9
            if method != "cg" else None,
            "working_set_bytes": wset, "cache_resident": wset <= CACHE_BYTES,
            "spmvs": r.spmvs,
            "spmvs_per_s": r.spmvs * steps / dt,   # p(l)-CG adds l fill/drain SpMVs
            "outer": r.outer,
            "host_waits": r.host_waits,
            "launch": "resident" if resident else "streaming",
            # a resident solve is one launch per restart segment
            "launches_per_iter": ((1 + r.restarts) / max(r.iters, 1)) if resident
            else kernels_per_iter,
            "solves_per_s": steps / dt, "steps": steps, "warmup": warmup,
        }
        if not args.quiet:
            print(f"# {name}: {json.dumps(rows[name])}", file=sys.stderr, flush=True)
    return rows


def roofline(workload, kind, head_method, hr):
    """HBM roofline of the headline method's iteration kernel: algorithmic bytes
    per launch over its average duration (HIP events), against 8 TB/s; traffic
    from the committed counter summary when it was taken with these kernels;
    and whether the kernel's working set fits the 256 MiB memory-side cache
    (whose hits the achieved rate then includes)."""
    d3 = 'true' if kind == '3d7' else 'false'
    if head_method[0] == "cg" and hr["launch"] != "resident":
        # two sweeps per iteration (A: 4 passes, B: 5 on average when paired):
        # their mean duration against half the iteration's bytes
        bytes_launch = hr["bytes_per_iter"] / 2
        achieved = bytes_launch / (hr["kernel_us"] * 1e-6) / 1e9
        ta = measured_traffic(workload, f"cg_sweep_a_kernel<{d3}>")
        tb = measured_traffic(workload, "cg_sweep_b_kernel<")
        return {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": (ta[1] + tb[1]) / 2 if ta and tb else None,
            "traffic_sweep_a": ta[1] if ta else None,
            "kernel": "mean of cg_sweep_a_kernel and cg_sweep_b_kernel",
            "kernel_us": hr["kernel_us"], "bytes_per_launch": bytes_launch,
            "working_set_bytes": hr["working_set_bytes"], "cache_resident": hr["cache_resident"],
        }
    if hr["launch"] == "resident":
        kname = f"plcg_resident_kernel<{head_method[1]},"
    elif kind == "diag":
        kname = f"plcg_diag_sweep_kernel<{head_method[1]},"
    elif kind == "csr":
        kname = f"plcg_csr_sweep_kernel<{head_method[1]},"
    elif kind == "2d5var":
        kname = f"plcg_var_sweep_kernel<{head_method[1]},"
    else:
        kname = f"plcg_sweep_kernel<{head_method[1]},{d3},"
    word = 4 if head_method[0] == "mixed" else 8
    bytes_launch = hr["bytes_per_iter"]
    achieved = bytes_launch / (hr["kernel_us"] * 1e-6) / 1e9
    full = kname + ("double>" if word == 8 else "float>")
    traffic = measured_traffic(workload, full)
    return {
        "bound": "hbm",
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic[1] if traffic else None,
        "kernel": traffic[0] if traffic else full,
        "kernel_us": hr["kernel_us"],
        "bytes_per_launch": bytes_launch,
        "working_set_bytes": hr["working_set_bytes"],
        "cache_resident": hr["cache_resident"],
    }


def block_3d(args, plcg, torch, dev):
    """The 256^3 3D 7-point Poisson workload at relative residual 1e-10 (b
    uniform, seed 0): CG, p(1)-CG and p(3)-CG in FP64 and FP32-stored p(3)-CG
    and p(1)-CG in FP64 refinement, each solved to the same final accuracy; its
    working set (1.3-1.6 GB in FP64) is far beyond the memory-side cache, so its
    roofline is HBM-true.  Fewer steps than the headline (each solve takes
    0.15-0.4 s)."""
    ctx = setup_workload(plcg, torch, dev, "poisson3d256")
    steps = max(1, min(args.steps, args.steps_3d))
    rows = run_methods(args, plcg, torch, ctx, [("cg", 0), ("plcg", 1), ("plcg", 3),
                                                 ("mixed", 3), ("mixed", 1)], steps, 1,
                       inner_tol=args.inner_tol_3d)
    del ctx
    torch.cuda.empty_cache()
    p3 = rows["p3"]
    return {
        "workload": "poisson3d256: 3D 7-point Dirichlet Poisson 256x256x256 (16777216 "
                    "unknowns), b uniform[-1,1) seed 0, x0 = 0, stop at relative residual "
                    "1e-10; Chebyshev shifts on [0,12]",
        "steps": steps, "warmup": 1,
        "time_to_solution_ms": {k: v["ms_per_solve"] for k, v in rows.items()},
        "true_relres": {k: v["true_relres"] for k, v in rows.items()},
        "iters_per_s": {k: v["iters_per_s"] for k, v in rows.items()},
        "mixed_inner_tol": args.inner_tol_3d,
        "mixed_vs_fp64_p3": p3["ms_per_solve"] / rows["m3"]["ms_per_solve"],
        "fastest": min(rows, key=lambda k: rows[k]["ms_per_solve"]),
        "roofline": roofline("poisson3d256", "3d7", ("plcg", 3), p3),
        "roofline_cg": roofline("poisson3d256", "3d7", ("cg", 0), rows["cg"]),
        "methods": rows,
    }


if __name__ == "__main__":
    main()
