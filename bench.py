"""Benchmark: full SPMESL solves/s at p = 5000 on one MI355X.

A step is one full solve (standardise -> S -> p scaled-lasso regressions ->
Omega, B and sigma written to HBM) of the block-AR(1) workload
(n = 400, p = 5000, 50 blocks of 100 with AR(1) covariance rho = 0.6,
lambda0 = sqrt(2 log p / n), tol 1e-8), with X already resident in HBM.
The headline is the mixed-precision form; the plain double form is timed
beside it.  `value` is the throughput of K solves enqueued back to back
(each the replay of the solve's HIP graph) and synchronised once; the rate
of one call at a time (each waiting for its result) is reported beside it.
Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"bf16": 2500.0, "fp32": 157.3, "fp64": 78.6}
WORKLOAD = "blockar_n400_p5000"


def kernel_costs(n, p, prec, mean_w=None):
    """Algorithmic work of one launch of each kernel step: (bytes, flops, flop dtype).

    S = Xs^T Xs / n needs n p (p + 1) flops (the upper triangle, one
    multiply-add per sample and pair); the mixed form issues three bf16
    products per term.  Its bytes are S written once (4 or 8 p^2) and the
    standardised data read once (the bf16 split: 4 npad p; double 8np,
    float 4np).  The mixed form's
    standardisation reads X once and writes Xt (double) and the bf16 split
    (8np + 8np + 4 npad p bytes).  The row-tiled KKT pass reads S once; the
    zero fill writes one dense p x p double output.  The double polish of
    the mixed form reads, for each column, the rows of the standardised data
    on its working set and its own (8 n (|W| + 1) bytes, with mean_w the mean
    final working set).  The column solves are latency-bound chains of small
    gathers and have no such figure.
    """
    tsz = 8 if prec == "fp64" else 4
    fl = float(n) * p * (p + 1)
    npad = (n + 63) // 64 * 64
    syrk = {"fp64": ("syrk_f64", (8.0 * p * p + 8.0 * n * p, fl, "fp64")),
            "fp32": ("syrk_f32", (4.0 * p * p + 4.0 * n * p, fl, "fp32")),
            "mixed": ("syrk_bf16x3", (4.0 * p * p + 4.0 * npad * p, 3 * fl, "bf16"))}[prec]
    costs = {
        syrk[0]: syrk[1],
        "kkt_rows": (float(tsz) * p * p, 0.0, None),
        "fill_B": (8.0 * p * p, 0.0, None),
        "fill_Omega": (8.0 * p * p, 0.0, None),
    }
    if prec == "mixed":
        costs["standardize"] = (16.0 * n * p + 4.0 * npad * p, 0.0, None)
        if mean_w is not None:
            costs["polish"] = (8.0 * n * (mean_w + 1.0) * p, 0.0, None)
    return costs


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "blockar_n400_p5000_hbm_traffic.md")
CSRC = os.path.join(ROOT, "paper_2203_15031_amd", "csrc")
# step name -> (row label in the traffic summary, source files of its kernel)
TRAFFIC_ROWS = {
    ("syrk_bf16x3", None): ("syrk_bf16x3", ["syrk.hip"]),
    ("syrk_f64", None): ("syrk_f64", ["syrk.hip"]),
    ("kkt_rows", "fp64"): ("kkt_rows (double)", ["kkt.hip"]),
    ("kkt_rows", "mixed"): ("kkt_rows (float)", ["kkt.hip"]),
    ("standardize", "mixed"): ("standardize (mixed)", ["standardize.hip"]),
    ("polish", None): ("polish", ["polish.hip"]),
    ("fill_B", None): ("fill_B / fill_Omega", ["output.hip"]),
    ("fill_Omega", None): ("fill_B / fill_Omega", ["output.hip"]),
}


def measured_traffic(step, prec):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by a copy of known size), or None when
    there is none for this step or its kernel's source has changed since."""
    import hashlib
    key = TRAFFIC_ROWS.get((step, prec)) or TRAFFIC_ROWS.get((step, None))
    if key is None or not os.path.exists(TRAFFIC_FILE):
        return None
    label, files = key
    h = hashlib.sha1()
    for fn in files:
        with open(os.path.join(CSRC, fn), "rb") as fh:
            h.update(fh.read())
    for line in open(TRAFFIC_FILE):
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if len(cells) == 7 and cells[0] == label:
            return float(cells[5]) if cells[6] == h.hexdigest()[:12] else None
    return None


def roofline_of(name, ms, cost):
    """Roofline of one kernel launch: algorithmic bytes or flops / its time."""
    nbytes, flops, fdt = cost
    t = ms * 1e-3
    t_hbm = nbytes / (PEAK_HBM_GBS * 1e9)
    t_mfma = flops / (PEAK_TFLOPS[fdt] * 1e12) if fdt else 0.0
    if t_mfma > t_hbm:
        ach = flops / t / 1e12
        peak = PEAK_TFLOPS[fdt]
        return {"kernel": name, "bound": "mfma", "achieved": round(ach, 2), "peak": peak,
                "unit": "TFLOP/s", "frac": round(ach / peak, 4), "traffic": None,
                "dtype": fdt, "ms_per_launch": round(ms, 5)}
    ach = nbytes / t / 1e9
    return {"kernel": name, "bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4), "traffic": None,
            "ms_per_launch": round(ms, 5)}


def whole_solve_roofline(n, p, prec, stats, ms):
    """T_roof / T_measured of one whole solve.

    T_roof sums, over the solve's phases, max(algorithmic bytes / HBM peak,
    algorithmic flops / matrix-core peak of the phase's precision):
      standardisation  X read, the standardised copies written
      covariance       S written once, the standardised data read once;
                       n p (p + 1) flops (three bf16 products per term in
                       the mixed form)
      KKT pass         S read once (the row-tiled pass over every column)
      active-set sweeps 16 B (float) or 32 B (double) per coordinate per
                       sweep (read and write of gradient and coefficient),
                       with the device counters' sweeps times the mean
                       final working set
      double polish    (mixed) the rows of the standardised data on each
                       column's working set plus its own: 8 n (|W| + 1)
      outputs          B and Omega written dense (16 p^2), sigma (8 p)
    The in-wave KKT passes of re-solved columns and the scatter of the
    nonzeros are left out (they only lower T_roof)."""
    tsz = 8 if prec == "fp64" else 4
    npad = (n + 63) // 64 * 64
    mean_w = stats["sum_working_set"] / p
    fl = float(n) * p * (p + 1)
    ph = {}
    if prec == "mixed":
        ph["standardize"] = (16.0 * n * p + 4.0 * npad * p, 0.0, None)
        ph["covariance"] = (4.0 * p * p + 4.0 * npad * p, 3 * fl, "bf16")
    else:
        ph["standardize"] = (8.0 * n * p + tsz * n * p, 0.0, None)
        ph["covariance"] = (tsz * p * p + tsz * n * p, fl, "fp64" if prec == "fp64" else "fp32")
    ph["kkt_pass"] = (float(tsz) * p * p, 0.0, None)
    ph["active_set_sweeps"] = (2.0 * 2 * tsz * stats["total_sweeps"] * mean_w, 0.0, None)
    if prec == "mixed":
        ph["polish"] = (8.0 * n * p * (mean_w + 1.0), 0.0, None)
    ph["outputs"] = (16.0 * p * p + 8.0 * p, 0.0, None)
    out, tot, nbytes, nflops = {}, 0.0, 0.0, 0.0
    for k, (b, f, dt) in ph.items():
        t = max(b / (PEAK_HBM_GBS * 1e9), f / (PEAK_TFLOPS[dt] * 1e12) if dt else 0.0)
        out[k] = {"bytes": b, "flops": f, "t_roof_us": round(t * 1e6, 3)}
        tot += t
        nbytes += b
        nflops += f
    return {"t_roof_ms": round(tot * 1e3, 5), "t_measured_ms": round(ms, 5), "frac": round(tot * 1e3 / ms, 4),
            "bytes": nbytes, "flops": nflops, "phases": out,
            "note": "T_measured is the pipelined time per solve; peaks as in roofline"}


# the forms a run can time: name -> (precision, data form)
FORMS = {"mixed": ("mixed", False), "fp64": ("fp64", False), "fp32": ("fp32", False), "data": ("fp64", True)}
DTYPES = {"mixed": "bf16x3-f32+f64", "fp64": "f64", "fp32": "f32", "data": "f64"}


def time_form(ctx, X, lam0, tol, form, steps, warmup, torch):
    prec, data = FORMS[form]
    p = X.shape[1]
    out = dict(B=torch.empty((p, p), dtype=torch.float64, device=X.device),
               sigma=torch.empty((p,), dtype=torch.float64, device=X.device),
               Omega=torch.empty((p, p), dtype=torch.float64, device=X.device))
    status = torch.full((1,), 99, dtype=torch.int32, device=X.device)
    for _ in range(warmup):
        ctx.solve(X, lam0, tol, prec, out=out, data_form=data)
        ctx.solve_async(X, lam0, status, tol, prec, out=out, data_form=data)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    # the job: K full solves enqueued back to back (each one replay of the
    # solve's HIP graph), then one synchronisation
    status.fill_(99)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        ctx.solve_async(X, lam0, status, tol, prec, out=out, data_form=data)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    if int(status.item()) != 0:
        raise RuntimeError(f"{prec} solve returned status {int(status.item())}")
    # one call at a time: each call waits for its solve and reads its status;
    # each call is bracketed by its own events (median, min, max per call)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for a, b in ev:
        a.record(stream)
        r = ctx.solve(X, lam0, tol, prec, out=out, data_form=data)
        b.record(stream)
    torch.cuda.synchronize()
    per_call = sorted(a.elapsed_time(b) for a, b in ev)
    ms_sync = {"median": per_call[len(per_call) // 2], "min": per_call[0], "max": per_call[-1],
               "mean": sum(per_call) / len(per_call)}
    # the same solves with the library's HIP events: per phase, and per
    # kernel launch on the stream each kernel runs on
    ph = {k: 0.0 for k in ("standardize", "covariance", "solve", "polish", "output", "total")}
    kern = {}
    reps = max(1, min(steps, 10))
    for _ in range(reps):
        r = ctx.solve(X, lam0, tol, prec, out=out, timing=True, data_form=data)
        for k in ph:
            ph[k] += r.stats["ms_" + k] / reps
        for name, kms in ctx.kernel_times():
            d = kern.setdefault(name, [0.0, 0])
            d[0] += kms
            d[1] += 1
    kern = {k: {"ms_per_solve": v[0] / reps, "launches": v[1] / reps, "ms_per_launch": v[0] / v[1]}
            for k, v in kern.items()}
    return ms, ms_sync, ph, kern, r


def cpu_baseline(X_np, lam0, tol, target_s=20.0):
    """The oracle (plain FP64 CPU Algorithm 1 per column, OpenMP over columns)
    on a sample of response columns; scaled to full solves/s."""
    import numpy as np
    import oracle
    n, p = X_np.shape
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    rng = np.random.default_rng(123)
    # calibrate on a few columns, then size the sample to ~target_s of CPU work
    probe = rng.choice(p, size=min(p, 2 * cores), replace=False)
    t0 = time.perf_counter()
    oracle.spmesl_columns(X_np, lam0, probe, tol=tol, nthreads=cores)
    dt = time.perf_counter() - t0
    per_col_cpu = dt * cores / len(probe)
    m = int(min(p, max(len(probe), target_s / max(per_col_cpu, 1e-6))))
    cols = rng.choice(p, size=m, replace=False)
    t0 = time.perf_counter()
    oracle.spmesl_columns(X_np, lam0, cols, tol=tol, nthreads=cores)
    wall = time.perf_counter() - t0
    full_s = wall * p / m
    return {"value": round(1.0 / full_s, 6), "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"{m} of {p} response columns of the same workload (Algorithm 1 per column, "
                      f"tol {tol:g}), {wall:.2f} s wall on {cores} threads, scaled by p/{m}; "
                      f"Omega assembly excluded"}


def cpu_baseline_single_thread(X_np, lam0, tol, target_s=10.0):
    """The oracle as cpu_baseline, on one host thread."""
    import numpy as np
    import oracle
    n, p = X_np.shape
    rng = np.random.default_rng(321)
    probe = rng.choice(p, size=4, replace=False)
    t0 = time.perf_counter()
    oracle.spmesl_columns(X_np, lam0, probe, tol=tol, nthreads=1)
    per_col = (time.perf_counter() - t0) / len(probe)
    m = int(min(p, max(len(probe), target_s / max(per_col, 1e-6))))
    cols = rng.choice(p, size=m, replace=False)
    t0 = time.perf_counter()
    oracle.spmesl_columns(X_np, lam0, cols, tol=tol, nthreads=1)
    wall = time.perf_counter() - t0
    return {"value": round(m / (wall * p), 7), "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"{m} of {p} response columns of the same workload (Algorithm 1 per column, "
                      f"tol {tol:g}), {wall:.2f} s on one thread, scaled by p/{m}; Omega assembly excluded"}


def errors_vs_oracle(X_np, lam0, results, m=32):
    """Per-result error of each form against the oracle's exact minimiser
    (tol 1e-12) on m sampled response columns: max |B_gpu - B_orc| /
    max |B_orc| over each sampled column of B, and the relative error of
    sigma, on the data's scale (Proposition 1 applied to the oracle)."""
    import numpy as np
    import oracle
    p = X_np.shape[1]
    cols = np.sort(np.random.default_rng(7).choice(p, size=m, replace=False))
    ref = oracle.spmesl_columns(X_np, lam0, cols, tol=1e-12, nthreads=0)
    c = ref["c"]
    Bo = ref["B"] * c[:, None] / c[cols][None, :]
    so = ref["sigma"] / c[cols]
    out = {"columns": m, "reference": "oracle, tol 1e-12"}
    for prec, (B, sig) in results.items():
        Bc = B[:, cols]
        eb = max(float(np.abs(Bc[:, i] - Bo[:, i]).max() / np.abs(Bo[:, i]).max()) if np.abs(Bo[:, i]).max() > 0
                 else float(np.abs(Bc[:, i]).max()) for i in range(m))
        es = float(np.max(np.abs(sig[cols] - so) / so))
        out[prec] = {"B_columns": eb, "sigma": es}
    return out


def batched_replicas(args, torch, spmesl, workloads, forms, tol):
    """The batched form on the headline shape: `--replicas` independent data
    sets of the workload's structure and size in one grouped call per step
    (every step of the path one launch over all of them); time per call and
    per solve, with the whole-solve roofline per solve."""
    k = args.replicas
    w = workloads.workload(args.workload)
    Xs = [torch.from_numpy(X).to("cuda:0") for X in workloads.generate_replicas(args.workload, k)]
    ctx = spmesl.Context(0)
    outs = [dict(B=torch.empty((w.p, w.p), dtype=torch.float64, device="cuda:0"),
                 sigma=torch.empty((w.p,), dtype=torch.float64, device="cuda:0"),
                 Omega=torch.empty((w.p, w.p), dtype=torch.float64, device="cuda:0")) for _ in Xs]
    out = {"count": k, "data": f"{k} independent draws of the workload (its own X and {k - 1} more seeds)"}
    steps = max(2, args.steps // 2)
    for prec in forms:
        for _ in range(max(1, args.warmup)):
            r = ctx.solve_batch(Xs, w.lambda0, tol, prec, outs=outs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = ctx.solve_batch(Xs, w.lambda0, tol, prec, outs=outs)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000 / steps
        ent = {"ms_per_call": round(ms, 4), "ms_per_solve": round(ms / k, 4),
               "solves_per_s": round(1000.0 * k / ms, 2)}
        if not FORMS[prec][1]:
            ent["whole_solve"] = whole_solve_roofline(w.n, w.p, prec, r[0].stats, ms / k)
        out[prec] = ent
        print(f"[bench] batched {prec}: {k} data sets in {ms:.3f} ms, {ms / k:.4f} ms per solve",
              file=sys.stderr, flush=True)
    del outs, Xs
    torch.cuda.empty_cache()
    return out


def bench_batch(args, torch, spmesl, workloads):
    """The batched hub workload: 64 data sets of uneven shape, one library call per step."""
    Xs_np = workloads.generate_batch()
    Xs = [torch.from_numpy(X).to("cuda:0") for X in Xs_np]
    lams = [math.sqrt(2 * math.log(X.shape[1]) / X.shape[0]) for X in Xs_np]
    ctx = spmesl.Context(0)
    line = {"metric": "batched SPMESL data sets/s (64 hub data sets, p~U{256..4096}, n=ceil(p/2))",
            "unit": "datasets/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "data": "synthetic",
            "config": {"workload": "hub_batch64", "count": len(Xs), "sum_p": int(sum(X.shape[1] for X in Xs_np)),
                       "tol": 1e-8}}
    outs = [dict(B=torch.empty((X.shape[1], X.shape[1]), dtype=torch.float64, device="cuda:0"),
                 sigma=torch.empty((X.shape[1],), dtype=torch.float64, device="cuda:0"),
                 Omega=torch.empty((X.shape[1], X.shape[1]), dtype=torch.float64, device="cuda:0"))
            for X in Xs]
    for prec in args.forms.split(","):
        for _ in range(args.warmup):
            ctx.solve_batch(Xs, lams, 1e-8, prec, outs=outs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            ctx.solve_batch(Xs, lams, 1e-8, prec, outs=outs)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000 / args.steps
        line.setdefault("forms", {})[prec] = {"ms_per_step": round(ms, 3),
                                              "datasets_per_s": round(len(Xs) * 1000 / ms, 2)}
        print(f"[bench] batch {prec}: {ms:.3f} ms per 64 data sets", file=sys.stderr, flush=True)
    head = args.forms.split(",")[0]
    line["value"] = line["forms"][head]["datasets_per_s"]
    line["ms_per_step"] = line["forms"][head]["ms_per_step"]
    line["dtype"] = {"mixed": "bf16x3-f32+f64", "fp64": "f64", "fp32": "f32"}[head]
    print(json.dumps(line), flush=True)


def bench_lasso(args, torch, spmesl, workloads):
    """The scaled lasso on its own: the regression example of Section 3
    (n = 250, p = 500, beta = (2 x 5, -1 x 5, 0 x 490)) with 256 responses on
    one design (noise levels sigma from 1 to 8), one library call per step
    (double form, tol 1e-8, lambda0 = sqrt(2 log p / n))."""
    import numpy as np
    m = 256
    X_np, Y_np, _ = workloads.sparse_regression(sigmas=np.linspace(1.0, 8.0, m))
    n, p = X_np.shape
    lam0 = math.sqrt(2 * math.log(p) / n)
    X = torch.from_numpy(X_np).to("cuda:0")
    Y = torch.from_numpy(Y_np).to("cuda:0")
    ctx = spmesl.Context(0)
    for _ in range(args.warmup):
        ctx.scaled_lasso(X, Y, lam0, 1e-8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, _, outer, st, stats = ctx.scaled_lasso(X, Y, lam0, 1e-8)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000 / args.steps
    line = {"metric": "scaled lassos/s (Section 3 regression example, 256 responses on one design)",
            "unit": "lassos/s", "value": round(m * 1000 / ms, 1), "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "lasso_n250_p500_m256", "n": n, "p": p, "responses": m,
                       "lambda0": round(lam0, 6), "tol": 1e-8},
            "status": st, "max_sigma_updates": int(outer.max().item()), "stats": stats}
    if not args.no_cpu:
        import oracle
        Xs, _, _ = oracle.standardize(X_np)
        sample = 16
        t0 = time.perf_counter()
        for r in range(0, m, m // sample):
            ys, _, _ = oracle.standardize(Y_np[:, r:r + 1])
            oracle.scaled_lasso(Xs, ys[:, 0], lam0, tol=1e-8)
        sec = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": round(sample / sec, 1), "unit": "lassos/s", "cores": 1,
                                "kind": "oracle",
                                "sample": f"every {m // sample}th of {m} responses (Algorithm 1 in residual form, "
                                          "one thread)"}
    print(f"[bench] scaled lasso: {ms:.3f} ms per {m} responses", file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


# The paper's Table 2: PCD-GPU seconds per fit (GTX 1080 Ti, double precision
# through R, lambda0 = sqrt(4 log p / n), mean of 10 data sets), by network,
# n and p.  Context only: other hardware, the paper's own generators.
TABLE2_PCD_GPU_S = {
    ("ar1", 250): (1.9528, 4.4149, 12.0651, 60.1581), ("ar1", 500): (1.7117, 4.2744, 12.8309, 64.4670),
    ("ar1", 1000): (1.7364, 4.9784, 15.8946, 85.5756),
    ("ar4", 250): (0.8794, 1.7679, 4.9945, 20.9527), ("ar4", 500): (0.9950, 2.2517, 6.2053, 26.2313),
    ("ar4", 1000): (1.5552, 4.1366, 12.1282, 57.1606),
    ("sf", 250): (1.1620, 2.9021, 6.8921, 35.0760), ("sf", 500): (1.1572, 2.9931, 8.3851, 44.9643),
    ("sf", 1000): (1.2210, 3.6376, 11.1231, 63.4638),
    ("hub", 250): (2.3266, 6.9508, 11.6372, 35.8963), ("hub", 500): (2.3915, 7.6092, 15.7290, 53.2606),
    ("hub", 1000): (2.6366, 9.6065, 21.4761, 77.6366),
}
TABLE2_P = (500, 1000, 2000, 5000)


def bench_table2(args, torch, spmesl, workloads):
    """The settings of the paper's timing table (Table 2): its four networks
    (Section 4.1), p in {500, 1000, 2000, 5000}, n in {250, 500, 1000},
    lambda0 = lambda_ub = sqrt(4 log p / n), one seeded data set per setting
    (the paper averages ten).  Each fit is one full solve (X resident, B,
    sigma and Omega written), timed one call at a time (median of --steps
    calls after --warmup), in both forms, beside the paper's seconds."""
    import numpy as np
    ctx = spmesl.Context(0)
    rows = []
    for kind in ("ar1", "ar4", "sf", "hub"):
        for pi, p in enumerate(TABLE2_P):
            om = workloads.paper_network(kind, p, np.random.default_rng(100 + pi))
            for n in (250, 500, 1000):
                X = torch.from_numpy(workloads.sample_from_precision(n, om, np.random.default_rng(n + p))).to(
                    "cuda:0")
                lam = spmesl.lambda_ub(n, p)
                row = {"network": kind, "n": n, "p": p, "lambda0": round(lam, 6),
                       "paper_pcd_gpu_s": TABLE2_PCD_GPU_S[(kind, n)][pi]}
                out = dict(B=torch.empty((p, p), dtype=torch.float64, device="cuda:0"),
                           sigma=torch.empty((p,), dtype=torch.float64, device="cuda:0"),
                           Omega=torch.empty((p, p), dtype=torch.float64, device="cuda:0"))
                for prec in ("mixed", "fp64"):
                    st = 0
                    for _ in range(args.warmup):
                        st = ctx.solve(X, lam, 1e-8, prec, out=out, check=False).status
                    per = []
                    for _ in range(args.steps):
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        st = ctx.solve(X, lam, 1e-8, prec, out=out, check=False).status
                        per.append((time.perf_counter() - t0) * 1000)
                    per.sort()
                    row[f"{prec}_ms"] = round(per[len(per) // 2], 4)
                    row[f"{prec}_status"] = st
                rows.append(row)
                print(f"[bench] table2 {kind} n={n} p={p}: mixed {row['mixed_ms']:.3f} ms, fp64 "
                      f"{row['fp64_ms']:.3f} ms (paper {row['paper_pcd_gpu_s']} s)", file=sys.stderr, flush=True)
    print(json.dumps({"table": "paper Table 2 settings", "unit": "ms per fit", "tol": 1e-8,
                      "timing": "host clock around spmesl_solve, median", "rows": rows}), flush=True)


def copy_calibration(torch):
    """A plain device-to-device copy of known size, for scaling the HBM byte
    counters (FETCH_SIZE, WRITE_SIZE) of a profiler run."""
    nbytes = 512 << 20
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 5}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="use the default launch shapes instead of the autotuner's")
    ap.add_argument("--replicas", type=int, default=8,
                    help="data sets of the headline shape in the batched figure (0 or 1: none)")
    ap.add_argument("--forms", default="mixed,fp64",
                    help="comma list of mixed, fp64, fp32, data (the double data form, no S)")
    ap.add_argument("--table2", action="store_true",
                    help="time the settings of the paper's timing table (four networks, p up to 5000)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 512 MiB device to device five times (profiler calibration)")
    ap.add_argument("--workload", default=WORKLOAD,
                    help="blockar_n400_p5000 (headline), sf_n1000_p20000, dense_n1500_p300 (every "
                         "column in the dense tier), hub_batch64, or lasso_n250_p500_m256 (the scaled "
                         "lasso on its own)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus_requested": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch
    if args.copy_calibration:
        return copy_calibration(torch)
    from paper_2203_15031_amd import spmesl, tuning, workloads

    if args.table2:
        return bench_table2(args, torch, spmesl, workloads)
    if args.workload == "hub_batch64":
        return bench_batch(args, torch, spmesl, workloads)
    if args.workload == "lasso_n250_p500_m256":
        return bench_lasso(args, torch, spmesl, workloads)
    w = workloads.workload(args.workload)
    X_np = workloads.generate(args.workload)
    X = torch.from_numpy(X_np).to("cuda:0")
    lam0, tol = w.lambda0, w.tol
    ctx = spmesl.Context(0)
    forms = args.forms.split(",")
    res = {}
    outs = {}
    tunes = {}
    for prec in forms:
        if not args.no_tune and not FORMS[prec][1]:
            # launch shapes for this problem from the autotuner (cached per
            # device, precision and shape; the tuning runs before the timed
            # region, like any one-time set-up)
            t, tms, hit = tuning.tuned(ctx, X, lam0, tol, FORMS[prec][0], reps=20)
            tunes[prec] = {"shapes": t, "ms_per_solve_when_tuned": round(tms, 5), "from_cache": hit}
            print(f"[bench] {prec}: tuned launch shapes {t} ({'cache' if hit else 'tuned here'})",
                  file=sys.stderr, flush=True)
        else:
            ctx.set_tuning(None)
        ms, ms_sync, ph, kern, r = time_form(ctx, X, lam0, tol, prec, args.steps, args.warmup, torch)
        res[prec] = (ms, ms_sync, ph, kern, r)
        outs[prec] = (r.B.cpu().numpy(), r.sigma.cpu().numpy())
        print(f"[bench] {prec}: {ms:.3f} ms/solve pipelined, {ms_sync['median']:.3f} median one call at a time; phases " +
              " ".join(f"{k}={v:.4f}" for k, v in ph.items()), file=sys.stderr, flush=True)
        print(f"[bench] {prec} kernels: " +
              " ".join(f"{k}={v['ms_per_solve']:.4f}" for k, v in kern.items()), file=sys.stderr, flush=True)

    head = forms[0]
    ms, ms_sync, ph, kern, r = res[head]
    mean_w = r.stats["sum_working_set"] / w.p if getattr(r, "stats", None) else None
    costs = kernel_costs(w.n, w.p, FORMS[head][0], mean_w) if not FORMS[head][1] else {}
    # the kernel step that takes longest per solve, among those on the
    # solver's stream (the output fill overlaps them on the second stream)
    main = {k: v for k, v in kern.items() if not k.startswith(("fill_", "wait_"))}
    dom = max(main, key=lambda k: main[k]["ms_per_solve"])
    roof = roofline_of(dom, main[dom]["ms_per_launch"], costs.get(dom, (0.0, 0.0, None)))
    if dom not in costs:
        roof["note"] = "latency-bound step with no algorithmic byte count; achieved is 0"
    on_traffic = args.workload == WORKLOAD
    roof["traffic"] = measured_traffic(dom, FORMS[head][0]) if on_traffic else None
    kernels = {}
    for k, v in kern.items():
        kernels[k] = dict(ms_per_solve=round(v["ms_per_solve"], 5), launches=v["launches"])
        if k in costs:
            rk = roofline_of(k, v["ms_per_launch"], costs[k])
            rk["traffic"] = measured_traffic(k, FORMS[head][0]) if on_traffic else None
            kernels[k]["roofline"] = rk
    line = {
        "metric": "full SPMESL solves/s at p=5000 (mixed vs FP64), % MFMA/HBM roofline",
        "value": round(1000.0 / ms, 3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "ms_per_solve_one_call_at_a_time": {k: round(v, 4) for k, v in ms_sync.items()},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPES[head],
        "data": "synthetic",
        "config": {"workload": args.workload, "n": w.n, "p": w.p, "lambda0": round(lam0, 6),
                   "tol": tol, "precision": head},
        "phases_ms": {k: round(v, 4) for k, v in ph.items()},
        "roofline": roof,
        "whole_solve": whole_solve_roofline(w.n, w.p, head, r.stats, ms) if not FORMS[head][1] else None,
        "tuning": tunes or None,
        "kernels": kernels,
        "stats": {k: r.stats[k] for k in ("total_outer", "max_outer", "total_sweeps",
                                          "total_updates", "total_rounds", "max_working_set",
                                          "columns_noconv", "polish_kkt_checks", "polish_added",
                                          "sum_working_set", "resolved_columns",
                                          "escalated_columns")},
    }
    for prec in forms[1:]:
        ms2, ms2_sync, ph2, kern2, r2 = res[prec]
        line[prec] = {"value": round(1000.0 / ms2, 3), "ms_per_step": round(ms2, 4),
                      "ms_per_solve_one_call_at_a_time": {k: round(v, 4) for k, v in ms2_sync.items()},
                      "phases_ms": {k: round(v, 4) for k, v in ph2.items()},
                      "kernels_ms": {k: round(v["ms_per_solve"], 5) for k, v in kern2.items()}}
        line[prec]["whole_solve"] = (whole_solve_roofline(w.n, w.p, prec, r2.stats, ms2)
                                     if not FORMS[prec][1] else None)
        line["speedup_vs_" + prec] = round(ms2 / ms, 3)
    if args.replicas > 1 and args.workload == WORKLOAD:
        line["batched"] = batched_replicas(args, torch, spmesl, workloads, forms, tol)
    if not args.no_cpu:
        line["errors_vs_oracle"] = errors_vs_oracle(X_np, lam0, outs)
        line["cpu_baseline"] = cpu_baseline(X_np, lam0, tol)
        line["cpu_baseline_single_thread"] = cpu_baseline_single_thread(X_np, lam0, tol)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
