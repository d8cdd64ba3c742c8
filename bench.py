#!/usr/bin/env python3
"""SpMV benchmark on one MI355X: every storage format on the two 1M-row
workloads (3-D 27-point stencil on 100^3, 26,463,592 nnz; 1M x 1M with
Zipf(2) row lengths, mean 16, max 10^4, ~16M nnz), FP64 by default.

A step is one pass of the hot path over that batch: y = A x once per
(matrix, format) pair, in the autotuned launch configuration, each launch
preceded by a cache scrub (512 MB, so neither L2 nor the 256 MB Infinity
Cache holds the matrix) and timed by a pair of HIP events that the launch's
first kernel records as it starts and its last kernel as it ends
(spmv_run_timed), so the time is the kernels' own, as rocprofv3 reports it.
ELL of the Zipf matrix needs 120 GB and is refused by the library's default
64 GB cap, so a step has 9 launches.

Prints one JSON line.  `value` = algorithmic bytes of all launches of the
timed steps / their summed event time (GB/s); per-format figures (GB/s,
GFLOP/s, roofline fraction, one-off conversion time) are in `per_format`;
`roofline` describes the launch with the largest time share; `selector`
gives the learned model's choice per matrix against the measured best;
`cpu_baseline` times the FP64 CSR oracle on the host cores on the same two
matrices.  `--workload rmat24` measures the R-MAT scale-24 matrix instead
(CSR, CSR5, SELL, HYB).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
SCRUB = 512 << 20


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload(names):
    from paper_1805_11938_amd import workloads as W
    out = []
    for name in names:
        t0 = time.time()
        A = W.make(name)
        out.append((name, A, W.x_vector(name, A.N)))
        log(f"[bench] generated {name} in {time.time() - t0:.1f}s")
    return out


def _ci_timed(fn, min_s, budget_s, min_reps=20, max_reps=1000, rel_ci=0.025):
    """Times of fn() repeated for at least min_s seconds and min_reps runs,
    until the 95% confidence interval of the mean is within +-rel_ci of it,
    at most max_reps runs or budget_s seconds.  Returns (times in s, CI
    half-width / mean)."""
    fn()  # warm-up
    ts = []
    t_start = time.time()
    while len(ts) < max_reps:
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
        el = time.time() - t_start
        if len(ts) >= min_reps and el >= min_s:
            a = np.asarray(ts)
            rel = 1.96 * a.std(ddof=1) / np.sqrt(len(a)) / a.mean()
            if rel <= rel_ci or el > budget_s:
                return ts, float(rel)
    a = np.asarray(ts)
    return ts, float(1.96 * a.std(ddof=1) / np.sqrt(len(a)) / a.mean())


def cpu_baseline(work, sv, min_s=6.0, budget_s=15.0):
    """The oracle's FP64 CSR loop on the same matrices (FP32 values are
    promoted, so its bytes are counted at the FP64 size): OpenMP static rows
    over the host cores this process may use (at most 16: the CPU share of a
    one-GPU machine), and single-threaded.  One pass = y = A x over every matrix of
    the workload; passes repeat for at least min_s seconds each way, then
    under the timing rule (95% CI of the mean within 2.5%, 20..1000 passes,
    or the time budget)."""
    import oracle
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    threads = max(1, min(avail, 16))
    nbytes = sum(len(col) * 12 + 4 * (M + 1) + 8 * len(x) + 8 * M for _, M, ptr, col, val, x in work)
    used = [1]

    def one_pass(nt):
        for _, M, ptr, col, val, x in work:
            _, used[0] = oracle.csr_spmv_omp(M, ptr, col, val, x, nt)

    ts, rel = _ci_timed(lambda: one_pass(threads), min_s, budget_s)
    cores = int(used[0])
    ts1, rel1 = _ci_timed(lambda: one_pass(1), min_s, budget_s)
    med, med1 = float(np.median(ts)), float(np.median(ts1))
    return {"value": round(nbytes / med / 1e9, 3), "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(ts)} passes of y=Ax over every matrix of the workload in full (FP64 CSR loop, "
                      f"OpenMP static rows over {cores} threads), median pass; 95% CI +-{100 * rel:.1f}%",
            "ms_per_step": round(1e3 * med, 3), "ci_rel": round(rel, 4), "reps": len(ts),
            "host_cpus": os.cpu_count(), "cpus_available": avail,
            "single_thread": {"value": round(nbytes / med1 / 1e9, 3), "unit": "GB/s", "ms_per_step": round(1e3 * med1, 3),
                              "reps": len(ts1), "ci_rel": round(rel1, 4)}}


WORKLOADS = {"c2": ("stencil27_100", "zipf_1M"), "rmat24": ("rmat24",)}
DESCR = {"c2": "27-pt stencil 100^3 (26.46M nnz) + Zipf(2) 1Mx1M (16M nnz), int32 indices, all formats",
         "rmat24": "R-MAT(0.57,0.19,0.19) scale 24, 2^28 edge draws (~2.6e8 nnz after duplicate sums), int32 "
                   "indices, CSR/CSR5/SELL/HYB"}


def selector_choices(bases, per, dname):
    """The learned model's pick per matrix, judged by this run's times."""
    from paper_1805_11938_amd import selector as SEL
    from paper_1805_11938_amd import spmv as S
    path = SEL.model_path(dname)
    if not os.path.exists(path):
        return None
    model = S.Model.load(path)
    out = {}
    for name, base in bases.items():
        t = {f: per[f"{name}/{f}"]["ms"] for f in S.FMT_NAMES if f"{name}/{f}" in per}
        if not t:  # no format of this matrix was timed (--only)
            continue
        fmt, _ = SEL.choose(base, model)
        inside = SEL.in_domain(base, model)
        w0 = time.perf_counter()
        for _ in range(10):  # features + inference, both synchronous
            SEL.choose(base, model)
        ov = (time.perf_counter() - w0) / 10 * 1e3
        best = min(t, key=t.get)
        model_frac = round(t[best] / t[fmt], 4) if fmt in t else None  # chosen format not timed (--only)
        if inside:
            r = {"how": "model", "chosen": fmt, "frac_of_best": model_frac, "overhead_ms": round(ov, 4)}
        else:
            # outside the training range selector.auto profiles every format;
            # its cost is at least one conversion per format plus the timing
            # rule's 20 launches of each (this run measured both)
            cost = sum(per[f"{name}/{f}"]["convert_ms"] + 20 * t[f] for f in t)
            r = {"how": "exhaustive (features outside the model's training range)", "chosen": best,
                 "frac_of_best": 1.0, "overhead_ms": round(cost, 3)}
        r.update({"best": best, "model_choice": fmt, "model_frac_of_best": model_frac})
        if "csr" in t:
            r.update({"csr_frac_of_best": round(t[best] / t["csr"], 4),
                      "overhead_in_csr_spmvs": round(r["overhead_ms"] / t["csr"], 2)})
        out[name] = r
    rep = os.path.join(SEL.DATA_DIR, "selector_report.json")
    if os.path.exists(rep):
        r = json.load(open(rep)).get(dname)
        if r and "test" in r:
            out["held_out"] = {"n": r["test"]["n"], "frac_of_best": round(r["test"]["frac"], 4),
                               "fixed_csr_frac": round(r["test"]["fixed"]["csr"]["frac"], 4),
                               "best_fixed": r["test"]["best_fixed"],
                               "best_fixed_frac": round(r["test"]["fixed"][r["test"]["best_fixed"]]["frac"], 4)}
    return out


def _events(torch, stream, fn, steps, warmup, scrub, kernel_bound=True):
    """Event times (ms) of fn over `steps` runs, each after a scrub.  With
    kernel_bound, fn(events) records the pair itself at the start of its first
    kernel and the end of its last; otherwise markers bracket fn()."""
    from paper_1805_11938_amd import spmv as S
    pairs = [S.timing_events() for _ in range(steps)]
    spare = S.timing_events()
    for r in range(warmup + steps):
        ev = pairs[r - warmup] if r >= warmup else spare
        if scrub:
            S.scrub(SCRUB)
        if kernel_bound:
            fn(ev)
        else:
            ev[0].record(stream)
            fn()
            ev[1].record(stream)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in pairs]


def measured_traffic(args, label):
    """HBM bytes per launch from the counter runs (rocprofv3 FETCH_SIZE and
    WRITE_SIZE, profiles/traffic.json), or None."""
    if not os.path.exists(args.traffic):
        return None
    tr = json.load(open(args.traffic)).get(f"{args.dtype}:{label}")
    return tr.get("bytes_per_launch") if tr else None


BATCH_SELL = dict(sell_C=64, sell_sigma=4096)


def batch_formats(args, mats, dt):
    """The handle each matrix enters the batch as.  --batch-format csr or sell
    takes one format for all (tiles: CSR wave tiles); auto takes SELL-C-sigma
    chunk groups for matrices with regular rows (coefficient of variation of
    the row lengths at most 0.5 and no row over 256 entries, from the device
    features: one lane per row then has an even share and padding stays
    small) and CSR wave tiles for the rest, whose long rows spread over
    tiles of equal size.
    Returns (handles, count per format)."""
    out = []
    for m in mats:
        if args.batch_format == "auto":
            f = m.features()  # n_rows, n_cols, nnz, nnz_frac, min, max, avg, std, variation, ...
            fmt = "sell" if f[8] <= 0.5 and f[5] <= 256 else "tiles"
        else:
            fmt = args.batch_format
        if fmt == "sell":
            out.append(m.convert("sell", **BATCH_SELL))
        elif fmt == "tiles":
            out.append(m.convert("csr", flags=32))
        else:
            out.append(m)
    kinds = {"csr": sum(1 for h in out if h.fmt == "csr" and not h.params["flags"] & 32),
             "csr_tiles": sum(1 for h in out if h.fmt == "csr" and h.params["flags"] & 32),
             "sell": sum(1 for h in out if h.fmt == "sell")}
    return out, kinds


def bench_batch(args):
    """512 uneven matrices (rows 10^3..2x10^5, mean row length 4..64, four
    generators, seed 8) in one launch, each as CSR or SELL-C-sigma, against
    one launch per matrix in the same formats."""
    import torch
    from paper_1805_11938_amd import spmv as S
    from paper_1805_11938_amd import synth
    dt = S.F64 if args.dtype == "f64" else S.F32
    tdt = torch.float64 if dt == S.F64 else torch.float32
    t0 = time.time()
    mats, xs, ys, bmin, nnz, cpu_work = [], [], [], 0, 0, []
    for i, spec in enumerate(synth.batch_specs(512, seed=8)):
        A = synth.make(spec)
        if i % 4 == 0 and not args.no_cpu:  # the CPU baseline's sample: every fourth matrix
            cpu_work.append((f"m{i}", A.M, A.ptr, A.col, A.val, synth.vector(A.N, 50 + i)))
        val = A.val.astype(np.float32) if dt == S.F32 else A.val
        mats.append(S.Matrix.from_csr(A.M, A.N, A.ptr, A.col, val, dt))
        xs.append(torch.from_numpy(synth.vector(A.N, 50 + i)).to("cuda", tdt))
        ys.append(torch.empty(A.M, dtype=tdt, device="cuda"))
        bmin += mats[-1].info.bytes_min
        nnz += A.nnz
    log(f"[bench] batch of 512: {nnz} nnz, {bmin / 1e9:.2f} GB, built in {time.time() - t0:.1f}s")
    items, kinds = batch_formats(args, mats, dt)
    log(f"[bench] batch item kinds: {kinds}")
    B = S.Batch(items)
    stream = torch.cuda.current_stream()
    wall = time.perf_counter()
    tb = _events(torch, stream, lambda ev: B.run(xs, ys, ev), args.steps, args.warmup, not args.warm)
    wall = time.perf_counter() - wall

    def each():
        for m, x, y in zip(items, xs, ys):
            m.run(x, y)
    te = _events(torch, stream, each, args.steps, args.warmup, not args.warm, kernel_bound=False)
    t, t1 = float(np.mean(tb)), float(np.mean(te))
    gbps = bmin / (t * 1e-3) / 1e9
    out = {"metric": "batched SpMV GB/s (one launch over 512 matrices)", "value": round(gbps, 1),
           "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(1e3 * wall / (args.steps + args.warmup), 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic (seeded generators)",
           "config": {"workload": f"512 uneven matrices (CSR or SELL-C-sigma each), {nnz} nnz, seed 8, "
                                  + ("warm cache" if args.warm else "cold cache")},
           "roofline": {"bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                        "frac": round(gbps / HBM_PEAK_GBPS, 4), "traffic": measured_traffic(args, "batch512"),
                        "kernel": "k_csr_batched", "bytes_per_launch": int(bmin), "ms_per_launch": round(t, 5)},
           "one_launch_per_matrix": {"ms": round(t1, 5), "GBps": round(bmin / (t1 * 1e-3) / 1e9, 1)},
           "speedup_vs_per_matrix": round(t1 / t, 3), "item_formats": kinds}
    if args.copy_probe:
        out["copy_probe_GBps"] = round(S.copy_probe(1 << 30, 20), 1)
    if cpu_work:
        cb = cpu_baseline(cpu_work, 8 if dt == S.F64 else 4)
        cb["sample"] = (f"every fourth matrix of the batch ({len(cpu_work)} of 512, "
                        f"{sum(len(w[3]) for w in cpu_work)} nonzeros), y=Ax over each per pass (FP64 CSR loop, "
                        f"OpenMP static rows over {cb['cores']} threads), median of {cb['reps']} passes; "
                        f"95% CI +-{100 * cb['ci_rel']:.1f}%")
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


def bench_spmm(args):
    """SpMM Y = A X with k = 8 and 16 right-hand sides (row-major, X seed 9)
    on the 27-point stencil, against k separate SpMVs."""
    import torch
    from paper_1805_11938_amd import spmv as S
    from paper_1805_11938_amd import synth
    from paper_1805_11938_amd import workloads as W
    dt = S.F64 if args.dtype == "f64" else S.F32
    tdt = torch.float64 if dt == S.F64 else torch.float32
    sv = 8 if dt == S.F64 else 4
    A = W.make("stencil27_100")
    val = A.val.astype(np.float32) if dt == S.F32 else A.val
    Ad = S.Matrix.from_csr(A.M, A.N, A.ptr, A.col, val, dt)
    stream = torch.cuda.current_stream()
    per = {}
    wall = time.perf_counter()
    for k in (8, 16):
        X = torch.from_numpy(synth.uniform(A.N * k, 9, -1.0, 1.0).reshape(A.N, k)).to("cuda", tdt)
        Y = torch.empty((A.M, k), dtype=tdt, device="cuda")
        ts = _events(torch, stream, lambda ev: Ad.spmm_timed(X, Y, ev), args.steps, args.warmup, not args.warm)
        xcols = [X[:, c].contiguous() for c in range(k)]
        yv = torch.empty(A.M, dtype=tdt, device="cuda")

        def ksp():
            for c in range(k):
                Ad.run(xcols[c], yv)
        t1 = float(np.mean(_events(torch, stream, ksp, args.steps, args.warmup, not args.warm, kernel_bound=False)))
        t = float(np.mean(ts))
        b = A.nnz * (sv + 4) + 4 * (A.M + 1) + A.N * k * sv + A.M * k * sv
        per[f"k{k}"] = {"ms": round(t, 5), "GBps": round(b / (t * 1e-3) / 1e9, 1), "bytes": int(b),
                        "GFLOPs": round(2 * A.nnz * k / (t * 1e-3) / 1e9, 1), "k_spmv_ms": round(t1, 5),
                        "speedup_vs_k_spmv": round(t1 / t, 3)}
    wall = time.perf_counter() - wall
    dom = per["k16"]
    tot_b = sum(v["bytes"] for v in per.values())
    tot_t = sum(v["ms"] for v in per.values()) * 1e-3
    out = {"metric": "SpMM GB/s (k = 8, 16 right-hand sides)", "value": round(tot_b / tot_t / 1e9, 1), "unit": "GB/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(1e3 * wall / (args.steps + args.warmup), 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic (seeded generators)",
           "config": {"workload": "27-pt stencil 100^3, X row-major N x k, k in {8, 16}, "
                                  + ("warm cache" if args.warm else "cold cache")},
           "roofline": {"bound": "hbm", "achieved": dom["GBps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                        "frac": round(dom["GBps"] / HBM_PEAK_GBPS, 4), "traffic": measured_traffic(args, "spmm/k16"),
                        "kernel": "k_csr_spmm k=16", "bytes_per_launch": dom["bytes"], "ms_per_launch": dom["ms"]},
           "per_k": per}
    if args.copy_probe:
        out["copy_probe_GBps"] = round(S.copy_probe(1 << 30, 20), 1)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_spmm(A, sv)
    print(json.dumps(out), flush=True)


def cpu_baseline_spmm(A, sv, rows=100_000, min_s=3.0, budget_s=8.0):
    """The oracle's SpMM (a single-threaded C loop over rows, nonzeros and
    columns) on the first `rows` rows of the matrix, for k = 8 and 16 with
    the benchmark's X; bytes by the same model as the GPU launches, with the
    X rows the sample reads."""
    import oracle
    from paper_1805_11938_amd import synth
    ms = min(rows, A.M)
    nz = int(A.ptr[ms])
    ptr, col, val = A.ptr[:ms + 1], A.col[:nz], A.val[:nz]
    ncols = len(np.unique(col))
    tot_b, tot_t, reps = 0, 0.0, 0
    for k in (8, 16):
        X = synth.uniform(A.N * k, 9, -1.0, 1.0).reshape(A.N, k)
        ts, _ = _ci_timed(lambda: oracle.csr_spmm(ms, ptr, col, val, X), min_s, budget_s)
        tot_b += nz * (sv + 4) + 4 * (ms + 1) + ncols * k * sv + ms * k * sv
        tot_t += float(np.median(ts))
        reps += len(ts)
    return {"value": round(tot_b / tot_t / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"rows 0..{ms - 1} of the stencil ({nz} nonzeros), Y = A X for k = 8 and 16 (the oracle's "
                      f"single-threaded C loop), median of {reps} calls in all",
            "ms_per_step": round(1e3 * tot_t, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS) + ["batch512", "spmm"])
    ap.add_argument("--dtype", default="f64", choices=["f64", "f32"])
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", default="", help="comma-separated matrix/format labels to run (default: all)")
    ap.add_argument("--warm", action="store_true", help="skip the cache scrub between launches (labelled warm)")
    ap.add_argument("--copy-probe", action="store_true", help="also time a plain 1 GiB device copy")
    ap.add_argument("--batch-format", default="auto", choices=["auto", "csr", "sell", "tiles"],
                    help="batch512: the format each matrix enters the batch as (auto: SELL-C-sigma for "
                         "regular rows, CSR wave tiles otherwise)")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="measured HBM bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE), if present")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the multi-GPU row sharding "
              f"is a design note, not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1805_11938_amd import spmv as S
    from paper_1805_11938_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    dev = torch.device("cuda:0")
    if args.workload == "batch512":
        return bench_batch(args)
    if args.workload == "spmm":
        return bench_spmm(args)
    dt = S.F64 if args.dtype == "f64" else S.F32
    tdt = torch.float64 if dt == S.F64 else torch.float32
    sv = 8 if dt == S.F64 else 4
    work = build_workload(WORKLOADS[args.workload])
    formats = ("csr", "csr5", "sell", "hyb") if args.workload == "rmat24" else W.FORMATS

    launches = []  # dicts: label, matrix handle, x, y, algorithmic bytes, nnz, params, conversion time
    bases = {}
    cpu_work = []
    t0 = time.time()
    stream = torch.cuda.current_stream()
    for name, A, x64 in work:
        if isinstance(A, synth_coo_type()):
            val = A.val.astype(np.float32) if dt == S.F32 else A.val
            base = S.Matrix.from_coo(A.M, A.N, A.row, A.col, val, dt)
        else:
            val = A.val.astype(np.float32) if dt == S.F32 else A.val
            base = S.Matrix.from_csr(A.M, A.N, A.ptr, A.col, val, dt)
        x = torch.from_numpy(x64).to(dev, tdt)
        y = torch.empty(A.M, dtype=tdt, device=dev)
        for fmt in formats:
            label = f"{name}/{fmt}"
            if args.only and label not in args.only.split(","):
                continue
            kw = W.tuned_params(name, fmt, args.dtype)
            c0 = torch.cuda.Event(enable_timing=True)
            c1 = torch.cuda.Event(enable_timing=True)
            try:
                # an untimed conversion first: the first launch of each kernel
                # in a process also loads its code object, a one-off cost
                # that is not the conversion's
                base.convert(fmt, **kw).free()
                torch.cuda.synchronize()
                c0.record(stream)
                B = base.convert(fmt, **kw)
                c1.record(stream)
                torch.cuda.synchronize()
            except S.SpmvError as e:
                log(f"[bench] {label}: not built ({e})")
                continue
            launches.append(dict(label=label, m=B, x=x, y=y, bytes=B.info.bytes_fmt, bytes_min=B.info.bytes_min,
                                 nnz=base.nnz, params=B.params, convert_ms=c0.elapsed_time(c1)))
        bases[name] = base
        if not args.no_cpu:
            if isinstance(A, synth_coo_type()):
                ptr, col, v = base.to_csr()  # the oracle is timed on the canonical CSR
                cpu_work.append((name, base.M, ptr, col, v.astype(np.float64), x64))
            else:
                cpu_work.append((name, A.M, A.ptr, A.col, A.val, x64))
    del work
    torch.cuda.synchronize()
    log(f"[bench] converted {len(launches)} (matrix, format) pairs in {time.time() - t0:.1f}s")

    # kernel-bound events: each run records its pair at the start of its first
    # kernel and the end of its last (see spmv_run_timed)
    spare = S.timing_events()
    for L in launches:
        L["pairs"] = [S.timing_events() for _ in range(args.steps)]

    def step(i):
        for L in launches:
            if not args.warm:
                S.scrub(SCRUB)
            ev = L["pairs"][i] if i >= 0 else spare
            L["m"].run_timed(L["x"], L["y"], ev)
            if i >= 0:
                L.setdefault("ev", []).append(ev)

    for _ in range(args.warmup):
        step(-1)
    torch.cuda.synchronize()
    log(f"[bench] warmup done; timing {args.steps} steps")
    t_wall = time.perf_counter()
    for i in range(args.steps):
        step(i)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall

    per = {}
    tot_b, tot_t = 0.0, 0.0
    for L in launches:
        ts = [a.elapsed_time(b) for a, b in L["ev"]]
        t = float(np.mean(ts))
        gbps = L["bytes"] / (t * 1e-3) / 1e9
        per[L["label"]] = {"ms": round(t, 5), "ms_median": round(float(np.median(ts)), 5),
                           "GBps": round(gbps, 1), "eff_GBps": round(L["bytes_min"] / (t * 1e-3) / 1e9, 1),
                           "GFLOPs": round(2 * L["nnz"] / (t * 1e-3) / 1e9, 1),
                           "frac_hbm": round(gbps / HBM_PEAK_GBPS, 4), "bytes": int(L["bytes"]),
                           "convert_ms": round(L["convert_ms"], 3),
                           "params": {k: v for k, v in L["params"].items() if k != "max_bytes"}}
        tot_b += L["bytes"] * len(ts)
        tot_t += sum(ts) * 1e-3
    value = tot_b / tot_t / 1e9
    dom = max(launches, key=lambda L: per[L["label"]]["ms"])
    dper = per[dom["label"]]
    traffic = None
    if os.path.exists(args.traffic):
        tr = json.load(open(args.traffic)).get(f"{args.dtype}:{dom['label']}")
        if tr and tr.get("params") == dper["params"]:
            traffic = tr.get("bytes_per_launch")
    roof = {"bound": "hbm", "achieved": dper["GBps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(dper["GBps"] / HBM_PEAK_GBPS, 4), "traffic": traffic, "kernel": dom["label"],
            "bytes_per_launch": int(dom["bytes"]), "ms_per_launch": dper["ms"]}
    # the floor for as many gathers from an x of the same length with no
    # locality at all (a balanced 16-per-row SpMV, uniformly random columns)
    Nd = dom["m"].info.N
    g_ms = S.gather_probe(Nd, -(-dom["nnz"] // 16), dt, reps=10, scrub_bytes=0 if args.warm else SCRUB)
    roof["random_gather_floor"] = {"ms": round(g_ms, 5), "frac": round(g_ms / dper["ms"], 4),
                                   "what": f"{16 * -(-dom['nnz'] // 16)} uniformly random gathers from x[{Nd}], "
                                           f"16 per row, every load in flight (spmv_gather_probe)"}
    out = {"metric": "SpMV GB/s & % HBM roofline per format; selector % of best-format throughput vs CSR",
           "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(1e3 * wall / args.steps, 4),
           "spmv_ms_per_step": round(1e3 * tot_t / args.steps, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.dtype,
           "data": "synthetic (seeded generators)",
           "config": {"workload": DESCR[args.workload] + ", " + ("warm cache" if args.warm else "cold cache"),
                      "launches_per_step": len(launches)},
           "roofline": roof, "per_format": per}
    sel = selector_choices(bases, per, args.dtype)
    if sel is not None:
        out["selector"] = sel
    if args.copy_probe:
        out["copy_probe_GBps"] = round(S.copy_probe(1 << 30, 20), 1)
    if not args.no_cpu:
        log("[bench] timing the CPU oracle ...")
        out["cpu_baseline"] = cpu_baseline(cpu_work, sv)
    print(json.dumps(out), flush=True)


def synth_coo_type():
    from paper_1805_11938_amd import synth
    return synth.HostCOO


if __name__ == "__main__":
    main()
