#!/usr/bin/env python3
"""SpMV benchmark on one MI355X: every storage format on the two 1M-row FP64
workloads (3-D 27-point stencil on 100^3, 26,463,592 nnz; 1M x 1M with
Zipf(2) row lengths, mean 16, max 10^4, ~16M nnz).

A step is one pass of the hot path over that batch: y = A x once per
(matrix, format) pair, each launch preceded by a cache scrub (512 MB, so
neither L2 nor the 256 MB Infinity Cache holds the matrix) and bracketed by
HIP events on the launch stream.  ELL of the Zipf matrix needs 120 GB and is
refused by the library's default 64 GB cap, so a step has 9 launches.

Prints one JSON line.  `value` = algorithmic bytes of all launches of the
timed steps / their summed event time (GB/s); per-format figures are in
`per_format`; `roofline` describes the launch with the largest time share;
`cpu_baseline` times the FP64 CSR oracle on the host cores on the same two
matrices.
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
FORMATS = [("csr", {}), ("csr5", {}), ("ell", {}), ("sell", {"sell_C": 32, "sell_sigma": 1}), ("hyb", {})]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def load_tuned():
    """Tuned parameters per workload, written by the autotuner run (optional)."""
    p = os.path.join(ROOT, "paper_1805_11938_amd", "tuned_params.json")
    if os.path.exists(p):
        return json.load(open(p))
    return {}


def build_workload():
    from paper_1805_11938_amd import synth
    t0 = time.time()
    a = synth.stencil27(100, seed=2)
    xa = synth.vector(a.N, 3)
    b = synth.zipf_rows(1_000_000, 1_000_000, 2.0, 16.0, 10_000, seed=4, val_seed=5)
    xb = synth.vector(b.N, 6)
    log(f"[bench] generated workloads in {time.time() - t0:.1f}s: stencil27 nnz={a.nnz}, zipf nnz={b.nnz}")
    return [("stencil27_100", a, xa), ("zipf_1M", b, xb)]


def cpu_baseline(work, budget_s=15.0):
    """The oracle's FP64 CSR loop, OpenMP rows over the host cores."""
    import oracle
    threads = min(os.cpu_count() or 1, 16)
    tot_bytes, tot_t, reps = 0.0, 0.0, 0
    t_start = time.time()
    while time.time() - t_start < budget_s or reps < 2:
        for name, A, x in work:
            t0 = time.perf_counter()
            _, used = oracle.csr_spmv_omp(A.M, A.ptr, A.col, A.val, x, threads)
            tot_t += time.perf_counter() - t0
            tot_bytes += A.nnz * 12 + 4 * (A.M + 1) + 8 * A.N + 8 * A.M
        reps += 1
        if reps >= 20000:
            break
    return {"value": round(tot_bytes / tot_t / 1e9, 3), "unit": "GB/s", "cores": int(used), "kind": "oracle",
            "sample": f"{reps} passes of y=Ax over both full matrices (FP64 CSR loop, OpenMP static rows)",
            "ms_per_step": round(1e3 * tot_t / reps, 3)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", default="", help="comma-separated matrix/format labels to run (default: all)")
    ap.add_argument("--warm", action="store_true", help="skip the cache scrub between launches (labelled warm)")
    ap.add_argument("--copy-probe", action="store_true", help="also time a plain 1 GiB device copy")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="measured HBM bytes per launch (rocprofv3 FETCH_SIZE/WRITE_SIZE), if present")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (multi-GPU sharding is a "
              f"design note, see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1805_11938_amd import spmv as S

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    dev = torch.device("cuda:0")
    work = build_workload()
    tuned = load_tuned()

    launches = []  # (label, matrix handle, x, y, bytes_fmt, nnz)
    t0 = time.time()
    for name, A, x64 in work:
        base = S.Matrix.from_host(A, S.F64)
        x = torch.from_numpy(x64).to(dev)
        y = torch.empty(A.M, dtype=torch.float64, device=dev)
        for fmt, kw in FORMATS:
            kw = dict(kw, **tuned.get(name, {}).get(fmt, {}))
            try:
                B = base.convert(fmt, **kw)
            except S.SpmvError as e:
                log(f"[bench] {name}/{fmt}: not built ({e})")
                continue
            if args.only and f"{name}/{fmt}" not in args.only.split(","):
                continue
            launches.append(dict(label=f"{name}/{fmt}", m=B, x=x, y=y, bytes=B.info.bytes_fmt,
                                 bytes_min=B.info.bytes_min, nnz=A.nnz, params=B.params))
        del base
    torch.cuda.synchronize()
    log(f"[bench] converted {len(launches)} (matrix, format) pairs in {time.time() - t0:.1f}s")

    stream = torch.cuda.current_stream()

    def step(record):
        for L in launches:
            if not args.warm:
                S.scrub(SCRUB)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            L["m"].run(L["x"], L["y"])
            e1.record(stream)
            if record:
                L.setdefault("ev", []).append((e0, e1))

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t_wall = time.perf_counter()
    for _ in range(args.steps):
        step(True)
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
                           "params": {k: v for k, v in L["params"].items() if k != "flags"}}
        tot_b += L["bytes"] * len(ts)
        tot_t += sum(ts) * 1e-3
    value = tot_b / tot_t / 1e9
    dom = max(launches, key=lambda L: per[L["label"]]["ms"])
    dper = per[dom["label"]]
    traffic = None
    if os.path.exists(args.traffic):
        tr = json.load(open(args.traffic)).get(dom["label"])
        if tr:
            traffic = tr.get("bytes_per_launch")
    roof = {"bound": "hbm", "achieved": dper["GBps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(dper["GBps"] / HBM_PEAK_GBPS, 4), "traffic": traffic, "kernel": dom["label"],
            "bytes_per_launch": int(dom["bytes"])}
    out = {"metric": "SpMV GB/s & % HBM roofline per format; selector % of best-format throughput vs CSR",
           "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(1e3 * wall / args.steps, 4),
           "spmv_ms_per_step": round(1e3 * tot_t / args.steps, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded generators)",
           "config": {"workload": "27-pt stencil 100^3 (26.46M nnz) + Zipf(2) 1Mx1M (16M nnz), FP64, int32 "
                                  "indices, all formats, " + ("warm cache" if args.warm else "cold cache"),
                      "launches_per_step": len(launches)},
           "roofline": roof, "per_format": per}
    if args.copy_probe:
        out["copy_probe_GBps"] = round(S.copy_probe(1 << 30, 20), 1)
    if not args.no_cpu:
        log("[bench] timing the CPU oracle ...")
        out["cpu_baseline"] = cpu_baseline(work)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
