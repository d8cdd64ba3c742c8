"""Summaries of rocprofv3 output for the benchmark's launches.

Two uses:

* ``stats``: per-kernel call counts and average durations from a
  ``--kernel-trace --stats`` run (``*_kernel_stats.csv``), as text;
  ``launches``: the span of each benchmark launch in the same run's trace
  (``*_kernel_trace.csv``).
* ``traffic``: HBM bytes per benchmark launch from two counter runs
  (``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``; both counters are KiB per
  dispatch).  The benchmark scrubs the caches before every launch, so the
  dispatches between two scrub kernels belong to one (matrix, format)
  launch, in the order the benchmark prints.  The counters are calibrated
  on a kernel whose traffic is known: the 1 GiB copy probe (1 GiB read,
  1 GiB written; ``bench.py --copy-probe``).

* ``gather``: the random-gather floor (``spmv_gather_probe``) for x of
  1, 4, 8 and 16 MB and 16.7 million gathers, FP64 and FP32 (needs the GPU).

    python -m paper_1805_11938_amd.profiling stats DIR/..._kernel_stats.csv
    python -m paper_1805_11938_amd.profiling launches DIR/..._kernel_trace.csv BENCH.json
    python -m paper_1805_11938_amd.profiling traffic FETCH.csv WRITE.csv BENCH.json OUT.json
    python -m paper_1805_11938_amd.profiling gather
"""
from __future__ import annotations

import collections
import csv
import json
import math
import os
import sys

SCRUB = "k_scrub"
COPY = "k_copy"
# kernels that spmv_run launches (conversion, feature and selection kernels
# run outside the scrubbed launches and are not counted)
RUN_KERNELS = ("k_csr_rows", "k_csr_waves", "k_csr_long_fix", "k_csr_vector", "k_csr5", "k_csr5_fix", "k_csr5_fix_short",
               "k_ell", "k_ell2", "k_ell_kc", "k_ell_kc4", "k_sell", "k_sell_kc", "k_sell_kcw", "k_sell_mixed", "k_sell_fix",
               "k_coo_tiles", "k_tile_fix", "k_csr_tiles", "k_csr_spmm", "k_csr_batched", "k_batch_tile_fix")


def _short(name: str) -> str:
    return name.split("(")[0].replace("void ", "").strip()


def stats(path: str, top: int = 40) -> str:
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"{'kernel':70s} {'calls':>7s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'total_%':>8s}"]
    for r in rows[:top]:
        out.append(f"{_short(r['Name'])[:70]:70s} {int(r['Calls']):7d} {float(r['AverageNs']) / 1e3:10.2f} "
                   f"{float(r['MinNs']) / 1e3:10.2f} {float(r['MaxNs']) / 1e3:10.2f} {float(r['Percentage']):8.2f}")
    return "\n".join(out)


def _per_dispatch(path: str, counter: str):
    """[(dispatch id, kernel, value in bytes)] in dispatch order."""
    vals = collections.OrderedDict()
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        d = int(r["Dispatch_Id"])
        k = _short(r["Kernel_Name"])
        v = float(r["Counter_Value"]) * 1024.0
        if d in vals:
            vals[d] = (k, vals[d][1] + v)
        else:
            vals[d] = (k, v)
    return [(d, k, v) for d, (k, v) in sorted(vals.items())]


def _segments(disp):
    """Groups of consecutive dispatches that follow a scrub kernel."""
    segs, cur = [], None
    for d, k, v in disp:
        if SCRUB in k:
            if cur:
                segs.append(cur)
            cur = []
        elif cur is not None and k.split("<")[0].split("::")[-1] in RUN_KERNELS:
            cur.append((k, v))
    if cur:
        segs.append(cur)
    return segs


def _calibration(disp):
    copy = [v for _, k, v in disp if COPY in k]
    if not copy:
        raise ValueError("no copy-probe dispatches: run the benchmark with --copy-probe")
    return float(sum(copy) / len(copy)), float(1 << 30), COPY


def _launches(bench):
    """(label, algorithmic bytes, params, kernel that marks its launches) of
    a benchmark line, in the order the benchmark runs them.  The SpMM line
    runs k = 8 then k = 16 (each followed by k separate SpMVs, whose launches
    hold no SpMM kernel); the batch line one batched launch per step."""
    if "per_format" in bench:
        return [(lab, v["bytes"], v["params"], None) for lab, v in bench["per_format"].items()]
    if "per_k" in bench:
        return [(f"spmm/{kk}", v["bytes"], None, "k_csr_spmm") for kk, v in bench["per_k"].items()]
    return [("batch512", bench["roofline"]["bytes_per_launch"], None, "k_csr_batched")]


def traffic(fetch_csv: str, write_csv: str, bench_json: str, out_json: str, merge: bool = True):
    """HBM bytes per launch of the benchmark line in bench_json; with merge,
    the entries are added to those already in out_json."""
    bench = json.loads(open(bench_json).read().strip().splitlines()[-1])
    launches = _launches(bench)
    dt = bench["dtype"]
    F = _per_dispatch(fetch_csv, "FETCH_SIZE")
    Wr = _per_dispatch(write_csv, "WRITE_SIZE")
    fm, fk, fsrc = _calibration(F)
    wm, wk, wsrc = _calibration(Wr)
    ff, wf = fk / fm, wk / wm
    sf, sw = _segments(F), _segments(Wr)
    mark = launches[0][3]
    if mark:  # keep the launches of the marking kernel only
        sf = [g for g in sf if any(mark in k for k, _ in g)]
        sw = [g for g in sw if any(mark in k for k, _ in g)]
    n = len(launches)
    if len(sf) < n or len(sf) % n or len(sw) != len(sf):
        raise ValueError(f"{len(sf)} launches in the FETCH run, {len(sw)} in the WRITE run, {n} labels")
    res = json.load(open(out_json)) if merge and os.path.exists(out_json) else {}
    res["_calibration"] = {"fetch_factor": ff, "write_factor": wf, "kernel": fsrc,
                           "fetch_raw_bytes": fm, "write_raw_bytes": wm, "known_bytes": fk}
    per = len(sf) // n
    for i, (lab, alg, params, m) in enumerate(launches):
        # per-format lines interleave their launches; marked lines run each
        # label's launches back to back
        idx = range(i * per, (i + 1) * per) if m else range(i, len(sf), n)
        fb = [sum(v for _, v in sf[j]) for j in idx]
        wb = [sum(v for _, v in sw[j]) for j in idx]
        fetch = ff * sum(fb) / len(fb)
        write = wf * sum(wb) / len(wb)
        res[f"{dt}:{lab}"] = {"bytes_per_launch": int(round(fetch + write)), "fetch_bytes": int(round(fetch)),
                              "write_bytes": int(round(write)), "algorithmic_bytes": alg,
                              "ratio": round((fetch + write) / alg, 4),
                              "kernels": sorted({k for j in idx for k, _ in sf[j]}), "params": params}
    json.dump(res, open(out_json, "w"), indent=1)
    return res


def launches(trace_csv: str, bench_json: str) -> str:
    """Per benchmark launch: the span from the first run kernel's start to
    the last one's end, from a --kernel-trace run of the benchmark (its
    launches follow the scrub kernels in the benchmark's order), next to the
    same run's kernel-bound event times and algorithmic bytes."""
    bench = json.loads(open(bench_json).read().strip().splitlines()[-1])
    labs = _launches(bench)
    rows = sorted(csv.DictReader(open(trace_csv)), key=lambda r: int(r["Dispatch_Id"]))
    segs, cur = [], None
    for r in rows:
        k = _short(r["Kernel_Name"])
        if SCRUB in k:
            if cur:
                segs.append(cur)
            cur = []
        elif cur is not None and k.split("<")[0].split("::")[-1] in RUN_KERNELS:
            cur.append((k, int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    if cur:
        segs.append(cur)
    mark = labs[0][3]
    if mark:
        segs = [g for g in segs if any(mark in k for k, _, _ in g)]
    n = len(labs)
    if len(segs) < n or len(segs) % n:
        raise ValueError(f"{len(segs)} launches in the trace for {n} labels")
    per = len(segs) // n
    out = ["| launch | kernels | rocprofv3 µs | benchmark events µs | algorithmic MB | GB/s (rocprof) |",
           "|---|---|---|---|---|---|"]
    for i, (lab, alg, _, m) in enumerate(labs):
        idx = range(i * per, (i + 1) * per) if m else range(i, len(segs), n)
        spans = [(segs[j][-1][2] - segs[j][0][1]) / 1e3 for j in idx]
        us = sum(spans) / len(spans)
        ks = {}  # kernel -> launches of it in one run (one per column band)
        for k, _, _ in segs[idx[0]]:
            ks[k] = ks.get(k, 0) + 1
        names = ", ".join(k if c == 1 else f"{k} ×{c}" for k, c in ks.items())
        ev = bench["per_format"][lab]["ms"] * 1e3 if "per_format" in bench else math.nan
        out.append(f"| {lab} | {names} | {us:.2f} | {ev:.2f} | {alg / 1e6:.1f} | {alg / us / 1e3:.0f} |")
    return "\n".join(out)


def main(argv):
    if argv[0] == "stats":
        print(stats(argv[1]))
    elif argv[0] == "launches":
        print(launches(argv[1], argv[2]))
    elif argv[0] == "traffic":
        r = traffic(*argv[1:5])
        labels = {f"{json.loads(open(argv[3]).read().strip().splitlines()[-1])['dtype']}:{lab}"
                  for lab, _, _, _ in _launches(json.loads(open(argv[3]).read().strip().splitlines()[-1]))}
        for k, v in r.items():
            if k.startswith("_"):
                print(k, v)
            elif k in labels:
                print(f"{k:40s} measured {v['bytes_per_launch'] / 1e6:10.1f} MB  algorithmic "
                      f"{v['algorithmic_bytes'] / 1e6:10.1f} MB  ratio {v['ratio']:.3f}")
    elif argv[0] == "gather":
        import torch
        from . import spmv as S
        assert torch.cuda.is_available(), "the gather probe needs the GPU"
        rows = 1 << 20
        print(f"random-gather floor: {16 * rows} gathers (16 per row, every load in flight), cold caches, "
              f"median of 10")
        print("| x bytes | x entries | dtype | ms | G gathers/s |")
        print("|---|---|---|---|---|")
        for dname, dt, sv in (("f64", S.F64, 8), ("f32", S.F32, 4)):
            for mb in (1, 4, 8, 16):
                nx = (mb << 20) // sv
                ms = S.gather_probe(nx, rows, dt, reps=10)
                print(f"| {mb} MiB | {nx} | {dname} | {ms:.4f} | {16 * rows / (ms * 1e-3) / 1e9:.1f} |", flush=True)
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
