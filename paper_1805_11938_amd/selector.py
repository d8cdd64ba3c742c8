"""Adaptive format selection (Sec. V of arXiv 1805.11938), on the GPU.

Pipeline (Sec. V-A, V-B): profile every format on training matrices and
label each matrix with its fastest format (a); extract static features and
scale them with the training set's min and max; train a classifier (b);
at run time: features -> scaled -> model -> format -> convert -> run (c).

The classifier is the multilayer perceptron that Sec. V-D lists among the
alternatives (12 -> 64 -> 64 -> 5, trained with Adam); training runs in the
library's HIP kernels (spmv_mlp_train), features come from spmv_features,
scaling from spmv_feature_range / spmv_scale_features, inference from
spmv_select.  This module is the driver: it loops, splits and records.

Labels follow the timing rule of Sec. V-B: a format's time is the median of
cold-cache launches repeated until the 95% confidence interval is within 5%
of the mean (20..200 launches); formats whose storage exceeds the byte cap
(ELL on skewed rows) get +inf.  Ties go to the lower class index.

    python -m paper_1805_11938_amd.selector collect --start 0 --stop 3000 --out ds.jsonl
    python -m paper_1805_11938_amd.selector train --dataset ds.jsonl --out-dir DIR
"""
from __future__ import annotations

import argparse
import json
import math
import os
import queue
import sys
import threading
import time

import numpy as np

from . import spmv as S
from . import synth

CLASSES = S.FMT_NAMES
HERE = os.path.dirname(os.path.abspath(__file__))
DATA_DIR = os.path.join(HERE, "data")
SCRUB = 512 << 20
COLLECT_CAP = 8 << 30  # padded formats above 8 GiB are treated as infeasible (time = inf)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# ----------------------------------------------------------- collection

def _to_device(A, dt):
    """Handle for a generated matrix: raw R-MAT triplets go through the
    device COO -> CSR canonicalisation; the other generators emit CSR."""
    if isinstance(A, synth.HostCOO):
        val = A.val.astype(np.float32) if dt == S.F32 else A.val
        return S.Matrix.from_coo(A.M, A.N, A.row, A.col, val, dt)
    val = A.val.astype(np.float32) if dt == S.F32 else A.val
    return S.Matrix.from_csr(A.M, A.N, A.ptr, A.col, val, dt)


def profile_matrix(Ad, x, y, reps_tune=3, scrub=SCRUB, max_bytes=None):
    """Autotune and time every format on one handle.  Returns
    (times_ms[5], ci_ms[5], params per format); a format refused by the byte
    cap (max_bytes, default COLLECT_CAP) takes time +inf."""
    times, cis, params = [], [], {}
    cap = COLLECT_CAP if max_bytes is None else max_bytes
    for f in CLASSES:
        try:
            p, _ = Ad.autotune(f, x, y, scrub_bytes=scrub, reps=reps_tune, max_bytes=cap)
            B = Ad.convert(f, **p)
            r = B.time(x, y, warmup=2, min_reps=20, max_reps=200, rel_ci=0.05, scrub_bytes=scrub)
            del B
            times.append(r["median_ms"])
            cis.append(r["ci_ms"])
            params[f] = {k: v for k, v in p.items() if k not in ("max_bytes",)}
        except S.SpmvError as e:
            if e.status not in (-4,):  # only "too large" is an expected outcome
                raise
            times.append(math.inf)
            cis.append(0.0)
            params[f] = None
    return times, cis, params


def collect(start, stop, out_path, dtypes=(S.F64, S.F32), seed0=100, budget_s=None, prefetch=3, workers=3):
    """Profile matrices [start, stop) of the selector workload; append one
    JSON line per (matrix, dtype) to out_path; skip records already there."""
    import torch
    done = set()
    if os.path.exists(out_path):
        for line in open(out_path):
            try:
                r = json.loads(line)
                done.add((r["index"], r["dtype"]))
            except (ValueError, KeyError):
                pass
    specs = [synth.selector_spec(i, seed0) for i in range(start, stop)]
    dname = {S.F64: "f64", S.F32: "f32"}
    todo = [s for s in specs if any((s["index"], dname[d]) not in done for d in dtypes)]
    log(f"[collect] {len(todo)} matrices to profile ({len(specs) - len(todo)} already done)")
    # host generation runs in worker threads (the generators are C calls
    # that release the GIL) and overlaps the GPU profiling; the bounded
    # queue keeps at most `prefetch` generated matrices in host memory.
    jobs: queue.Queue = queue.Queue()
    for s in todo:
        jobs.put(s)
    ready: queue.Queue = queue.Queue(maxsize=prefetch)
    stop_flag = threading.Event()

    def producer():
        while not stop_flag.is_set():
            try:
                s = jobs.get_nowait()
            except queue.Empty:
                break
            try:
                A = synth.make(s)
            except Exception as e:  # surfaced in the consumer
                A = e
            while not stop_flag.is_set():
                try:
                    ready.put((s, A), timeout=0.5)
                    break
                except queue.Full:
                    pass

    threads = [threading.Thread(target=producer, daemon=True) for _ in range(workers)]
    for th in threads:
        th.start()
    t0 = time.time()
    n = 0
    with open(out_path, "a") as fo:
        while n < len(todo):
            spec, A = ready.get()
            if isinstance(A, Exception):
                stop_flag.set()
                raise RuntimeError(f"generation of matrix {spec['index']} failed") from A
            for dt in dtypes:
                if (spec["index"], dname[dt]) in done:
                    continue
                Ad = _to_device(A, dt)
                feats = Ad.features().tolist()
                x64 = synth.vector(Ad.N, spec["seed"] + 17)
                tdt = torch.float64 if dt == S.F64 else torch.float32
                x = torch.from_numpy(x64).to("cuda", tdt)
                y = torch.empty(Ad.M, dtype=tdt, device="cuda")
                times, cis, params = profile_matrix(Ad, x, y)
                rec = dict(index=spec["index"], kind=spec["kind"], M=Ad.M, N=Ad.N, nnz=Ad.nnz,
                           dtype=dname[dt], features=feats, times_ms=times, ci_ms=cis,
                           params=params, label=int(label_of(times)))
                fo.write(json.dumps(rec) + "\n")
                fo.flush()
                del Ad
            n += 1
            if n % 10 == 0:
                el = time.time() - t0
                log(f"[collect] {n}/{len(todo)} matrices in {el:.0f}s (last index {spec['index']})")
            if budget_s and time.time() - t0 > budget_s:
                log(f"[collect] time budget reached after {n} matrices")
                break
    stop_flag.set()
    return n


# ------------------------------------------------------------- metrics

def label_of(times):
    """Fastest format; exact ties go to the lower class index."""
    t = np.asarray(times, dtype=np.float64)
    return int(np.argmin(t))


def _geo(r):
    return float(np.exp(np.mean(np.log(r)))) if len(r) else math.nan


def evaluate(times, pred):
    """Metrics of a prediction against the profiled time table.

    times: (n, 5) ms (inf = infeasible); pred: (n,) class indices.
    frac = mean over matrices of t_best / t_pred (arithmetic, infeasible
    choices count 0; the geometric mean over feasible choices is also
    given), per fixed format the same with pred = f, the
    Table II analogue (best-format counts) and the Table III analogue (mean
    slowdown t_f / t_best over the matrices where f is feasible)."""
    T = np.asarray(times, dtype=np.float64)
    pred = np.asarray(pred, dtype=np.int64)
    n = len(T)
    best = T.min(axis=1)
    ratio = best / T[np.arange(n), pred]
    fixed = {}
    for f, name in enumerate(CLASSES):
        r = best / T[:, f]
        feas = np.isfinite(T[:, f])
        fixed[name] = dict(frac=float(np.mean(r)), geo=_geo(r[feas]),
                           slowdown=float(np.mean(T[feas, f] / best[feas])) if feas.any() else math.inf,
                           infeasible=int((~feas).sum()))
    labels = np.array([label_of(t) for t in T])
    best_fixed = max(fixed, key=lambda k: fixed[k]["frac"])
    return dict(n=n, frac=float(np.mean(ratio)), geo=_geo(ratio[np.isfinite(T[np.arange(n), pred])]),
                accuracy=float(np.mean(pred == labels)), fixed=fixed, best_fixed=best_fixed,
                best_counts={name: int((labels == f).sum()) for f, name in enumerate(CLASSES)})


def split(records, test_frac=0.2, seed=7):
    """Seeded matrix-level split, stratified by generator kind; both dtypes
    of a matrix land on the same side."""
    kinds = sorted({r["kind"] for r in records})
    rng = np.random.default_rng(seed)
    test = set()
    for k in kinds:
        idx = sorted({r["index"] for r in records if r["kind"] == k})
        perm = rng.permutation(len(idx))
        ntest = int(round(test_frac * len(idx)))
        test |= {idx[i] for i in perm[:ntest]}
    return test


def load(path):
    recs = [json.loads(l) for l in open(path) if l.strip()]
    for r in recs:
        r["times_ms"] = [math.inf if t is None else t for t in r["times_ms"]]
    return recs


# -------------------------------------------------------------- training

def train(records, dtype="f64", epochs=500, batch=128, lr=1e-3, seed=1, test=None):
    """Train one model on the GPU; returns (Model, report)."""
    import torch
    rs = [r for r in records if r["dtype"] == dtype]
    if test is None:
        test = split(records)
    tr = [r for r in rs if r["index"] not in test]
    te = [r for r in rs if r["index"] in test]
    Ftr = np.array([r["features"] for r in tr], np.float64)
    ytr = np.array([label_of(r["times_ms"]) for r in tr], np.int32)
    dF = torch.from_numpy(Ftr).cuda()
    lo = np.empty(12)
    hi = np.empty(12)
    S.check(S.lib().spmv_feature_range(S.dptr(dF), len(Ftr), S.hptr(lo), S.hptr(hi), S.stream()))
    X = torch.empty((len(Ftr), 12), dtype=torch.float32, device="cuda")
    S.check(S.lib().spmv_scale_features(S.dptr(dF), len(Ftr), S.hptr(lo), S.hptr(hi), S.dptr(X), S.stream()))
    params = np.concatenate([a.ravel() for a in synth.mlp_init(seed)]).astype(np.float32)
    dP = torch.from_numpy(params.copy()).cuda()
    dy = torch.from_numpy(ytr).cuda()
    rng = np.random.default_rng(seed + 1)
    order = np.concatenate([rng.permutation(len(Ftr)) for _ in range(epochs)]).astype(np.int32)
    dord = torch.from_numpy(order).cuda()
    losses = np.empty(epochs, np.float32)
    t0 = time.perf_counter()
    S.check(S.lib().spmv_mlp_train(S.dptr(dP), S.dptr(X), S.dptr(dy), len(Ftr), S.dptr(dord),
                                   epochs, batch, lr, S.stream(), S.hptr(losses)))
    train_s = time.perf_counter() - t0
    model = S.Model.create(dP.cpu().numpy(), lo, hi)
    report = dict(dtype=dtype, n_train=len(tr), n_test=len(te), epochs=epochs, batch=batch, lr=lr,
                  train_seconds=round(train_s, 3), loss_first=float(losses[0]), loss_last=float(losses[-1]))
    if te:
        pred = [CLASSES.index(model.select(r["features"])[0]) for r in te]
        report["test"] = evaluate([r["times_ms"] for r in te], pred)
        ptr = [CLASSES.index(model.select(r["features"])[0]) for r in tr]
        report["train"] = evaluate([r["times_ms"] for r in tr], ptr)
    return model, report


# --------------------------------------------------------- deployment

def model_path(dtype="f64"):
    return os.path.join(DATA_DIR, f"selector_{dtype}.bin")


def choose(Ad: "S.Matrix", model: "S.Model"):
    """Sec. V-A at run time: features of a CSR handle -> predicted format."""
    f = Ad.features()
    fmt, scores = model.select(f)
    return fmt, scores


DOMAIN_TOL = 0.02  # how far (in units of each feature's training span) a feature may lie outside it


def scaled_features(Ad: "S.Matrix", model: "S.Model") -> np.ndarray:
    """The matrix's 12 features after the model's transform and min-max
    scaling, on the device (spmv_scale_features): 0 and 1 are the smallest
    and largest values among the model's training matrices."""
    import torch
    f = torch.tensor(Ad.features(), dtype=torch.float64, device="cuda")
    _, lo, hi = model.params()
    X = torch.empty(12, dtype=torch.float32, device="cuda")
    S.check(S.lib().spmv_scale_features(S.dptr(f), 1, S.hptr(lo), S.hptr(hi), S.dptr(X), S.stream()))
    return X.cpu().numpy().astype(np.float64)


def in_domain(Ad: "S.Matrix", model: "S.Model", tol: float = DOMAIN_TOL) -> bool:
    """Whether every feature lies within the range the model was trained on
    (widened by tol of its span).  Outside it the network extrapolates, and
    the exhaustive fallback decides instead."""
    X = scaled_features(Ad, model)
    return bool(np.all(X >= -tol) and np.all(X <= 1.0 + tol))


def exhaustive(Ad, x, y, max_bytes=None):
    """The fallback and judge: profile all five formats, return the fastest."""
    times, _, params = profile_matrix(Ad, x, y, max_bytes=max_bytes)
    f = label_of(times)
    return CLASSES[f], params[CLASSES[f]], times


REFUSED = (-4, -5)  # too large for the byte cap, or a combination the kernels do not implement


def auto(Ad, x, y, model=None, margin=0.0, tune=True, scrub=SCRUB, max_bytes=None):
    """Pick a format and its parameters for a CSR handle and return the
    converted handle with how it was chosen.

    With a model: predicted format, then (tune=True) the autotuner's
    parameters for it.  Without a model, when the matrix's features lie
    outside the model's training range (in_domain), when the model's top
    softmax probability beats the runner-up by less than `margin`, or when
    the predicted format cannot hold the matrix (e.g. ELL above the byte cap
    max_bytes, default COLLECT_CAP: the training labels give such formats
    time +inf, but nothing stops the network from predicting one), every
    format is profiled and the fastest is taken (the exhaustive fallback)."""
    cap = COLLECT_CAP if max_bytes is None else max_bytes
    if model is not None and in_domain(Ad, model):
        fmt, z = choose(Ad, model)
        p = np.exp(z - z.max())
        p = np.sort(p / p.sum())[::-1]
        if p[0] - p[1] >= margin:
            try:
                params = {"max_bytes": cap}
                if tune:
                    params, _ = Ad.autotune(fmt, x, y, scrub_bytes=scrub, reps=3, max_bytes=cap)
                return Ad.convert(fmt, **params), fmt, "model"
            except S.SpmvError as e:
                if e.status not in REFUSED:
                    raise
    fmt, params, _ = exhaustive(Ad, x, y, max_bytes=cap)
    return Ad.convert(fmt, **dict(params or {}, max_bytes=cap)), fmt, "exhaustive"


def worth_converting(t_convert_ms, t_csr_ms, t_fmt_ms, calls):
    """Conversion-aware choice: converting pays off when the time saved over
    `calls` SpMVs exceeds the one-off conversion (the paper measures SpMV
    alone and notes that conversion costs a few SpMVs)."""
    return calls * (t_csr_ms - t_fmt_ms) > t_convert_ms


def auto_for_calls(Ad, x, y, model, calls, scrub=SCRUB):
    """The model's format, kept only if its conversion is repaid within
    `calls` SpMVs: the conversion is timed, then one cold launch of each of
    CSR and the converted handle.  Returns (handle, format, detail)."""
    import torch
    fmt, _ = choose(Ad, model)
    if fmt == "csr":
        return Ad, "csr", {"reason": "model chose csr"}
    e0, e1 = S.timing_events()
    e0.record()
    try:
        B = Ad.convert(fmt, max_bytes=COLLECT_CAP)
    except S.SpmvError as e:
        if e.status not in REFUSED:
            raise
        return Ad, "csr", {"reason": f"model chose {fmt}, which cannot hold this matrix ({e})"}
    e1.record()
    torch.cuda.synchronize()
    t_conv = e0.elapsed_time(e1)
    t_csr = Ad.time(x, y, warmup=1, min_reps=5, max_reps=20, scrub_bytes=scrub)["median_ms"]
    t_fmt = B.time(x, y, warmup=1, min_reps=5, max_reps=20, scrub_bytes=scrub)["median_ms"]
    detail = {"t_convert_ms": t_conv, "t_csr_ms": t_csr, "t_fmt_ms": t_fmt, "calls": calls}
    if worth_converting(t_conv, t_csr, t_fmt, calls):
        return B, fmt, detail
    return Ad, "csr", detail


def host_scale(F, lo=None, hi=None):
    """The feature transform and min-max scaling of spmv_scale_features,
    on the host, for the CPU classifiers below (returns X, lo, hi)."""
    F = np.array(F, dtype=np.float64, copy=True)
    logs = [0, 1, 2, 4, 5, 6, 7, 9, 10]
    F[:, logs] = np.log2(1.0 + F[:, logs])
    F[:, 3] = np.log2(np.maximum(F[:, 3], 2.0 ** -64))
    if lo is None:
        lo, hi = F.min(axis=0), F.max(axis=0)
    span = hi - lo
    X = np.zeros_like(F)
    nz = span > 0
    X[:, nz] = (F[:, nz] - lo[nz]) / span[nz]
    return X, lo, hi


def compare_classifiers(records, dtype="f64", test=None, seed=0):
    """The paper's model comparison (Sec. V-D, Fig. 11) on this GPU's time
    table: decision tree (the paper's model), Gaussian naive Bayes, 1-nearest
    neighbour, logistic regression, random forest and their soft vote, each
    trained on the same 80% and judged on the same held-out 20% as the MLP.
    CPU (scikit-learn); an offline evaluation, not part of the run path."""
    from sklearn.ensemble import RandomForestClassifier, VotingClassifier
    from sklearn.linear_model import LogisticRegression
    from sklearn.naive_bayes import GaussianNB
    from sklearn.neighbors import KNeighborsClassifier
    from sklearn.tree import DecisionTreeClassifier
    rs = [r for r in records if r["dtype"] == dtype]
    if test is None:
        test = split(records)
    tr = [r for r in rs if r["index"] not in test]
    te = [r for r in rs if r["index"] in test]
    Xtr, lo, hi = host_scale([r["features"] for r in tr])
    Xte, _, _ = host_scale([r["features"] for r in te], lo, hi)
    ytr = np.array([label_of(r["times_ms"]) for r in tr])
    T = [r["times_ms"] for r in te]
    models = {
        "dtc": DecisionTreeClassifier(random_state=seed),
        "gnb": GaussianNB(),
        "knn1": KNeighborsClassifier(n_neighbors=1),
        "lr": LogisticRegression(max_iter=2000),
        "rfc": RandomForestClassifier(n_estimators=100, random_state=seed),
    }
    models["vote"] = VotingClassifier([(k, v) for k, v in models.items() if k != "knn1"], voting="soft")
    out = {}
    for name, m in models.items():
        m.fit(Xtr, ytr)
        pred = m.predict(Xte)
        ev = evaluate(T, pred)
        out[name] = {"frac": ev["frac"], "geo": ev["geo"], "accuracy": ev["accuracy"]}
    out["fixed_csr"] = {"frac": evaluate(T, [0] * len(T))["frac"]}
    return out


PARAM_KEYS = {"csr": ("csr_lanes_per_row", "flags", "bands"), "csr5": ("csr5_omega", "csr5_sigma", "bands"), "ell": (),
              "sell": ("sell_C", "sell_sigma", "bands"), "hyb": ("hyb_K", "bands")}


def merge(out_path, parts):
    """Join collection parts into one table sorted by (matrix, dtype); each
    format keeps only the parameters that apply to it."""
    recs = {}
    for p in parts:
        for r in load(p):
            r["params"] = {f: (None if v is None else {k: v[k] for k in PARAM_KEYS[f] if k in v})
                           for f, v in r["params"].items()}
            recs[(r["index"], r["dtype"])] = r
    with open(out_path, "w") as fo:
        for key in sorted(recs):
            fo.write(json.dumps(recs[key]) + "\n")
    return len(recs)


# ---------------------------------------------------------------- CLI

def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--start", type=int, default=0)
    c.add_argument("--stop", type=int, default=3000)
    c.add_argument("--out", required=True)
    c.add_argument("--budget", type=float, default=None, help="stop after this many seconds")
    t = sub.add_parser("train")
    t.add_argument("--dataset", required=True)
    t.add_argument("--out-dir", default=DATA_DIR)
    t.add_argument("--epochs", type=int, default=500)
    cp = sub.add_parser("compare")
    cp.add_argument("--dataset", required=True)
    m = sub.add_parser("merge")
    m.add_argument("out")
    m.add_argument("parts", nargs="+")
    a = ap.parse_args(argv)
    if a.cmd == "collect":
        collect(a.start, a.stop, a.out, budget_s=a.budget)
    elif a.cmd == "compare":
        recs = load(a.dataset)
        for dt in ("f64", "f32"):
            print(dt, json.dumps(compare_classifiers(recs, dt)))
    elif a.cmd == "merge":
        log(f"[merge] {merge(a.out, a.parts)} records")
    else:
        recs = load(a.dataset)
        os.makedirs(a.out_dir, exist_ok=True)
        reports = {}
        for dt in ("f64", "f32"):
            if not any(r["dtype"] == dt for r in recs):
                continue
            m, rep = train(recs, dt, epochs=a.epochs)
            m.save(os.path.join(a.out_dir, f"selector_{dt}.bin"))
            reports[dt] = rep
            log(json.dumps(rep))
        json.dump(reports, open(os.path.join(a.out_dir, "selector_report.json"), "w"), indent=1)


if __name__ == "__main__":
    main()
