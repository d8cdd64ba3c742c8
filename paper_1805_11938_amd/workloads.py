"""The named workloads and the launch configuration they are measured in.

* ``stencil27_100``: 3-D 27-point stencil on a 100^3 grid, 10^6 rows,
  26,463,592 nnz, values N(0,1) (seed 2), x U[-1,1] (seed 3).
* ``zipf_1M``: 10^6 x 10^6, Zipf(alpha=2) row lengths with mean 16 and cap
  10^4, uniform distinct columns (seed 4), values N(0,1) (seed 5), x seed 6.
* ``rmat24``: R-MAT(0.57, 0.19, 0.19, 0.05) with 2^24 rows and 2^28 edge
  draws (seed 10), duplicates summed on the device, values N(0,1)
  (seed 12), x seed 11.  Scale-free: ~56% empty rows, longest row ~3.7e5.

They stand in for the regular and irregular matrices of the paper's
evaluation (Sec. III-C: square matrices with 10^5..2x10^7 nonzeros from
scientific and graph problems), which are not reproduced here.

The launch configuration of each (workload, format) pair -- the parameters
the benchmark converts with -- comes from the autotuner (Sec. II-B's tuning
knobs: SELL chunk C and window sigma, CSR lanes per row, HYB width K, CSR5
sigma) and is stored in ``data/tuned_params.json``; formats missing there use
the library defaults.
"""
from __future__ import annotations

import json
import os

from . import synth

HERE = os.path.dirname(os.path.abspath(__file__))
TUNED = os.path.join(HERE, "data", "tuned_params.json")
FORMATS = ("csr", "csr5", "ell", "sell", "hyb")
TUNE_KEYS = ("sell_C", "sell_sigma", "csr_lanes_per_row", "hyb_K", "csr5_omega", "csr5_sigma", "flags",
             "bands")

X_SEED = {"stencil27_100": 3, "zipf_1M": 6, "rmat24": 11}


def stencil27_100():
    return synth.stencil27(100, seed=2)


def zipf_1m():
    return synth.zipf_rows(1_000_000, 1_000_000, 2.0, 16.0, 10_000, seed=4, val_seed=5)


def rmat24():
    """Raw triplets (HostCOO); the device canonicalises them."""
    return synth.rmat_coo(24, 1 << 28, seed=10, val_seed=12)


BUILDERS = {"stencil27_100": stencil27_100, "zipf_1M": zipf_1m, "rmat24": rmat24}


def make(name):
    return BUILDERS[name]()


def x_vector(name, n):
    return synth.vector(n, X_SEED[name])


def tuned_params(name: str, fmt: str, dtype: str = "f64") -> dict:
    """Launch parameters of (workload, format, dtype); {} = library defaults."""
    if not os.path.exists(TUNED):
        return {}
    t = json.load(open(TUNED))
    return dict(t.get(name, {}).get(dtype, {}).get(fmt, {}))


def tune(names=("stencil27_100", "zipf_1M"), dtypes=("f64",), out=TUNED, reps=10):
    """Run the autotuner for each (workload, format, dtype) on the GPU and
    store the winners."""
    import sys
    import numpy as np
    import torch
    from . import spmv as S
    res = json.load(open(out)) if os.path.exists(out) else {}
    for name in names:
        A = make(name)
        for dn in dtypes:
            dt = S.F64 if dn == "f64" else S.F32
            tdt = torch.float64 if dt == S.F64 else torch.float32
            if isinstance(A, synth.HostCOO):
                val = A.val.astype(np.float32) if dt == S.F32 else A.val
                base = S.Matrix.from_coo(A.M, A.N, A.row, A.col, val, dt)
            else:
                val = A.val.astype(np.float32) if dt == S.F32 else A.val
                base = S.Matrix.from_csr(A.M, A.N, A.ptr, A.col, val, dt)
            x = torch.from_numpy(x_vector(name, A.N)).to("cuda", tdt)
            y = torch.empty(A.M, dtype=tdt, device="cuda")
            for fmt in FORMATS:
                try:
                    p, ms = base.autotune(fmt, x, y, reps=reps)
                except S.SpmvError as e:
                    print(f"[tune] {name}/{dn}/{fmt}: {e}", file=sys.stderr, flush=True)
                    continue
                keep = {k: int(p[k]) for k in TUNE_KEYS}
                res.setdefault(name, {}).setdefault(dn, {})[fmt] = keep
                print(f"[tune] {name}/{dn}/{fmt}: {ms * 1e3:.1f} us with {keep}", file=sys.stderr, flush=True)
            del base
        del A
    os.makedirs(os.path.dirname(out), exist_ok=True)
    json.dump(res, open(out, "w"), indent=1, sort_keys=True)
    return res


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["tune"])
    ap.add_argument("--names", default="stencil27_100,zipf_1M")
    ap.add_argument("--dtypes", default="f64")
    ap.add_argument("--out", default=TUNED)
    a = ap.parse_args()
    tune(a.names.split(","), a.dtypes.split(","), a.out)
