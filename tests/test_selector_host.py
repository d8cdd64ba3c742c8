"""Host logic of the selector driver: labels, metrics and the split.

These run without a GPU; the metric definitions are checked on tables whose
answers are worked out by hand."""
import math

import numpy as np
import pytest

from paper_1805_11938_amd import selector as SEL

INF = math.inf


def test_label_is_argmin_with_low_index_ties():
    assert SEL.label_of([3, 2, 2, 5, 9]) == 1
    assert SEL.label_of([INF, INF, 7, INF, 7]) == 2
    assert SEL.label_of([1, 1, 1, 1, 1]) == 0


def test_evaluate_hand_worked_table():
    # two matrices; best times 1 and 1
    T = [[1.0, 2.0, 4.0, 1.0, 8.0],
         [2.0, 1.0, INF, 4.0, 2.0]]
    r = SEL.evaluate(T, [3, 4])
    # t_best/t_pred = 1/1 and 1/2
    assert r["frac"] == pytest.approx(0.75)
    assert r["geo"] == pytest.approx(math.sqrt(0.5))
    assert r["accuracy"] == 0.0  # labels are 0 (tie goes to csr) and 1
    assert r["best_counts"] == {"csr": 1, "csr5": 1, "ell": 0, "sell": 0, "hyb": 0}
    f = r["fixed"]
    assert f["csr"]["frac"] == pytest.approx((1 + 0.5) / 2)
    assert f["csr5"]["frac"] == pytest.approx((0.5 + 1) / 2)
    # infeasible ELL counts as 0 in the arithmetic mean and is left out of
    # the slowdown and the geometric mean
    assert f["ell"]["frac"] == pytest.approx(0.25 / 2)
    assert f["ell"]["infeasible"] == 1
    assert f["ell"]["slowdown"] == pytest.approx(4.0)
    assert f["ell"]["geo"] == pytest.approx(0.25)
    assert f["hyb"]["slowdown"] == pytest.approx((8 + 2) / 2)
    assert r["best_fixed"] in ("csr", "csr5")


def test_evaluate_perfect_prediction_is_one():
    rng = np.random.default_rng(0)
    T = rng.uniform(1, 10, (50, 5))
    T[rng.random((50, 5)) < 0.1] = INF
    T[:, 0] = np.minimum(T[:, 0], 10)  # at least one feasible format per row
    pred = [SEL.label_of(t) for t in T]
    r = SEL.evaluate(T, pred)
    assert r["frac"] == 1.0 and r["accuracy"] == 1.0 and r["geo"] == 1.0


def _records(n_per_kind, kinds=("banded", "blockdiag", "uniform", "zipf", "rmat")):
    out = []
    i = 0
    for k in kinds:
        for _ in range(n_per_kind):
            for dt in ("f64", "f32"):
                out.append(dict(index=i, kind=k, dtype=dt))
            i += 1
    return out


def test_split_is_stratified_seeded_and_dtype_consistent():
    recs = _records(100)
    a = SEL.split(recs, 0.2, seed=7)
    b = SEL.split(recs, 0.2, seed=7)
    c = SEL.split(recs, 0.2, seed=8)
    assert a == b and a != c
    assert len(a) == 100  # 20% of 500 matrices
    for k in ("banded", "blockdiag", "uniform", "zipf", "rmat"):
        idx = {r["index"] for r in recs if r["kind"] == k}
        assert len(idx & a) == 20
    # the split is over matrices, so both dtypes of a matrix share a side
    assert all(isinstance(i, int) for i in a)


def test_host_scale_matches_the_oracle_transform():
    import oracle
    rng = np.random.default_rng(3)
    F = np.abs(rng.standard_normal((40, 12))) * 10.0 ** rng.integers(0, 6, (40, 12))
    F[:, 3] = rng.uniform(1e-9, 1e-2, 40)
    X, lo, hi = SEL.host_scale(F)
    T = oracle.feature_transform(F)
    olo, ohi = oracle.minmax_fit(T)
    assert np.allclose(lo, olo, rtol=0, atol=0) and np.allclose(hi, ohi, rtol=0, atol=0)
    assert np.allclose(X, oracle.minmax_apply(T, olo, ohi), rtol=0, atol=1e-15)


def test_paper_classifiers_on_the_profiled_table():
    """Sec. V-D's comparison on the committed time table: every model beats
    fixed CSR on the held-out matrices; the decision tree (the paper's model)
    reaches 95% of the best."""
    import os
    path = os.path.join(SEL.DATA_DIR, "selector_dataset.jsonl")
    if not os.path.exists(path):
        pytest.skip("no profiled time table")
    pytest.importorskip("sklearn")
    recs = SEL.load(path)
    r = SEL.compare_classifiers(recs, "f64")
    assert r["dtc"]["frac"] >= 0.95
    for name in ("dtc", "knn1", "lr", "rfc", "vote"):
        assert r[name]["frac"] > r["fixed_csr"]["frac"], name


def test_conversion_pays_off_rule():
    # 10 ms to convert, 1 ms saved per call: worth it from 11 calls on
    assert not SEL.worth_converting(10.0, 3.0, 2.0, 10)
    assert SEL.worth_converting(10.0, 3.0, 2.0, 11)
    assert not SEL.worth_converting(0.0, 2.0, 3.0, 1000)  # a slower format never pays


def test_merge_keeps_each_formats_own_parameters(tmp_path):
    """Collection parts are joined by (matrix, dtype), later parts winning,
    and each format keeps only its own parameters (column bands included
    for CSR, CSR5, SELL and HYB)."""
    import json
    full = dict(csr_lanes_per_row=0, flags=32, bands=2, csr5_omega=64, csr5_sigma=16, sell_C=64,
                sell_sigma=1000, hyb_K=3)
    rec = dict(index=4, kind="zipf", M=10, N=10, nnz=20, dtype="f64", features=[0.0] * 12,
               times_ms=[1.0, 2.0, None, 3.0, 4.0], ci_ms=[0.0] * 5,
               params={f: dict(full) for f in SEL.CLASSES}, label=0)
    rec["params"]["ell"] = None
    a, b = tmp_path / "a.jsonl", tmp_path / "b.jsonl"
    a.write_text(json.dumps(rec) + "\n")
    rec2 = dict(rec, times_ms=[5.0, 2.0, None, 3.0, 4.0], label=1)
    b.write_text(json.dumps(rec2) + "\n" + json.dumps(dict(rec, index=1)) + "\n")
    out = tmp_path / "m.jsonl"
    assert SEL.merge(str(out), [str(a), str(b)]) == 2
    recs = SEL.load(str(out))
    assert [r["index"] for r in recs] == [1, 4]
    p = recs[1]["params"]
    assert recs[1]["times_ms"][0] == 5.0 and recs[1]["times_ms"][2] == INF
    assert p["csr"] == dict(csr_lanes_per_row=0, flags=32, bands=2)
    assert p["csr5"] == dict(csr5_omega=64, csr5_sigma=16, bands=2)
    assert p["sell"] == dict(sell_C=64, sell_sigma=1000, bands=2)
    assert p["hyb"] == dict(hyb_K=3, bands=2)
    assert p["ell"] is None
