"""The learned selector end to end (Sec. V): train on the GPU from the
profiled time table, evaluate on the held-out 20%, and check what the
trained network gains over fixed formats and over the untrained network.

The time table (paper_1805_11938_amd/data/selector_dataset.jsonl) was
measured by exhaustive profiling of this library's own kernels; it is the
judge of every selection, as the exhaustive search is in the paper."""
import os

import numpy as np
import pytest

import oracle
from paper_1805_11938_amd import selector as SEL
from paper_1805_11938_amd import spmv as S
from paper_1805_11938_amd import synth

from gpu_util import TOL, device_vec, reference, rowwise_err

pytestmark = pytest.mark.gpu

DATASET = os.path.join(SEL.DATA_DIR, "selector_dataset.jsonl")


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.fixture(scope="module")
def records():
    if not os.path.exists(DATASET):
        pytest.skip("no profiled time table")
    return SEL.load(DATASET)


@pytest.fixture(scope="module")
def trained(torch, records):
    test = SEL.split(records)
    return {dt: SEL.train(records, dt, test=test) for dt in ("f64", "f32")}, test


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_selector_reaches_ninety_percent_of_best_and_beats_fixed_csr(trained, dt):
    (models, test) = trained
    _, rep = models[dt]
    ev = rep["test"]
    assert rep["n_test"] >= 0.19 * (rep["n_train"] + rep["n_test"])
    assert ev["frac"] >= 0.90, ev
    assert ev["frac"] > ev["fixed"]["csr"]["frac"], ev
    assert ev["frac"] >= ev["fixed"][ev["best_fixed"]]["frac"] - 1e-12, ev
    assert rep["loss_last"] < rep["loss_first"]


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_training_gains_over_untrained_network(torch, trained, records, dt):
    (models, test) = trained
    model, rep = models[dt]
    te = [r for r in records if r["dtype"] == dt and r["index"] in test]
    _, lo, hi = model.params()
    flat = np.concatenate([a.ravel() for a in synth.mlp_init(1)]).astype(np.float32)
    untrained = S.Model.create(flat, lo, hi)
    pred0 = [S.FMT_NAMES.index(untrained.select(r["features"])[0]) for r in te]
    ev0 = SEL.evaluate([r["times_ms"] for r in te], pred0)
    assert rep["test"]["frac"] > ev0["frac"]
    assert rep["test"]["accuracy"] > ev0["accuracy"]


def test_device_inference_matches_oracle_forward(trained, records):
    (models, test) = trained
    model, _ = models["f64"]
    p, lo, hi = model.params()
    shapes = [(12, 64), (64,), (64, 64), (64,), (64, 5), (5,)]
    params, off = [], 0
    for sh in shapes:
        k = int(np.prod(sh))
        params.append(p[off:off + k].astype(np.float64).reshape(sh))
        off += k
    te = [r for r in records if r["dtype"] == "f64" and r["index"] in test][:200]
    F = np.array([r["features"] for r in te])
    z_ref, _ = oracle.mlp_forward(params, oracle.minmax_apply(oracle.feature_transform(F), lo, hi))
    for f, z in zip(F, z_ref):
        best, sc = model.select(f)
        assert np.max(np.abs(sc - z)) <= 1e-4 * max(1.0, np.abs(z).max())
        order = np.argsort(-z, kind="stable")
        if z[order[0]] - z[order[1]] > 1e-3:
            assert best == S.FMT_NAMES[order[0]]


def test_selected_format_runs_correctly_on_held_out_matrices(torch, trained, records):
    """features -> select -> convert (recorded tuned parameters) -> run, on
    the three smallest held-out matrices, against the FP64 oracle."""
    (models, test) = trained
    model, _ = models["f64"]
    te = sorted((r for r in records if r["dtype"] == "f64" and r["index"] in test), key=lambda r: r["nnz"])[:3]
    for r in te:
        spec = synth.selector_spec(r["index"])
        A = synth.make(spec)
        Ad = SEL._to_device(A, S.F64)
        f = Ad.features()
        assert np.array_equal(f, np.array(r["features"]))  # same kernel, same matrix
        fmt, _ = SEL.choose(Ad, model)
        p = r["params"][fmt] or {}
        B = Ad.convert(fmt, **p)
        ptr, col, val = Ad.to_csr()
        H = synth.HostCSR(Ad.M, Ad.N, ptr, col, val)
        x64 = synth.vector(Ad.N, 5)
        yref, den = reference(H, x64, 0)
        out = B.run(device_vec(x64, 0)).cpu().numpy()
        assert rowwise_err(out, yref, den) <= TOL[0], (r["index"], fmt)


def test_auto_uses_model_or_exhaustive_fallback(torch, trained):
    (models, _) = trained
    model, _ = models["f64"]
    A = synth.zipf_rows(30_000, 30_000, 2.0, 16, 3_000, 21, 22)
    Ad = S.Matrix.from_host(A)
    x64 = synth.vector(A.N, 23)
    yref, den = reference(A, x64, 0)
    x = device_vec(x64, 0)
    y = torch.empty(A.M, dtype=torch.float64, device="cuda")
    B, fmt, how = SEL.auto(Ad, x, y, model, margin=0.0, scrub=64 << 20)
    assert how == "model" and B.fmt == fmt == SEL.choose(Ad, model)[0]
    assert rowwise_err(B.run(x).cpu().numpy(), yref, den) <= TOL[0]
    B2, fmt2, how2 = SEL.auto(Ad, x, y, model, margin=1.01, scrub=64 << 20)  # no margin can reach 1.01
    assert how2 == "exhaustive" and B2.fmt == fmt2
    assert rowwise_err(B2.run(x).cpu().numpy(), yref, den) <= TOL[0]
    B3, _, how3 = SEL.auto(Ad, x, y, None, scrub=64 << 20)
    assert how3 == "exhaustive"


def test_auto_falls_back_outside_the_training_range(torch, trained, records):
    """A matrix smaller than every training matrix (4,096 rows; the set has
    10^4..2x10^6) is decided by exhaustive profiling, a training-range matrix
    by the model; the scaled features agree with the host transform."""
    (models, test) = trained
    model, _ = models["f64"]
    A = synth.laplace2d(64)
    Ad = S.Matrix.from_host(A)
    assert not SEL.in_domain(Ad, model)
    x = device_vec(synth.vector(A.N, 3), 0)
    y = torch.empty(A.M, dtype=torch.float64, device="cuda")
    B, fmt, how = SEL.auto(Ad, x, y, model, scrub=16 << 20)
    assert how == "exhaustive" and B.fmt == fmt
    r = next(r for r in records if r["index"] in test and r["dtype"] == "f64")
    H = SEL._to_device(synth.make(synth.selector_spec(r["index"])), S.F64)
    X = SEL.scaled_features(H, model)
    _, lo, hi = model.params()
    Xh, _, _ = SEL.host_scale(np.array([H.features()]), lo, hi)
    assert np.allclose(X, Xh[0], rtol=0, atol=1e-5)
    assert SEL.in_domain(H, model) == bool(np.all(Xh >= -SEL.DOMAIN_TOL) and np.all(Xh <= 1 + SEL.DOMAIN_TOL))


def test_auto_for_calls_keeps_csr_for_few_calls(torch, trained):
    (models, _) = trained
    model, _ = models["f64"]
    A = synth.zipf_rows(200_000, 200_000, 2.0, 16, 8_000, 31, 32)
    Ad = SEL._to_device(A, S.F64)
    x = device_vec(synth.vector(A.N, 33), 0)
    y = torch.empty(A.M, dtype=torch.float64, device="cuda")
    fmt, _ = SEL.choose(Ad, model)
    B1, f1, d1 = SEL.auto_for_calls(Ad, x, y, model, calls=1, scrub=64 << 20)
    Bn, fn, dn = SEL.auto_for_calls(Ad, x, y, model, calls=10**6, scrub=64 << 20)
    if fmt != "csr":
        for f, d, calls in ((f1, d1, 1), (fn, dn, 10**6)):
            pays = SEL.worth_converting(d["t_convert_ms"], d["t_csr_ms"], d["t_fmt_ms"], calls)
            assert f == (fmt if pays else "csr")
        assert d1["t_convert_ms"] > 0
    yref, den = reference(A, synth.vector(A.N, 33), 0)
    assert rowwise_err(Bn.run(x).cpu().numpy(), yref, den) <= TOL[0]


def test_deployed_models_decide_the_benchmark_matrices(torch):
    """The models shipped in data/ cover the benchmark's 100^3 27-point
    stencil and its Zipf matrix (features inside the training range), so
    selection there is one feature pass and one inference, not the
    exhaustive fallback; the stencil's pick is a regular-row format."""
    from paper_1805_11938_amd import workloads as W
    for name, want in (("stencil27_100", ("sell", "ell", "hyb")), ("zipf_1M", None)):
        A = W.make(name)
        for dname, dt in (("f64", S.F64), ("f32", S.F32)):
            m = S.Model.load(SEL.model_path(dname))
            Ad = S.Matrix.from_csr(A.M, A.N, A.ptr, A.col, A.val.astype(np.float32) if dt == S.F32 else A.val, dt)
            assert SEL.in_domain(Ad, m), (name, dname, SEL.scaled_features(Ad, m))
            fmt, _ = SEL.choose(Ad, m)
            if want:
                assert fmt in want, (name, dname, fmt)
            del Ad
