"""GPU parity of the selector path: device features, feature scaling, MLP
forward / backward / Adam against the FP64 oracle, model files and select."""
import numpy as np
import pytest

import oracle
from paper_1805_11938_amd import synth
from paper_1805_11938_amd import spmv as S

pytestmark = pytest.mark.gpu

EXACT = [0, 1, 2, 4, 5, 10]  # integer-valued features


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def mats():
    A = np.zeros((30, 40))
    A[5, 3:30] = 1
    return [synth.laplace2d(64), synth.random_pattern(500, 700, 0.01, 3), synth.zipf_rows(50_000, 50_000, 2.0, 16, 10_000, 4, 5),
            synth.uniform_random(20_000, 30_000, 1.2, 5, 6), synth.from_dense(A), synth.from_dense(np.zeros((9, 9))),
            synth.stencil27(20)]


@pytest.mark.parametrize("i", range(7))
def test_features_match_oracle(torch, i):
    A = mats()[i]
    f_ref = oracle.features(A.M, A.N, A.ptr, A.col)
    f = S.Matrix.from_host(A).features()
    assert np.array_equal(f[EXACT], f_ref[EXACT]), (f, f_ref)
    rel = np.abs(f - f_ref) / np.maximum(np.abs(f_ref), 1e-300)
    assert np.all((rel <= 1e-12) | (f == f_ref)), (f, f_ref)


def _dev(torch, a, dt=None):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_forward_backward_adam_match_oracle(torch):
    rng = np.random.default_rng(0)
    p64 = synth.mlp_init(7)
    p64 = [a + 0.05 * rng.standard_normal(a.shape) for a in p64]
    flat = np.concatenate([a.ravel() for a in p64]).astype(np.float32)
    assert flat.size == S.NPARAM
    p32 = [a.astype(np.float32).astype(np.float64) for a in p64]  # the values the device holds
    B = 37
    X = rng.random((B, 12)).astype(np.float32)
    y = rng.integers(0, 5, B).astype(np.int32)
    dP, dX, dy = _dev(torch, flat), _dev(torch, X), _dev(torch, y)
    Z = torch.empty((B, 5), dtype=torch.float32, device="cuda")
    S.check(S.lib().spmv_mlp_forward(S.dptr(dP), S.dptr(dX), B, S.dptr(Z), None, None, S.stream()))
    z_ref, _ = oracle.mlp_forward(p32, X.astype(np.float64))
    assert np.max(np.abs(Z.cpu().numpy() - z_ref)) <= 1e-5 * max(1.0, np.abs(z_ref).max())
    G = torch.empty(S.NPARAM, dtype=torch.float32, device="cuda")
    L = torch.empty(1, dtype=torch.float32, device="cuda")
    S.check(S.lib().spmv_mlp_backward(S.dptr(dP), S.dptr(dX), S.dptr(dy), B, S.dptr(G), S.dptr(L), S.stream()))
    loss_ref, g_ref = oracle.mlp_loss_and_grads(p32, X.astype(np.float64), y)
    g_ref = np.concatenate([a.ravel() for a in g_ref])
    g = G.cpu().numpy()
    assert np.max(np.abs(g - g_ref)) <= 1e-4 * np.abs(g_ref).max()
    assert abs(L.item() - loss_ref) <= 1e-5 * abs(loss_ref)
    # one Adam step from zero moments on the oracle's gradient
    m = torch.zeros(S.NPARAM, dtype=torch.float32, device="cuda")
    v = torch.zeros(S.NPARAM, dtype=torch.float32, device="cuda")
    Gd = _dev(torch, g_ref.astype(np.float32))
    S.check(S.lib().spmv_mlp_adam(S.dptr(dP), S.dptr(Gd), S.dptr(m), S.dptr(v), 1, 1e-3, 0.9, 0.999, 1e-8, S.stream()))
    (p1,), _, _ = oracle.adam_step([flat.astype(np.float64)], [g_ref.astype(np.float32).astype(np.float64)],
                                   [np.zeros(S.NPARAM)], [np.zeros(S.NPARAM)], 1)
    assert np.max(np.abs(dP.cpu().numpy() - p1) / np.maximum(np.abs(p1), 1e-3)) <= 1e-5


def test_scaling_matches_oracle(torch):
    F = np.stack([S.Matrix.from_host(A).features() for A in mats()])
    T = oracle.feature_transform(F)
    lo, hi = oracle.minmax_fit(T)
    want = oracle.minmax_apply(T, lo, hi)
    dF = _dev(torch, F)
    X = torch.empty(F.shape, dtype=torch.float32, device="cuda")
    S.check(S.lib().spmv_scale_features(S.dptr(dF), len(F), S.hptr(lo), S.hptr(hi), S.dptr(X), S.stream()))
    assert np.max(np.abs(X.cpu().numpy() - want)) <= 1e-6


def test_model_roundtrip_and_select(torch, tmp_path):
    p64 = synth.mlp_init(11)
    flat = np.concatenate([a.ravel() for a in p64]).astype(np.float32)
    F = np.stack([S.Matrix.from_host(A).features() for A in mats()])
    T = oracle.feature_transform(F)
    lo, hi = oracle.minmax_fit(T)
    m = S.Model.create(flat, lo, hi)
    path = str(tmp_path / "m.bin")
    m.save(path)
    m2 = S.Model.load(path)
    p, lo2, hi2 = m2.params()
    assert np.array_equal(p, flat) and np.array_equal(lo2, lo) and np.array_equal(hi2, hi)
    p32 = [a.astype(np.float32).astype(np.float64) for a in p64]
    for f in F:
        z_ref, _ = oracle.mlp_forward(p32, oracle.minmax_apply(oracle.feature_transform(f[None]), lo, hi))
        best, sc = m2.select(f)
        assert np.max(np.abs(sc - z_ref[0])) <= 1e-5 * max(1.0, np.abs(z_ref).max())
        order = np.argsort(-z_ref[0], kind="stable")
        if z_ref[0][order[0]] - z_ref[0][order[1]] > 1e-4:
            assert best == S.FMT_NAMES[order[0]]
    with pytest.raises(S.SpmvError):
        S.Model.load(str(tmp_path / "missing.bin"))


def test_training_reduces_loss_like_the_oracle(torch):
    rng = np.random.default_rng(5)
    n, epochs, batch = 96, 30, 32
    X = rng.random((n, 12)).astype(np.float32)
    y = (X[:, 0] * 5).astype(np.int32).clip(0, 4)  # learnable labels
    order = np.concatenate([rng.permutation(n) for _ in range(epochs)]).astype(np.int32)
    flat = np.concatenate([a.ravel() for a in synth.mlp_init(3)]).astype(np.float32)
    dP = _dev(torch, flat.copy())
    dX, dy, dord = _dev(torch, X), _dev(torch, y), _dev(torch, order)  # keep the tensors alive for the call
    losses = np.empty(epochs, np.float32)
    S.check(S.lib().spmv_mlp_train(S.dptr(dP), S.dptr(dX), S.dptr(dy), n, S.dptr(dord), epochs, batch, 1e-2,
                                   S.stream(), S.hptr(losses)))
    assert losses[-1] < 0.7 * losses[0]
    # FP64 oracle on the same initial parameters, order and batches
    shapes = [(12, 64), (64,), (64, 64), (64,), (64, 5), (5,)]
    params, off = [], 0
    for sh in shapes:
        k = int(np.prod(sh))
        params.append(flat[off:off + k].astype(np.float64).reshape(sh))
        off += k
    mo = [np.zeros_like(a) for a in params]
    vo = [np.zeros_like(a) for a in params]
    t, ref = 0, []
    for e in range(epochs):
        ls = 0.0
        for b0 in range(0, n, batch):
            idx = order[e * n + b0:e * n + min(n, b0 + batch)]
            loss, g = oracle.mlp_loss_and_grads(params, X[idx].astype(np.float64), y[idx])
            ls += loss * len(idx) / n
            t += 1
            params, mo, vo = oracle.adam_step(params, g, mo, vo, t, lr=1e-2)
        ref.append(ls)
    rel = np.abs(losses - np.array(ref)) / np.array(ref)
    # FP32 device training tracks the FP64 oracle; rounding differences grow slowly over the run
    assert np.max(rel[:5]) <= 1e-3 and np.max(rel) <= 5e-2, (losses[:5], ref[:5], rel)


def test_training_epochs_match_the_oracle_from_the_same_start(torch):
    """Each epoch of device training (spmv_mlp_train with epochs = 1, fresh
    Adam moments per call) against the FP64 oracle's epoch started from the
    parameters the device holds at that point, so rounding differences do not
    compound over the run: the epoch's mean loss and the parameters after it
    agree within FP32 accuracy."""
    rng = np.random.default_rng(9)
    n, epochs, batch = 96, 6, 32
    X = rng.random((n, 12)).astype(np.float32)
    y = (X[:, 0] * 5).astype(np.int32).clip(0, 4)
    flat = np.concatenate([a.ravel() for a in synth.mlp_init(4)]).astype(np.float32)
    dP = _dev(torch, flat.copy())
    dX, dy = _dev(torch, X), _dev(torch, y)
    shapes = [(12, 64), (64,), (64, 64), (64,), (64, 5), (5,)]

    def unflat(v):
        out, off = [], 0
        for sh in shapes:
            k = int(np.prod(sh))
            out.append(np.asarray(v[off:off + k], np.float64).reshape(sh))
            off += k
        return out

    for e in range(epochs):
        start = dP.cpu().numpy().copy()
        order = rng.permutation(n).astype(np.int32)
        dord = _dev(torch, order)
        loss = np.empty(1, np.float32)
        S.check(S.lib().spmv_mlp_train(S.dptr(dP), S.dptr(dX), S.dptr(dy), n, S.dptr(dord), 1, batch, 1e-2,
                                       S.stream(), S.hptr(loss)))
        params = unflat(start)
        mo = [np.zeros_like(a) for a in params]
        vo = [np.zeros_like(a) for a in params]
        ref = 0.0
        for t, b0 in enumerate(range(0, n, batch), start=1):
            idx = order[b0:b0 + batch]
            lb, g = oracle.mlp_loss_and_grads(params, X[idx].astype(np.float64), y[idx])
            ref += lb * len(idx) / n
            params, mo, vo = oracle.adam_step(params, g, mo, vo, t, lr=1e-2)
        assert abs(loss[0] - ref) <= 1e-5 * ref, (e, loss[0], ref)
        got = dP.cpu().numpy().astype(np.float64)
        want = np.concatenate([a.ravel() for a in params])
        # an Adam step moves a parameter by at most about lr = 1e-2; FP32
        # rounding changes it by far less, except where a gradient is so
        # small that its FP32 and FP64 values differ in relative terms
        d = np.abs(got - want)
        assert np.max(d) <= 3e-2, (e, np.max(d))
        assert np.mean(d <= 1e-5) >= 0.99, (e, np.mean(d <= 1e-5), np.sort(d)[-10:])
