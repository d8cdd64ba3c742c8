"""GPU parity of the multi-RHS SpMM, the batched launch and the
autotuner's choices, against the FP64 oracle."""
import numpy as np
import pytest

import oracle
from paper_1805_11938_amd import synth
from paper_1805_11938_amd import spmv as S

from gpu_util import TOL, device_vec, reference, rowwise_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


SPMM_MATS = [("stencil27_12", synth.stencil27(12)), ("zipf_long", synth.zipf_rows(8000, 8000, 2.0, 16, 6000, 4, 5)),
             ("empty_rows", synth.uniform_random(5000, 7000, 1.0, 3, 4)), ("laplace", synth.laplace2d(32))]


@pytest.mark.parametrize("k", [1, 3, 8, 16, 64])
@pytest.mark.parametrize("mi", range(len(SPMM_MATS)), ids=[m[0] for m in SPMM_MATS])
def test_spmm_matches_oracle(torch, mi, k):
    name, A = SPMM_MATS[mi]
    X = synth.uniform(A.N * k, 9 + k, -1.0, 1.0).reshape(A.N, k)
    Yref = oracle.csr_spmm(A.M, A.ptr, A.col, A.val, X)
    den = np.stack([oracle.csr_absspmv(A.M, A.ptr, A.col, A.val, X[:, c]) for c in range(k)], axis=1)
    Ad = S.Matrix.from_host(A)
    Y = Ad.spmm(torch.from_numpy(X).cuda()).cpu().numpy()
    for c in range(k):
        assert rowwise_err(Y[:, c], Yref[:, c], den[:, c]) <= TOL[0], (name, k, c)
    # padded leading dimensions
    Xp = np.zeros((A.N, k + 5))
    Xp[:, :k] = X
    Yp = torch.full((A.M, k + 3), float("nan"), dtype=torch.float64, device="cuda")
    Xd = torch.from_numpy(Xp).cuda()
    S.check(S.lib().spmv_spmm(Ad.h, S.dptr(Xd), k + 5, S.dptr(Yp), k + 3, k, S.stream()))
    Ypn = Yp.cpu().numpy()
    assert np.all(np.isnan(Ypn[:, k:]))  # columns past k untouched
    for c in range(k):
        assert rowwise_err(Ypn[:, c], Yref[:, c], den[:, c]) <= TOL[0]


@pytest.mark.parametrize("dt", [0, 1])
@pytest.mark.parametrize("k,ldx,ldy", [(8, 8, 8), (8, 10, 12), (6, 6, 6), (4, 4, 8), (12, 16, 12)])
def test_spmm_wide_lanes(torch, dt, k, ldx, ldy):
    """The 16-byte-lane SpMM (k, ldx, ldy multiples of 2 in FP64 / 4 in
    FP32, aligned X and Y) and its fallback agree with the oracle, and the
    columns past k are left alone."""
    for name, A in SPMM_MATS[:2]:
        X = synth.uniform(A.N * k, 29 + k, -1.0, 1.0).reshape(A.N, k)
        if dt == 1:
            X = X.astype(np.float32).astype(np.float64)
        Yref = oracle.csr_spmm(A.M, A.ptr, A.col, A.val if dt == 0 else A.val.astype(np.float32).astype(np.float64), X)
        val = A.val if dt == 0 else A.val.astype(np.float32)
        Ad = S.Matrix.from_csr(A.M, A.N, A.ptr, A.col, val, dt)
        tdt = torch.float64 if dt == 0 else torch.float32
        Xp = torch.zeros((A.N, ldx), dtype=tdt, device="cuda")
        Xp[:, :k] = torch.from_numpy(X).to("cuda", tdt)
        Yp = torch.full((A.M, ldy), float("nan"), dtype=tdt, device="cuda")
        S.check(S.lib().spmv_spmm(Ad.h, S.dptr(Xp), ldx, S.dptr(Yp), ldy, k, S.stream()))
        Y = Yp.cpu().numpy().astype(np.float64)
        assert np.all(np.isnan(Y[:, k:]))
        for c in range(k):
            den = oracle.csr_absspmv(A.M, A.ptr, A.col, A.val, X[:, c])
            assert rowwise_err(Y[:, c], Yref[:, c], den) <= TOL[dt], (name, dt, k, c)


def _spmm_block_case(kind):
    """Row-length patterns around the SpMM block rule: blocks of max(G, 64)
    rows are taken when that many rows of the longest row, plus the 3
    entries staging may start below a block's first one, fit the 2,048
    staged entries (k = 8 and 16 in FP64: 64 rows, so rows of up to 31;
    k = 4: 128 rows of up to 15), else the SpMV row blocks.  M = 1,000
    leaves a ragged last block."""
    M, N = 1000, 3000
    rng = np.random.default_rng(7)
    lens = rng.integers(0, 20, M).astype(np.int32)
    if kind == "max31":          # the rule's limit: 64 x 31 + 3 <= 2,048 entries
        lens[rng.choice(M, 40, replace=False)] = 31
        lens[64:128] = 31        # one whole block at the limit
    elif kind == "max32":        # one past it: the SpMV row blocks
        lens[rng.choice(M, 40, replace=False)] = 31
        lens[500] = 32
    elif kind == "max15":        # k = 4 (128-row blocks) at its limit: 128 x 15
        lens = rng.integers(0, 16, M).astype(np.int32)
        lens[128:256] = 15
    elif kind == "empty_blocks":  # whole blocks without entries, then entries
        lens[:256] = 0
        lens[900:] = 0
    return synth.from_lengths(M, N, lens, 11, 12)


@pytest.mark.parametrize("k", [4, 8, 16])
@pytest.mark.parametrize("kind", ["max31", "max32", "max15", "empty_blocks"])
def test_spmm_block_rule_edges(torch, kind, k):
    A = _spmm_block_case(kind)
    X = synth.uniform(A.N * k, 40 + k, -1.0, 1.0).reshape(A.N, k)
    Yref = oracle.csr_spmm(A.M, A.ptr, A.col, A.val, X)
    Y = S.Matrix.from_host(A).spmm(torch.from_numpy(X).cuda()).cpu().numpy()
    for c in range(k):
        den = oracle.csr_absspmv(A.M, A.ptr, A.col, A.val, X[:, c])
        assert rowwise_err(Y[:, c], Yref[:, c], den) <= TOL[0], (kind, k, c)


def test_spmm_integer_exact(torch):
    A = synth.random_pattern(900, 700, 0.02, 7, integer_values=True)
    X = np.round(synth.uniform(700 * 8, 3, -8, 8)).reshape(700, 8)
    Y = S.Matrix.from_host(A).spmm(torch.from_numpy(X).cuda()).cpu().numpy()
    assert np.array_equal(Y, oracle.csr_spmm(A.M, A.ptr, A.col, A.val, X))


@pytest.mark.parametrize("dt", [0, 1])
def test_batched_matches_per_matrix_oracle(torch, dt):
    specs = synth.batch_specs(24, seed=8, rows_lo=200, rows_hi=20_000)
    mats = [synth.make(s) for s in specs]
    mats.append(synth.zipf_rows(3000, 3000, 2.0, 16, 3000, 1, 2))  # long rows inside the batch
    mats.append(synth.from_dense(np.zeros((17, 5))))  # all-empty matrix
    handles, xs, ys, refs = [], [], [], []
    for i, A in enumerate(mats):
        val = A.val.astype(np.float32) if dt == 1 else A.val
        handles.append(S.Matrix.from_csr(A.M, A.N, A.ptr, A.col, val, dt))
        x64 = synth.vector(A.N, 50 + i)
        if dt == 1:
            x64 = x64.astype(np.float32).astype(np.float64)
        xs.append(device_vec(x64, dt))
        ys.append(torch.full((A.M,), float("nan"), dtype=S.torch_dtype(dt), device="cuda"))
        refs.append(reference(A, x64, dt))
    B = S.Batch(handles)
    for rep in range(2):  # second run reuses the uploaded pointer table
        B.run(xs, ys)
        torch.cuda.synchronize()
        for y, (yref, den) in zip(ys, refs):
            assert rowwise_err(y.cpu().numpy().astype(np.float64), yref, den) <= TOL[dt]


SELL_PARAMS = [dict(sell_C=64, sell_sigma=1), dict(sell_C=64, sell_sigma=1 << 30), dict(sell_C=32, sell_sigma=256),
               dict(sell_C=8, sell_sigma=8), dict(sell_C=16, sell_sigma=1, flags=64), dict(sell_C=64, sell_sigma=4096)]


@pytest.mark.parametrize("dt", [0, 1])
def test_mixed_csr_sell_batch_matches_per_matrix_oracle(torch, dt):
    """One launch over CSR row blocks, CSR wave tiles (with the fix-up pass
    for rows crossing tiles) and SELL-C-sigma chunk groups of several C and
    sigma (sorted and unsorted, chunks wider than 8 slots, rows of thousands
    of entries, an empty matrix): every matrix meets the bar."""
    specs = synth.batch_specs(20, seed=18, rows_lo=100, rows_hi=30_000)
    mats = [synth.make(s) for s in specs]
    mats.append(synth.zipf_rows(4000, 5000, 2.0, 16, 3000, 3, 4))
    mats.append(synth.from_dense(np.zeros((33, 9))))
    mats.append(synth.laplace2d(20))
    mats.append(synth.from_dense(np.zeros((40, 7))))
    mats.append(synth.laplace2d(9))
    mats.append(synth.zipf_rows(6000, 6000, 2.0, 24, 5000, 5, 6))  # index 25, as wave tiles: rows across tiles
    handles, keep, xs, ys, refs = [], [], [], [], []
    for i, A in enumerate(mats):
        val = A.val.astype(np.float32) if dt == 1 else A.val
        base = S.Matrix.from_csr(A.M, A.N, A.ptr, A.col, val, dt)
        if i % 4 == 2:
            handles.append(base)
        elif i % 4 == 1:
            keep.append(base)
            handles.append(base.convert("csr", flags=32))  # wave tiles
        else:
            keep.append(base)
            handles.append(base.convert("sell", **SELL_PARAMS[i % len(SELL_PARAMS)]))
        x64 = synth.vector(A.N, 70 + i)
        if dt == 1:
            x64 = x64.astype(np.float32).astype(np.float64)
        xs.append(device_vec(x64, dt))
        ys.append(torch.full((A.M,), float("nan"), dtype=S.torch_dtype(dt), device="cuda"))
        refs.append(reference(A, x64, dt))
    assert {h.fmt for h in handles} == {"csr", "sell"}
    assert handles[25].params["flags"] & 32 and handles[21].params["flags"] & 32  # tiles; 21 has no entries
    B = S.Batch(handles)
    for rep in range(2):
        B.run(xs, ys)
        torch.cuda.synchronize()
        for j, (y, (yref, den)) in enumerate(zip(ys, refs)):
            assert rowwise_err(y.cpu().numpy().astype(np.float64), yref, den) <= TOL[dt], (j, handles[j].fmt)


def test_batch_rejects_other_formats(torch):
    A = synth.laplace2d(8)
    base = S.Matrix.from_host(A)
    for fmt in ("csr5", "ell", "hyb"):
        with pytest.raises(S.SpmvError):
            S.Batch([base, base.convert(fmt)])
    with pytest.raises(S.SpmvError):
        S.Batch([base, base.convert("sell", bands=2)])


@pytest.mark.parametrize("fmt", ["csr", "csr5", "ell", "sell", "hyb"])
def test_autotune_picks_a_valid_configuration(torch, fmt):
    A = synth.zipf_rows(60_000, 60_000, 2.0, 12, 2000, 6, 7)
    x64 = synth.vector(A.N, 2)
    yref, den = reference(A, x64, 0)
    Ad = S.Matrix.from_host(A)
    x = device_vec(x64, 0)
    y = torch.empty(A.M, dtype=torch.float64, device="cuda")
    p, ms = Ad.autotune(fmt, x, y, scrub_bytes=64 << 20, reps=5)
    assert ms > 0
    B = Ad.convert(fmt, **{k: v for k, v in p.items()})
    out = B.run(x).cpu().numpy()
    assert rowwise_err(out, yref, den) <= TOL[0]
    if fmt == "sell":
        assert p["sell_C"] in (8, 16, 32, 64)
    if fmt == "csr5":
        assert p["csr5_sigma"] in (4, 8, 16, 32)


def test_autotune_csr_over_column_bands(torch):
    """x of 5.6 MB: the CSR grid includes row blocks and wave tiles over 2
    and 4 column bands, the HYB grid tails over 2 and 4 bands; whatever wins
    converts and runs to the bar."""
    A = synth.zipf_rows(40_000, 700_000, 2.0, 12, 3000, 11, 12)
    x64 = synth.vector(A.N, 2)
    yref, den = reference(A, x64, 0)
    Ad = S.Matrix.from_host(A)
    x = device_vec(x64, 0)
    y = torch.empty(A.M, dtype=torch.float64, device="cuda")
    p, ms = Ad.autotune("csr", x, y, scrub_bytes=64 << 20, reps=3)
    assert ms > 0 and p["bands"] in (1, 2, 4)
    for nb in (2, 4):
        for fl in (0, 32):
            out = Ad.convert("csr", bands=nb, flags=fl).run(x).cpu().numpy()
            assert rowwise_err(out, yref, den) <= TOL[0], (nb, fl)
    out = Ad.convert("csr", **p).run(x).cpu().numpy()
    assert rowwise_err(out, yref, den) <= TOL[0]
    # HYB: every K also with its COO tail over 2 and 4 bands
    p, ms = Ad.autotune("hyb", x, y, scrub_bytes=64 << 20, reps=3)
    assert ms > 0 and p["bands"] in (1, 2, 4)
    out = Ad.convert("hyb", **p).run(x).cpu().numpy()
    assert rowwise_err(out, yref, den) <= TOL[0]
    S.lib().spmv_autotune_cache_clear()


def test_autotune_cache_by_structure(torch):
    import time
    A = synth.zipf_rows(30_000, 30_000, 2.0, 12, 2000, 8, 9)
    x = device_vec(synth.vector(A.N, 2), 0)
    y = torch.empty(A.M, dtype=torch.float64, device="cuda")
    S.lib().spmv_autotune_cache_clear()
    Ad = S.Matrix.from_host(A)
    t0 = time.perf_counter()
    p1, ms1 = Ad.autotune("sell", x, y, scrub_bytes=64 << 20, reps=5)
    t_first = time.perf_counter() - t0
    # same structure, other values: served from the cache, no timing
    A2 = synth.HostCSR(A.M, A.N, A.ptr, A.col, -2.0 * A.val)
    t0 = time.perf_counter()
    p2, ms2 = S.Matrix.from_host(A2).autotune("sell", x, y, scrub_bytes=64 << 20, reps=5)
    t_second = time.perf_counter() - t0
    assert p2 == p1 and ms2 == ms1
    assert t_second < t_first
    # another structure is tuned afresh
    B = synth.uniform_random(30_000, 30_000, 12.0, 3, 4)
    p3, _ = S.Matrix.from_host(B).autotune("sell", x, y, scrub_bytes=64 << 20, reps=5)
    assert p3["sell_C"] in (8, 16, 32, 64)
    S.lib().spmv_autotune_cache_clear()
