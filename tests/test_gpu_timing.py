"""Kernel-bound event timing (spmv_run_timed and friends): same results as
the untimed calls, and a positive elapsed time that is not longer than the
same run bracketed by ordinary event records."""
import numpy as np
import pytest

from paper_1805_11938_amd import spmv as S
from paper_1805_11938_amd import synth

from gpu_util import TOL, device_vec, reference, rowwise_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("fmt,kw", [("csr", {}), ("csr5", {}), ("ell", {}), ("sell", {"sell_C": 8, "sell_sigma": 64}),
                                    ("hyb", {})])
def test_run_timed_matches_run(torch, fmt, kw):
    A = synth.zipf_rows(40_000, 40_000, 2.0, 16, 4_000, 3, 4)
    x64 = synth.vector(A.N, 5)
    yref, den = reference(A, x64, 0)
    B = S.Matrix.from_host(A).convert(fmt, **kw)
    x = device_vec(x64, 0)
    y = torch.full((A.M,), float("nan"), dtype=torch.float64, device="cuda")
    ev = S.timing_events()
    for _ in range(3):
        B.run_timed(x, y, ev)
    torch.cuda.synchronize()
    assert rowwise_err(y.cpu().numpy(), yref, den) <= TOL[0]
    t_kernel = min(_timed(torch, lambda: B.run_timed(x, y, ev), ev) for _ in range(5))
    m0, m1 = S.timing_events()
    ts = []
    for _ in range(5):
        m0.record()
        B.run(x, y)
        m1.record()
        torch.cuda.synchronize()
        ts.append(m0.elapsed_time(m1))
    assert 0 < t_kernel <= min(ts) * 1.05


def _timed(torch, fn, ev):
    fn()
    torch.cuda.synchronize()
    return ev[0].elapsed_time(ev[1])


def test_timed_spmm_batch_and_empty(torch):
    A = synth.stencil27(16)
    Ad = S.Matrix.from_host(A)
    X = torch.from_numpy(synth.uniform(A.N * 8, 3, -1, 1).reshape(A.N, 8)).cuda()
    Y = torch.empty((A.M, 8), dtype=torch.float64, device="cuda")
    ev = S.timing_events()
    Ad.spmm_timed(X, Y, ev)
    torch.cuda.synchronize()
    assert ev[0].elapsed_time(ev[1]) > 0
    assert torch.equal(Y, Ad.spmm(X))
    mats = [S.Matrix.from_host(synth.laplace2d(20)), Ad]
    xs = [device_vec(synth.vector(m.N, 1 + i), 0) for i, m in enumerate(mats)]
    ys = [torch.empty(m.M, dtype=torch.float64, device="cuda") for m in mats]
    Bt = S.Batch(mats)
    Bt.run(xs, ys, ev)
    torch.cuda.synchronize()
    assert ev[0].elapsed_time(ev[1]) > 0
    for m, x, y in zip(mats, xs, ys):
        assert torch.equal(y, m.run(x))
    E = S.Matrix.from_host(synth.from_dense(np.zeros((0, 4))))
    E.run_timed(xs[0][:4].contiguous(), torch.empty(0, dtype=torch.float64, device="cuda"), ev)
    torch.cuda.synchronize()
    assert ev[0].elapsed_time(ev[1]) >= 0


def test_gather_probe_sees_the_cache_levels(torch):
    """The random-gather floor: positive, and gathers from an x that fits an
    XCD's L2 (1 MiB) are clearly cheaper than from one that only fits the
    Infinity Cache (16 MiB).  Bad sizes are rejected."""
    small = S.gather_probe(1 << 17, 1 << 20, S.F64, reps=5)
    big = S.gather_probe(1 << 21, 1 << 20, S.F64, reps=5)
    assert 0 < small < 0.8 * big, (small, big)
    assert S.gather_probe(1 << 17, 1 << 16, S.F32, reps=3) > 0
    for nx, rows in [(0, 10), (10, 0), (1 << 31, 10), (10, (1 << 27) + 1)]:
        with pytest.raises(S.SpmvError) as e:
            S.gather_probe(nx, rows, S.F64, reps=1)
        assert e.value.status == -1
