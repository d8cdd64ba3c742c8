"""Hypothesis properties of the device path (through the C-ABI) on random
small matrices: shapes down to 1 x 1, empty rows and columns, one dense row,
explicit zeros.  Integer-valued data make every summation order exact, so each
format configuration drawn must give the oracle's y bit for bit, and its
conversion must round-trip bit-exactly."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import oracle
from paper_1805_11938_amd import synth
from paper_1805_11938_amd import spmv as S

from gpu_util import FORMAT_CONFIGS

pytestmark = pytest.mark.gpu


@st.composite
def matrices(draw):
    M = draw(st.integers(1, 300))
    N = draw(st.integers(1, 300))
    density = draw(st.sampled_from([0.0, 0.005, 0.05, 0.3]))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    rng = np.random.default_rng(seed)
    D = np.where(rng.random((M, N)) < density, rng.integers(-8, 9, (M, N)), 0).astype(float)
    if draw(st.booleans()):
        D[rng.integers(0, M), :] = rng.integers(1, 9, N)
    A = synth.from_dense(D)
    if draw(st.booleans()) and A.nnz:
        A.val[rng.integers(0, A.nnz)] = 0.0
    return A, rng.integers(-8, 9, N).astype(float)


@settings(max_examples=40, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.function_scoped_fixture])
@given(matrices(), st.lists(st.integers(0, len(FORMAT_CONFIGS) - 1), min_size=4, max_size=4, unique=True),
       st.sampled_from([0, 1]))
def test_device_formats_bit_exact_on_integer_data(Ax, cfgs, dt):
    import torch
    assert torch.cuda.is_available()
    A, x64 = Ax
    want = oracle.csr_spmv(A.M, A.ptr, A.col, A.val, x64)  # exact: |partial sums| < 2^24
    base = S.Matrix.from_host(A, dt)
    x = torch.from_numpy(x64.astype(np.float32) if dt else x64).cuda()
    print(f"hypothesis M={A.M} N={A.N} nnz={A.nnz} dt={dt} cfgs={cfgs}", flush=True)
    for ci in cfgs:
        fmt, kw = FORMAT_CONFIGS[ci]
        B = base.convert(fmt, **kw)
        y = B.run(x).cpu().numpy().astype(np.float64)
        assert np.array_equal(y, want), (fmt, kw)
        p, c, v = B.to_csr()
        assert np.array_equal(p, A.ptr) and np.array_equal(c, A.col), (fmt, kw)
        assert np.array_equal(v.astype(np.float64), A.val), (fmt, kw)
