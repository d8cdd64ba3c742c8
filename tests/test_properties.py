"""Hypothesis properties of the CPU oracle on random small matrices (no GPU):
shapes down to 1 x 1, empty rows and columns, one dense row, integer values so
that every summation order is exact.  Every format's interpreter equals dense
brute force, and every conversion round-trips bit-exactly, for random C and
sigma (SELL-C-sigma), K (HYB) and omega, sigma (CSR5)."""
import numpy as np
from hypothesis import given, settings, strategies as st, HealthCheck

import oracle
from paper_1805_11938_amd import synth


@st.composite
def matrices(draw):
    M = draw(st.integers(1, 40))
    N = draw(st.integers(1, 40))
    density = draw(st.sampled_from([0.0, 0.02, 0.1, 0.4, 1.0]))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    rng = np.random.default_rng(seed)
    D = np.where(rng.random((M, N)) < density, rng.integers(-8, 9, (M, N)), 0).astype(float)
    if draw(st.booleans()):
        D[rng.integers(0, M), :] = rng.integers(1, 9, N)   # one full row
    A = synth.from_dense(D)
    # explicit zeros are entries too: put one in where the pattern has room
    if draw(st.booleans()) and A.nnz:
        A.val[rng.integers(0, A.nnz)] = 0.0
    x = rng.integers(-8, 9, N).astype(float)
    return A, x


def dense(A):
    D = np.zeros((A.M, A.N))
    for i in range(A.M):
        for k in range(A.ptr[i], A.ptr[i + 1]):
            D[i, A.col[k]] = A.val[k]
    return D


def same(a, b):
    return all(np.array_equal(np.asarray(p).view(np.uint8), np.asarray(q).view(np.uint8)) for p, q in zip(a, b))


@settings(max_examples=150, deadline=None, derandomize=True, suppress_health_check=[HealthCheck.too_slow])
@given(matrices(), st.sampled_from([1, 2, 4, 8, 32]), st.integers(1, 64), st.integers(-1, 6),
       st.sampled_from([(1, 1), (2, 2), (4, 3), (16, 2), (64, 4)]))
def test_formats_equal_brute_force_and_round_trip(Ax, C, sigma, K, ws):
    A, x = Ax
    M = A.M
    want = dense(A) @ x  # integer-valued: exact in any order
    csr = (A.ptr, A.col, A.val)
    assert np.array_equal(oracle.csr_spmv(M, *csr, x), want)
    Ke, ec, ev = oracle.csr_to_ell(M, *csr)
    assert np.array_equal(oracle.ell_spmv(M, Ke, ec, ev, x), want)
    assert same(oracle.ell_to_csr(M, Ke, ec, ev), csr)
    s = oracle.csr_to_sell(M, *csr, C, sigma)
    assert np.array_equal(oracle.sell_spmv(M, C, s, x), want)
    assert same(oracle.sell_to_csr(M, C, s), csr)
    h = oracle.csr_to_hyb(M, *csr, None if K < 0 else K)
    assert np.array_equal(oracle.hyb_spmv(M, h, x), want)
    assert same(oracle.hyb_to_csr(M, h), csr)
    w, sg = ws
    c5 = oracle.csr_to_csr5(M, *csr, w, sg)
    assert np.array_equal(oracle.csr5_spmv(M, A.ptr, c5, x), want)
    assert same(oracle.csr5_to_csr(A.nnz, c5), (A.col, A.val))
    # the error denominator bounds the product, and is exact for integer data
    den = oracle.csr_absspmv(M, *csr, x)
    assert np.all(den >= np.abs(want)) and np.array_equal(den, np.abs(dense(A)) @ np.abs(x))
