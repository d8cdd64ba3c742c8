"""Pins of the CPU oracle against things other than itself (no GPU).

* Table I of the paper (Sec. II-B): every printed array, exactly.
* Hand-derived products of the Table I matrix.
* Dense brute force (python loops) on tiny random matrices with empty rows,
  full rows and single columns; integer-valued cases must be bit-exact.
* Closed forms: 2-D Laplacian eigenvectors, stencil row sums, identity,
  permutation, features of the 64x64 Laplacian, Gini by the pairwise formula.
* Format invariants (slot counts, permutations, CSR5 flag counts).
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from paper_1805_11938_amd import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1.json")))


def t1():
    g = GOLD["coo"]
    return oracle.coo_to_csr(4, 4, g["row"], g["col"], g["data"])


def brute(M, N, ptr, col, val, x):
    """Dense mat-vec with python loops: A is materialised, then y_i = sum_j A_ij x_j."""
    A = [[0.0] * N for _ in range(M)]
    for i in range(M):
        for k in range(ptr[i], ptr[i + 1]):
            A[i][col[k]] += val[k]
    return np.array([sum(A[i][j] * x[j] for j in range(N)) for i in range(M)])


def rowwise_err(y, yref, den):
    e = np.abs(np.asarray(y) - np.asarray(yref))
    z = den == 0
    assert np.all(e[z] == 0)
    return float(np.max(e[~z] / den[~z])) if np.any(~z) else 0.0


# ------------------------------------------------------------- Table I

def test_table1_csr_from_coo():
    ptr, col, val = t1()
    assert ptr.tolist() == GOLD["csr"]["ptr"]
    assert col.tolist() == GOLD["csr"]["indices"]
    assert val.tolist() == GOLD["csr"]["data"]
    # and the CSR is the dense matrix
    D = np.zeros((4, 4))
    for i in range(4):
        for k in range(ptr[i], ptr[i + 1]):
            D[i, col[k]] = val[k]
    assert D.tolist() == GOLD["dense"]


def test_table1_products_by_hand():
    ptr, col, val = t1()
    assert oracle.csr_spmv(4, ptr, col, val, np.ones(4)).tolist() == [7, 13, 4, 12]
    assert oracle.csr_spmv(4, ptr, col, val, np.array([1.0, 2, 3, 4])).tolist() == [15, 38, 12, 29]


def _ell_rows(K, ec, ev, M):
    rows_c, rows_v = [], []
    for i in range(M):
        rc, rv = [], []
        for k in range(K):
            c = int(ec[k * M + i])
            rc.append(None if c < 0 else c)
            rv.append(None if c < 0 else float(ev[k * M + i]))
        rows_c.append(rc)
        rows_v.append(rv)
    return rows_c, rows_v


def test_table1_ell():
    ptr, col, val = t1()
    K, ec, ev = oracle.csr_to_ell(4, ptr, col, val)
    assert K == GOLD["ell"]["K"]
    rc, rv = _ell_rows(K, ec, ev, 4)
    assert rc == GOLD["ell"]["indices"]
    assert rv == GOLD["ell"]["data"]
    assert np.all(ev[ec < 0] == 0.0) and not np.any(np.signbit(ev[ec < 0]))


def _sell_rows(s, C):
    out_c, out_v = [], []
    for c in range(len(s["widths"])):
        for p in range(C):
            rc, rv = [], []
            for k in range(int(s["widths"][c])):
                q = int(s["cs"][c]) + k * C + p
                cc = int(s["col"][q])
                rc.append(None if cc < 0 else cc)
                rv.append(None if cc < 0 else float(s["val"][q]))
            out_c.append(rc)
            out_v.append(rv)
    return out_c, out_v


@pytest.mark.parametrize("key", ["sell", "sell_c_sigma"])
def test_table1_sell(key):
    g = GOLD[key]
    ptr, col, val = t1()
    s = oracle.csr_to_sell(4, ptr, col, val, g["C"], g["sigma"])
    assert s["widths"].tolist() == g["slices"]
    rc, rv = _sell_rows(s, g["C"])
    assert rc == g["indices"]
    assert rv == g["data"]
    if "row_order" in g:
        assert s["perm"].tolist() == g["row_order"]


def test_table1_hyb():
    g = GOLD["hyb"]
    ptr, col, val = t1()
    h = oracle.csr_to_hyb(4, ptr, col, val)
    assert h["K"] == g["K"]
    rc, rv = _ell_rows(h["K"], h["ell_col"], h["ell_val"], 4)
    assert rc == g["ell_indices"] and rv == g["ell_data"]
    assert h["coo_row"].tolist() == g["coo"]["row"]
    assert h["coo_col"].tolist() == g["coo"]["col"]
    assert h["coo_val"].tolist() == g["coo"]["data"]


def test_table1_csr5():
    g = GOLD["csr5"]
    ptr, col, val = t1()
    c5 = oracle.csr_to_csr5(4, ptr, col, val, g["omega"], g["sigma"])
    w, s = g["omega"], g["sigma"]
    assert c5["tile_ptr"].tolist() == g["tile_ptr"]
    T = c5["ntiles"]
    flags = [[bool((c5["bit_flag"][t * w + l] >> i) & 1) for i in range(s) for l in range(w)] for t in range(T)]
    assert flags == g["bit_flag"]
    assert c5["y_off"].reshape(T, w).tolist() == g["y_off"]
    assert c5["seg_off"].reshape(T, w).tolist() == g["seg_off"]
    assert c5["col"].reshape(T, w * s).tolist() == g["indices"]
    assert c5["val"].reshape(T, w * s).tolist() == g["data"]
    # flag count invariant: row starts in the tiles + tiles not starting a row (4 + 1)
    assert sum(map(sum, flags)) == 5


def test_table1_every_interpreter():
    ptr, col, val = t1()
    x = np.array([1.0, 2, 3, 4])
    want = [15, 38, 12, 29]
    K, ec, ev = oracle.csr_to_ell(4, ptr, col, val)
    assert oracle.ell_spmv(4, K, ec, ev, x).tolist() == want
    for C, sg in [(2, 1), (2, 4), (1, 1), (4, 4), (8, 8)]:
        assert oracle.sell_spmv(4, C, oracle.csr_to_sell(4, ptr, col, val, C, sg), x).tolist() == want
    assert oracle.hyb_spmv(4, oracle.csr_to_hyb(4, ptr, col, val), x).tolist() == want
    for w, s in [(2, 2), (1, 1), (2, 1), (1, 3), (4, 2), (64, 8)]:
        assert oracle.csr5_spmv(4, ptr, oracle.csr_to_csr5(4, ptr, col, val, w, s), x).tolist() == want


# ------------------------------------------------------- brute force

def _cases():
    out = []
    for seed in range(6):
        for (M, N, d) in [(1, 1, 1.0), (7, 5, 0.3), (33, 40, 0.15), (64, 64, 0.05), (50, 1, 0.5), (1, 64, 0.7)]:
            out.append(synth.random_pattern(M, N, d, seed * 31 + M, integer_values=(seed % 2 == 0)))
    # one dense row among empty rows, and an all-empty matrix
    A = np.zeros((20, 30)); A[7, :] = np.arange(1, 31)
    out.append(synth.from_dense(A))
    out.append(synth.from_dense(np.zeros((9, 4))))
    # single column
    A = np.zeros((40, 1)); A[::3, 0] = 2.0
    out.append(synth.from_dense(A))
    return out


@pytest.mark.parametrize("idx", range(39))
def test_interpreters_match_brute_force(idx):
    A = _cases()[idx]
    M, N = A.M, A.N
    rng = np.random.default_rng(idx)
    integer = np.all(A.val == np.round(A.val))
    x = rng.integers(-8, 9, N).astype(float) if integer else rng.standard_normal(N)
    ref = brute(M, N, A.ptr, A.col, A.val, x)
    den = oracle.csr_absspmv(M, A.ptr, A.col, A.val, x)
    ys = {"csr": oracle.csr_spmv(M, A.ptr, A.col, A.val, x)}
    K, ec, ev = oracle.csr_to_ell(M, A.ptr, A.col, A.val)
    ys["ell"] = oracle.ell_spmv(M, K, ec, ev, x)
    for C, sg in [(1, 1), (2, 4), (4, 1), (8, 16), (32, 64)]:
        ys[f"sell{C}_{sg}"] = oracle.sell_spmv(M, C, oracle.csr_to_sell(M, A.ptr, A.col, A.val, C, sg), x)
    ys["hyb"] = oracle.hyb_spmv(M, oracle.csr_to_hyb(M, A.ptr, A.col, A.val), x)
    for Kh in [0, 1, 3]:
        ys[f"hybK{Kh}"] = oracle.hyb_spmv(M, oracle.csr_to_hyb(M, A.ptr, A.col, A.val, Kh), x)
    for w, s in [(1, 1), (2, 2), (4, 3), (8, 4), (64, 2)]:
        ys[f"csr5_{w}_{s}"] = oracle.csr5_spmv(M, A.ptr, oracle.csr_to_csr5(M, A.ptr, A.col, A.val, w, s), x)
    for name, y in ys.items():
        if integer:
            assert np.array_equal(y, ref), name
        else:
            assert rowwise_err(y, ref, den) <= 1e-14, name


@pytest.mark.parametrize("idx", range(39))
def test_round_trips_bit_exact(idx):
    A = _cases()[idx]
    M = A.M
    K, ec, ev = oracle.csr_to_ell(M, A.ptr, A.col, A.val)
    for got in [oracle.ell_to_csr(M, K, ec, ev)] + \
               [oracle.sell_to_csr(M, C, oracle.csr_to_sell(M, A.ptr, A.col, A.val, C, sg))
                for C, sg in [(1, 1), (2, 4), (8, 16)]] + \
               [oracle.hyb_to_csr(M, oracle.csr_to_hyb(M, A.ptr, A.col, A.val, Kh)) for Kh in (None, 0, 2)]:
        assert np.array_equal(got[0], A.ptr)
        assert np.array_equal(got[1], A.col)
        assert np.array_equal(got[2].view(np.uint64), A.val.view(np.uint64))
    for w, s in [(1, 1), (2, 2), (4, 3), (64, 2)]:
        c, v = oracle.csr5_to_csr(A.nnz, oracle.csr_to_csr5(M, A.ptr, A.col, A.val, w, s))
        assert np.array_equal(c, A.col) and np.array_equal(v.view(np.uint64), A.val.view(np.uint64))


# ----------------------------------------------------- invariants

@pytest.mark.parametrize("idx", range(0, 39, 3))
def test_format_invariants(idx):
    A = _cases()[idx]
    M, lens = A.M, A.lengths()
    K, ec, ev = oracle.csr_to_ell(M, A.ptr, A.col, A.val)
    assert len(ec) == M * K and K == (lens.max() if M else 0)
    assert int((ec >= 0).sum()) == A.nnz
    for C, sg in [(2, 1), (4, 8), (8, 8)]:
        s = oracle.csr_to_sell(M, A.ptr, A.col, A.val, C, sg)
        real = s["perm"][s["perm"] >= 0]
        assert sorted(real.tolist()) == list(range(M))
        assert len(s["col"]) == int(s["cs"][-1]) >= A.nnz
        if sg == 1:
            assert np.array_equal(real, np.arange(M))
        # inside each sigma window, lengths are non-increasing
        L = np.where(s["perm"] >= 0, lens[np.maximum(s["perm"], 0)], -1)
        for w0 in range(0, M, sg):
            seg = L[w0:min(w0 + sg, M)]
            assert np.all(np.diff(seg) <= 0)
    h = oracle.csr_to_hyb(M, A.ptr, A.col, A.val)
    assert int((h["ell_col"] >= 0).sum()) + len(h["coo_row"]) == A.nnz
    for w, s in [(2, 2), (4, 3)]:
        c5 = oracle.csr_to_csr5(M, A.ptr, A.col, A.val, w, s)
        T, W = c5["ntiles"], w * s
        nflag = sum(bin(int(f)).count("1") for f in c5["bit_flag"])
        starts = sum(1 for i in range(M) if lens[i] > 0 and A.ptr[i] < T * W)
        tiles_mid = sum(1 for t in range(T) if t * W not in set(A.ptr[:-1][lens > 0].tolist()))
        assert nflag == starts + tiles_mid


def test_hyb_k_rule_closed_cases():
    # Table I lengths 2,3,1,2 -> K = 2 (printed); all-equal rows -> that length
    assert oracle.hyb_k_rule(4, np.array([0, 2, 5, 6, 8])) == 2
    ptr = np.arange(0, 5 * 10 + 1, 5)
    assert oracle.hyb_k_rule(10, ptr) == 5
    # one third of rows have length >= 7: lengths 7,7,7 then 1 x 6
    lens = [7, 7, 7, 1, 1, 1, 1, 1, 1]
    assert oracle.hyb_k_rule(9, np.concatenate([[0], np.cumsum(lens)])) == 7
    lens = [7, 7, 1, 1, 1, 1, 1, 1, 1]
    assert oracle.hyb_k_rule(9, np.concatenate([[0], np.cumsum(lens)])) == 1


# ----------------------------------------------------- special cases

def test_identity_and_permutation_exact():
    n = 257
    rng = np.random.default_rng(3)
    x = rng.standard_normal(n)
    I = synth.from_dense(np.eye(n))
    perm = rng.permutation(n)
    P = synth.from_dense(np.eye(n)[perm])
    for A, want in [(I, x), (P, x[perm])]:
        assert np.array_equal(oracle.csr_spmv(n, A.ptr, A.col, A.val, x), want)
        K, ec, ev = oracle.csr_to_ell(n, A.ptr, A.col, A.val)
        assert np.array_equal(oracle.ell_spmv(n, K, ec, ev, x), want)
        assert np.array_equal(oracle.sell_spmv(n, 8, oracle.csr_to_sell(n, A.ptr, A.col, A.val, 8, 64), x), want)
        assert np.array_equal(oracle.csr5_spmv(n, A.ptr, oracle.csr_to_csr5(n, A.ptr, A.col, A.val, 4, 4), x), want)


def test_laplacian_row_sums_and_eigenvectors():
    A = synth.laplace2d(64)
    n = 64
    y = oracle.csr_spmv(A.M, A.ptr, A.col, A.val, np.ones(A.M)).reshape(n, n)
    assert np.all(y[1:-1, 1:-1] == 0)
    assert y[0, 0] == y[0, -1] == y[-1, 0] == y[-1, -1] == 2
    assert np.all(y[0, 1:-1] == 1) and np.all(y[1:-1, 0] == 1)
    i = np.arange(1, n + 1)
    for p, q in [(1, 1), (3, 7), (64, 2), (33, 50)]:
        v = np.outer(np.sin(p * math.pi * i / (n + 1)), np.sin(q * math.pi * i / (n + 1))).ravel()
        lam = 4 - 2 * math.cos(p * math.pi / (n + 1)) - 2 * math.cos(q * math.pi / (n + 1))
        Av = oracle.csr_spmv(A.M, A.ptr, A.col, A.val, v)
        assert np.max(np.abs(Av - lam * v)) <= 1e-13 * np.max(np.abs(v)) * 8


def test_stencil27_unit_row_sums():
    A = synth.stencil27(6)
    ones = np.ones(A.nnz)
    y = oracle.csr_spmv(A.M, A.ptr, A.col, ones, np.ones(A.M)).reshape(6, 6, 6)
    assert y[2, 2, 2] == 27 and y[0, 2, 2] == 18 and y[0, 0, 2] == 12 and y[0, 0, 0] == 8
    assert A.nnz == (3 * 6 - 2) ** 3


def test_empty_matrix():
    ptr = np.zeros(6, np.int32)
    c = np.zeros(0, np.int32)
    v = np.zeros(0)
    x = np.ones(3)
    assert np.array_equal(oracle.csr_spmv(5, ptr, c, v, x), np.zeros(5))
    assert oracle.csr_to_ell(5, ptr, c, v)[0] == 0
    c5 = oracle.csr_to_csr5(5, ptr, c, v, 4, 4)
    assert c5["ntiles"] == 0
    assert np.array_equal(oracle.csr5_spmv(5, ptr, c5, x), np.zeros(5))


def test_nan_in_x_reaches_only_its_rows():
    A = synth.random_pattern(40, 30, 0.1, 5)
    x = np.ones(30)
    x[7] = np.nan
    touched = np.array([7 in A.col[A.ptr[i]:A.ptr[i + 1]] for i in range(40)])
    K, ec, ev = oracle.csr_to_ell(40, A.ptr, A.col, A.val)
    for y in [oracle.csr_spmv(40, A.ptr, A.col, A.val, x), oracle.ell_spmv(40, K, ec, ev, x),
              oracle.sell_spmv(40, 4, oracle.csr_to_sell(40, A.ptr, A.col, A.val, 4, 8), x),
              oracle.hyb_spmv(40, oracle.csr_to_hyb(40, A.ptr, A.col, A.val), x),
              oracle.csr5_spmv(40, A.ptr, oracle.csr_to_csr5(40, A.ptr, A.col, A.val, 4, 2), x)]:
        assert np.array_equal(np.isnan(y), touched)


# --------------------------------------------------- COO -> CSR

def test_coo_duplicates_summed_in_input_order():
    # (0,0) appears three times; left-to-right order decides the FP64 result
    row = [0, 1, 0, 0]
    col = [0, 1, 0, 0]
    ptr, c, v = oracle.coo_to_csr(2, 2, row, col, [1e16, 5.0, 1.0, -1e16])
    assert v.tolist() == [0.0, 5.0]  # (1e16 + 1) - 1e16 = 0 in FP64
    ptr, c, v = oracle.coo_to_csr(2, 2, row, col, [-1e16, 5.0, 1e16, 1.0])
    assert v.tolist() == [1.0, 5.0]
    assert ptr.tolist() == [0, 1, 2] and c.tolist() == [0, 1]


def test_coo_to_csr_matches_dense_accumulation():
    rng = np.random.default_rng(11)
    M, N, n = 37, 23, 600
    row = rng.integers(0, M, n)
    col = rng.integers(0, N, n)
    val = rng.integers(-5, 6, n).astype(float)
    val[::17] = 0.0
    ptr, c, v = oracle.coo_to_csr(M, N, row, col, val)
    D = np.zeros((M, N))
    np.add.at(D, (row, col), val)
    present = np.zeros((M, N), bool)
    present[row, col] = True
    assert ptr[-1] == present.sum()  # explicit zeros kept
    for i in range(M):
        cols = c[ptr[i]:ptr[i + 1]]
        assert cols.tolist() == sorted(np.nonzero(present[i])[0].tolist())
        assert np.array_equal(v[ptr[i]:ptr[i + 1]], D[i, cols])
    assert oracle.csr_check(M, N, ptr, c) == 0


def test_coo_out_of_range_rejected():
    with pytest.raises(ValueError):
        oracle.coo_to_csr(2, 2, [0, 2], [0, 0], [1.0, 1.0])


def test_csr_check_error_codes():
    good = (np.array([0, 2, 3]), np.array([0, 1, 1]))
    assert oracle.csr_check(2, 2, *good) == 0
    assert oracle.csr_check(2, 2, np.array([0, 2, 3]), np.array([1, 0, 1])) == -2   # unsorted
    assert oracle.csr_check(2, 2, np.array([0, 2, 3]), np.array([0, 0, 1])) == -2   # duplicate
    assert oracle.csr_check(2, 2, np.array([0, 2, 3]), np.array([0, 2, 1])) == -2   # col >= N
    assert oracle.csr_check(2, 2, np.array([0, 3, 2]), np.array([0, 1, 1])) == -2   # ptr not monotone
    assert oracle.csr_check(2, 2, np.array([1, 2, 3]), np.array([0, 1, 1])) == -2   # ptr[0] != 0


# ------------------------------------------------------------ features

def test_features_laplacian_closed_form():
    A = synth.laplace2d(64)
    f = oracle.features(A.M, A.N, A.ptr, A.col)
    assert f[0] == 4096 and f[1] == 4096 and f[2] == 20224
    assert f[3] == 20224 / 4096 ** 2
    assert f[4] == 3 and f[5] == 5 and f[6] == 20224 / 4096
    assert f[9] == 4096 * 5 / 20224 and f[10] == 64
    # std by counting: 4 corners (3), 248 edge rows (4), 3844 interior rows (5)
    mean = 20224 / 4096
    var = (4 * (3 - mean) ** 2 + 248 * (4 - mean) ** 2 + 3844 * (5 - mean) ** 2) / 4096
    assert abs(f[7] - math.sqrt(var)) < 1e-15 and abs(f[8] - math.sqrt(var) / mean) < 1e-15


def test_features_constant_rows_and_gini():
    ptr = np.arange(0, 7 * 100 + 1, 7)
    col = np.tile(np.arange(7), 100)
    f = oracle.features(100, 7, ptr, col)
    assert f[7] == 0 and f[8] == 0 and f[11] == 0 and f[9] == 1
    # Gini by the pairwise mean-difference formula sum_ij |Li - Lj| / (2 M^2 mean)
    rng = np.random.default_rng(2)
    lens = rng.integers(0, 30, 57)
    ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    col = np.concatenate([np.arange(l) for l in lens]).astype(np.int32)
    f = oracle.features(57, 30, ptr, col)
    pair = np.abs(lens[:, None] - lens[None, :]).sum() / (2 * 57 ** 2 * lens.mean())
    assert abs(f[11] - pair) < 1e-14
    assert f[10] == max(abs(i - c) for i in range(57) for c in col[ptr[i]:ptr[i + 1]])


def test_zipf_gini_matches_exact_distribution():
    A = synth.zipf_rows(200_000, 200_000, seed=4, val_seed=5)
    f = oracle.features(A.M, A.N, A.ptr, A.col)
    assert abs(f[6] - 16.0) < 0.6 and f[5] <= 10_000 and f[4] >= 3
    assert abs(f[11] - 0.755) < 0.03


# ------------------------------------------- pins of the remaining oracle parts

def _brute_abs(M, N, ptr, col, val, x):
    """Sum over row i of |a_ij * x_j| with python loops over the dense matrix."""
    A = [[0.0] * N for _ in range(M)]
    for i in range(M):
        for k in range(ptr[i], ptr[i + 1]):
            A[i][col[k]] += val[k]
    return np.array([sum(abs(A[i][j] * x[j]) for j in range(N)) for i in range(M)])


@pytest.mark.parametrize("idx", range(0, 39, 2))
def test_absspmv_matches_brute_force(idx):
    # the denominator of the row-wise error: mixed signs, so |sum| != sum of || unless the
    # magnitudes are taken term by term; integer values make every sum exact
    A = _cases()[idx]
    rng = np.random.default_rng(100 + idx)
    val = rng.integers(-8, 9, A.nnz).astype(float)
    x = rng.integers(-8, 9, A.N).astype(float)
    got = oracle.csr_absspmv(A.M, A.ptr, A.col, val, x)
    assert np.array_equal(got, _brute_abs(A.M, A.N, A.ptr.tolist(), A.col.tolist(), val.tolist(), x.tolist()))
    # never below the magnitude of the product itself
    assert np.all(got >= np.abs(oracle.csr_spmv(A.M, A.ptr, A.col, val, x)))


def test_absspmv_table1_by_hand():
    # Table I's matrix with x = [1, -2, 3, -4]: rows 6*2 + 1*3, 2*1 + 8*3 + 3*4, 4*3, 7*2 + 5*3
    ptr, col, val = t1()
    x = np.array([1.0, -2.0, 3.0, -4.0])
    assert oracle.csr_absspmv(4, ptr, col, val, x).tolist() == [15, 38, 12, 29]
    assert oracle.csr_spmv(4, ptr, col, val, x).tolist() == [-9, 14, 12, 1]


@pytest.mark.parametrize("idx", range(0, 39, 3))
def test_spmm_columns_match_brute_force(idx):
    # each column of Y = A X is the dense product of column c, integer-exact; the leading
    # dimensions are wider than k, and the padding columns of Y are left untouched
    import ctypes
    A = _cases()[idx]
    rng = np.random.default_rng(200 + idx)
    val = rng.integers(-8, 9, A.nnz).astype(float)
    k, ldx, ldy = 5, 7, 9
    X = np.ascontiguousarray(rng.integers(-8, 9, (A.N, ldx)).astype(float))
    Y = np.full((A.M, ldy), 12345.0)
    L = oracle.lib()
    ptr = np.ascontiguousarray(A.ptr, np.int32)
    col = np.ascontiguousarray(A.col, np.int32)
    vp = lambda a: ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)  # noqa: E731
    L.orc_csr_spmm(A.M, vp(ptr), vp(col), vp(val), k, vp(X), ldx, vp(Y), ldy)
    for c in range(k):
        want = brute(A.M, A.N, A.ptr.tolist(), A.col.tolist(), val.tolist(), X[:, c].tolist())
        assert np.array_equal(Y[:, c], want), c
        assert np.array_equal(Y[:, c], oracle.csr_spmv(A.M, A.ptr, A.col, val, np.ascontiguousarray(X[:, c])))
    assert np.all(Y[:, k:] == 12345.0)
    # the wrapper (ld = k) agrees
    Xk = np.ascontiguousarray(X[:, :k])
    assert np.array_equal(oracle.csr_spmm(A.M, A.ptr, A.col, val, Xk), Y[:, :k])


def test_spmm_table1_by_hand():
    # columns x = 1 and x = [1, 2, 3, 4] of Table I's matrix (row sums and the hand product)
    ptr, col, val = t1()
    X = np.array([[1.0, 1], [1, 2], [1, 3], [1, 4]])
    assert oracle.csr_spmm(4, ptr, col, val, X).tolist() == [[7, 15], [13, 38], [4, 12], [12, 29]]


@pytest.mark.parametrize("threads", [1, 2, 7])
def test_threaded_oracle_loop_bit_identical(threads):
    # the CPU-baseline loop: rows split over threads, each row still one sequential sum,
    # so the result is the serial loop's bit for bit (non-integer values: rounding matters)
    A = synth.zipf_rows(3000, 2500, seed=9, val_seed=10)
    x = synth.vector(A.N, 11)
    ptr, col = np.ascontiguousarray(A.ptr, np.int32), np.ascontiguousarray(A.col, np.int32)
    val = np.ascontiguousarray(A.val, np.float64)
    serial = oracle.csr_spmv(A.M, ptr, col, val, x)
    y, used = oracle.csr_spmv_omp(A.M, ptr, col, val, x, threads)
    assert used == threads
    assert np.array_equal(y.view(np.uint64), serial.view(np.uint64))


def _csr5_case(lens, w, s):
    lens = np.asarray(lens)
    ptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int32)
    col = np.concatenate([np.arange(n) for n in lens]).astype(np.int32)
    val = np.arange(1, ptr[-1] + 1, dtype=np.float64)
    return ptr, col, val, oracle.csr_to_csr5(len(lens), ptr, col, val, w, s)


def test_csr5_seg_off_hand_worked():
    # Sec. II-B / Table I readings, worked by hand.  Rows of lengths 5 and 3, omega = sigma = 2:
    # tile 0 holds entries 0-3 (lane 0: 0,1; lane 1: 2,3), tile 1 entries 4-7 (lane 0: 4,5;
    # lane 1: 6,7).  Flags: entry 0 (row 0 starts), tile 1's first slot (forced, mid-row 0)
    # and entry 5 (row 1 starts).  Lane 1 of each tile holds no flag, so lane 0 is followed by
    # one flag-free lane.
    ptr, col, val, c5 = _csr5_case([5, 3], 2, 2)
    assert c5["tile_ptr"].tolist() == [0, 0, 2]
    assert c5["bit_flag"].tolist() == [0b01, 0b00, 0b11, 0b00]
    assert c5["y_off"].tolist() == [0, 1, 0, 2]
    assert c5["seg_off"].tolist() == [1, 0, 1, 0]
    # omega = 4, sigma = 2, rows of lengths 4 and 12: tile 0 flags lanes 0 (row 0) and 2
    # (row 1 starts at entry 4); tile 1 (entries 8-15, all row 1) only its forced first slot
    ptr, col, val, c5 = _csr5_case([4, 12], 4, 2)
    assert c5["tile_ptr"].tolist() == [0, 1, 2]
    assert c5["bit_flag"].tolist() == [1, 0, 1, 0, 1, 0, 0, 0]
    assert c5["y_off"].tolist() == [0, 1, 1, 2, 0, 1, 1, 1]
    assert c5["seg_off"].tolist() == [1, 0, 1, 0, 3, 2, 1, 0]
    # Table I's own case is the all-zero one (every lane flagged)
    ptr, col, val = t1()
    assert oracle.csr_to_csr5(4, ptr, col, val, 2, 2)["seg_off"].tolist() == [0, 0, 0, 0]


def test_csr5_seg_off_counts_flag_free_runs():
    # on random layouts: seg_off[l] + 1 lanes from l reach the next flagged lane (or the tile's
    # end), checked lane by lane from the flags alone
    for seed in range(4):
        A = synth.zipf_rows(300, 300, seed=20 + seed, val_seed=1)
        for w, s in [(4, 2), (8, 3), (16, 4)]:
            c5 = oracle.csr_to_csr5(A.M, A.ptr, A.col, A.val, w, s)
            fl = c5["bit_flag"].reshape(-1, w)
            so = c5["seg_off"].reshape(-1, w)
            for t in range(fl.shape[0]):
                for l in range(w):
                    nxt = next((m for m in range(l + 1, w) if fl[t, m]), w)
                    assert so[t, l] == nxt - l - 1
