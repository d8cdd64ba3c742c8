"""Matrix Market coordinate input: tiny files written here by hand."""
import numpy as np
import pytest

import oracle
from paper_1805_11938_amd import mmio


def _w(tmp_path, name, text):
    p = tmp_path / name
    p.write_text(text)
    return str(p)


def test_general_real_with_comments(tmp_path):
    p = _w(tmp_path, "a.mtx", "%%MatrixMarket matrix coordinate real general\n% a comment\n%\n3 4 4\n"
                              "1 1 2.5\n3 4 -1\n2 2 1e-3\n1 1 0.5\n")
    A = mmio.read(p)
    assert (A.M, A.N) == (3, 4)
    assert A.row.tolist() == [0, 2, 1, 0] and A.col.tolist() == [0, 3, 1, 0]
    assert A.val.tolist() == [2.5, -1.0, 1e-3, 0.5]
    # canonical CSR: duplicate (0,0) summed in input order
    ptr, col, val = oracle.coo_to_csr(A.M, A.N, A.row, A.col, A.val)
    assert ptr.tolist() == [0, 1, 2, 3] and col.tolist() == [0, 1, 3] and val.tolist() == [3.0, 1e-3, -1.0]


def test_pattern_symmetric_and_skew(tmp_path):
    p = _w(tmp_path, "p.mtx", "%%MatrixMarket matrix coordinate pattern symmetric\n3 3 3\n1 1\n2 1\n3 2\n")
    A = mmio.read(p)
    got = sorted(zip(A.row.tolist(), A.col.tolist(), A.val.tolist()))
    assert got == [(0, 0, 1.0), (0, 1, 1.0), (1, 0, 1.0), (1, 2, 1.0), (2, 1, 1.0)]
    q = _w(tmp_path, "k.mtx", "%%MatrixMarket matrix coordinate integer skew-symmetric\n2 2 1\n2 1 7\n")
    B = mmio.read(q)
    assert sorted(zip(B.row.tolist(), B.col.tolist(), B.val.tolist())) == [(0, 1, -7.0), (1, 0, 7.0)]


def test_round_trip_and_errors(tmp_path):
    rng = np.random.default_rng(4)
    r, c = rng.integers(0, 50, 200), rng.integers(0, 40, 200)
    v = rng.standard_normal(200)
    p = str(tmp_path / "r.mtx")
    mmio.write(p, 50, 40, r, c, v)
    A = mmio.read(p)
    assert A.row.tolist() == r.tolist() and A.col.tolist() == c.tolist()
    assert np.array_equal(A.val, v)  # repr() round-trips doubles exactly
    with pytest.raises(ValueError):
        mmio.read(_w(tmp_path, "d.mtx", "%%MatrixMarket matrix array real general\n2 2\n1\n2\n3\n4\n"))
    with pytest.raises(ValueError):
        mmio.read(_w(tmp_path, "o.mtx", "%%MatrixMarket matrix coordinate real general\n2 2 1\n3 1 1.0\n"))
    with pytest.raises(ValueError):
        mmio.read(_w(tmp_path, "n.mtx", "not a matrix\n"))
