"""Generator determinism and statistics (host only)."""
import numpy as np

from paper_1805_11938_amd import synth
import oracle


def test_seed_determinism_byte_identical():
    a = synth.zipf_rows(5000, 5000, seed=4, val_seed=5)
    b = synth.zipf_rows(5000, 5000, seed=4, val_seed=5)
    assert a.ptr.tobytes() == b.ptr.tobytes() and a.col.tobytes() == b.col.tobytes()
    assert a.val.tobytes() == b.val.tobytes()
    c = synth.zipf_rows(5000, 5000, seed=5, val_seed=5)
    assert c.col.tobytes() != a.col.tobytes()


def test_generated_csr_is_canonical():
    for A in [synth.laplace2d(16), synth.stencil27(7), synth.zipf_rows(3000, 2000, seed=1, val_seed=2),
              synth.uniform_random(4000, 4000, 5.0, 3, 4), synth.banded(3000, 9, 0.3, 5, 6),
              synth.blockdiag(3000, 40, 0.4, 7, 8)]:
        assert oracle.csr_check(A.M, A.N, A.ptr, A.col) == 0, A.name


def test_zipf_statistics():
    A = synth.zipf_rows(1_000_000, 1_000_000, seed=4, val_seed=5)
    L = A.lengths()
    assert L.min() == 3 and L.max() == 10_000
    assert abs(L.mean() - 16.0) < 0.5
    assert 60 <= (L == 10_000).sum() <= 160  # about 107 expected


def test_rmat_quadrant_frequencies():
    C = synth.rmat_coo(10, 200_000, seed=10, val_seed=11)
    top_r = C.row >> 9
    top_c = C.col >> 9
    freq = [np.mean((top_r == r) & (top_c == c)) for r, c in [(0, 0), (0, 1), (1, 0), (1, 1)]]
    assert np.allclose(freq, [0.57, 0.19, 0.19, 0.05], atol=0.005)


def test_normals_and_uniforms():
    z = synth.normal(200_000, 1)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1) < 0.01
    u = synth.vector(200_000, 3)
    assert u.min() >= -1 and u.max() < 1 and abs(u.mean()) < 0.01


def test_selector_specs_cover_generators_and_ranges():
    specs = synth.selector_specs(40)
    kinds = [s["kind"] for s in specs]
    assert all(kinds.count(k) == 8 for k in synth.GENERATORS)
    assert all(1e4 / 2 <= s["M"] <= 2e6 * 1.5 for s in specs)
    assert specs == synth.selector_specs(40)


def test_batch_specs():
    specs = synth.batch_specs(16)
    assert len(specs) == 16 and all(1e3 <= s["M"] <= 2e5 for s in specs)


def test_large_selector_specs_span_the_benchmark_shapes():
    """Matrices 3000.. of the selector set: 3-D stencils, banded, uniform,
    Zipf and R-MAT with 2x10^7..3x10^8 expected nonzeros and up to 1.7x10^7
    rows, so the benchmark matrices (the 100^3 stencil: 10^6 rows, 2.6x10^7
    nonzeros; R-MAT scale 24) lie inside the training range."""
    specs = [synth.selector_spec(i) for i in range(synth.N_BASE, synth.N_BASE + 40)]
    assert [s["kind"] for s in specs[:5]] == list(synth.LARGE_KINDS)
    assert all(s["kind"] in synth.LARGE_KINDS for s in specs)
    for s in specs:
        p = s["params"]
        if s["kind"] == "stencil27":
            assert 100 <= p["n"] <= 220 and s["M"] == p["n"] ** 3
            nnz = 27 * p["n"] ** 3
        elif s["kind"] == "rmat":
            assert 20 <= p["scale"] <= 24 and s["M"] == 1 << p["scale"]
            nnz = s["M"] * p["edge_factor"] * 0.9
        elif s["kind"] == "banded":
            nnz = s["M"] * (1 + 2 * p["halfwidth"] * p["fill"])
        else:
            nnz = s["M"] * p["mean"]
        assert 1e6 <= s["M"] <= 1.7e7 and nnz <= 3.3e8, s
        if s["kind"] != "stencil27":
            assert nnz >= 2e7, s
    assert specs == [synth.selector_spec(i) for i in range(synth.N_BASE, synth.N_BASE + 40)]
    # the base set is unchanged by the extension
    assert synth.selector_spec(5) == synth.selector_specs(6)[5]
    small = synth.make(dict(index=0, kind="stencil27", M=8, seed=3, params=dict(n=2)))
    assert small.M == 8 and small.nnz == 64  # every pair of the 2x2x2 grid is a neighbour
