"""Seeded synthetic inputs shared by the GPU library's tests/benchmarks and the oracle.

Holds no SpMV arithmetic: it only draws structure and values (see ``synth.c``).
Every generator is a pure function of its parameters and seed.

Workloads (the paper's SuiteSparse set, Sec. III-C, is not available; these
stand in for its regular and irregular, scientific-to-social-network
structure with nnz in 1e5..2e7):

* ``laplace2d(64)``        2-D 5-point Dirichlet Laplacian, 4,096 rows, 20,224 nnz
* ``stencil27(100)``       3-D 27-point stencil, 1e6 rows, 26,463,592 nnz
* ``zipf_rows(...)``       1e6 x 1e6, Zipf(2) row lengths (mean 16, max 1e4), uniform columns
* ``selector_specs()``     3,000 mixed matrices (banded, block-diagonal, uniform, Zipf, R-MAT)
* ``batch_specs()``        512 uneven matrices for the batched launch
* ``rmat_coo(24, 2**28)``  scale-free R-MAT edge list (duplicates kept)
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "libsynth.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(path)
        i64, u64, f64, vp = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p
        sig = {
            "syn_u64": (u64, [u64, u64, u64]),
            "syn_normal": (None, [i64, u64, u64, vp]),
            "syn_uniform": (None, [i64, f64, f64, u64, u64, vp]),
            "syn_laplace2d_nnz": (i64, [i64]),
            "syn_laplace2d": (None, [i64, vp, vp, vp]),
            "syn_stencil27_nnz": (i64, [i64]),
            "syn_stencil27": (None, [i64, vp, vp]),
            "syn_zipf_mean": (f64, [f64, f64, i64]),
            "syn_lens_zipf": (None, [i64, i64, f64, f64, i64, u64, vp]),
            "syn_lens_poisson": (None, [i64, i64, f64, u64, vp]),
            "syn_lens_uniform_int": (None, [i64, i64, i64, i64, u64, vp]),
            "syn_fill_random_cols": (None, [i64, i64, vp, u64, vp]),
            "syn_banded": (None, [i64, i64, i64, f64, u64, vp, vp, vp]),
            "syn_blockdiag": (None, [i64, i64, i64, f64, u64, vp, vp, vp]),
            "syn_rmat": (None, [i64, i64, f64, f64, f64, u64, vp, vp]),
            "syn_lens_to_ptr": (i64, [i64, vp, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def _p(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data) if a is not None and a.size else ctypes.c_void_p(0)


@dataclass
class HostCSR:
    """A CSR matrix in host memory: int32 ptr[M+1], int32 col[nnz], float64 val[nnz]."""

    M: int
    N: int
    ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.ptr[-1]) if self.M > 0 else 0

    def lengths(self) -> np.ndarray:
        return np.diff(self.ptr.astype(np.int64))


@dataclass
class HostCOO:
    """Raw triplets (unsorted, duplicates allowed): int32 row/col, float64 val."""

    M: int
    N: int
    row: np.ndarray
    col: np.ndarray
    val: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)


# ----------------------------------------------------------------- values

def normal(n: int, seed: int, stream: int = 0) -> np.ndarray:
    out = np.empty(int(n), dtype=np.float64)
    if n:
        _lib().syn_normal(int(n), int(seed), int(stream), _p(out))
    return out


def uniform(n: int, seed: int, lo: float = -1.0, hi: float = 1.0, stream: int = 0) -> np.ndarray:
    out = np.empty(int(n), dtype=np.float64)
    if n:
        _lib().syn_uniform(int(n), float(lo), float(hi), int(seed), int(stream), _p(out))
    return out


def vector(n: int, seed: int) -> np.ndarray:
    """x ~ U[-1, 1] from `seed`."""
    return uniform(n, seed, -1.0, 1.0)


# ----------------------------------------------------------- generators

def laplace2d(n: int = 64) -> HostCSR:
    L = _lib()
    nnz = L.syn_laplace2d_nnz(n)
    ptr = np.empty(n * n + 1, np.int32)
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    L.syn_laplace2d(n, _p(ptr), _p(col), _p(val))
    return HostCSR(n * n, n * n, ptr, col, val, name=f"laplace2d_{n}")


def stencil27(n: int = 100, seed: int = 2) -> HostCSR:
    L = _lib()
    nnz = L.syn_stencil27_nnz(n)
    ptr = np.empty(n ** 3 + 1, np.int32)
    col = np.empty(nnz, np.int32)
    L.syn_stencil27(n, _p(ptr), _p(col))
    return HostCSR(n ** 3, n ** 3, ptr, col, normal(nnz, seed), name=f"stencil27_{n}")


def zipf_scale(alpha: float, mean: float, lmax: int) -> float:
    """Scale s so that L = min(lmax, max(1, round(s*Z))) has the requested mean."""
    L = _lib()
    lo, hi = 1e-6, float(lmax)
    if L.syn_zipf_mean(alpha, hi, lmax) < mean:
        return hi
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if L.syn_zipf_mean(alpha, mid, lmax) < mean:
            lo = mid
        else:
            hi = mid
    return hi


def _from_lens(M: int, N: int, lens: np.ndarray) -> tuple[np.ndarray, int]:
    ptr = np.empty(M + 1, np.int32)
    nnz = _lib().syn_lens_to_ptr(M, _p(lens), _p(ptr))
    if nnz < 0:
        raise ValueError("generated matrix exceeds int32 nnz")
    return ptr, nnz


def _random_cols(M: int, N: int, lens: np.ndarray, seed: int) -> tuple[np.ndarray, np.ndarray]:
    ptr, nnz = _from_lens(M, N, lens)
    col = np.empty(nnz, np.int32)
    _lib().syn_fill_random_cols(M, N, _p(ptr), int(seed), _p(col))
    return ptr, col


def zipf_rows(M: int, N: int, alpha: float = 2.0, mean: float = 16.0, lmax: int = 10_000,
              seed: int = 4, val_seed: int = 5) -> HostCSR:
    s = zipf_scale(alpha, mean, lmax)
    lens = np.empty(M, np.int32)
    _lib().syn_lens_zipf(M, N, alpha, s, lmax, int(seed), _p(lens))
    ptr, col = _random_cols(M, N, lens, seed)
    return HostCSR(M, N, ptr, col, normal(len(col), val_seed), name=f"zipf_{M}",
                   meta=dict(alpha=alpha, mean=mean, lmax=lmax, scale=s))


def uniform_random(M: int, N: int, mean: float, seed: int, val_seed: int) -> HostCSR:
    lens = np.empty(M, np.int32)
    _lib().syn_lens_poisson(M, N, float(mean), int(seed), _p(lens))
    ptr, col = _random_cols(M, N, lens, seed)
    return HostCSR(M, N, ptr, col, normal(len(col), val_seed), name=f"uniform_{M}", meta=dict(mean=mean))


def from_lengths(M: int, N: int, lens, seed: int, val_seed: int) -> HostCSR:
    """Rows of the given lengths (each <= N) with distinct uniformly random
    columns, sorted, and standard-normal values."""
    lens = np.ascontiguousarray(lens, np.int32)
    assert lens.shape == (M,) and (lens >= 0).all() and (lens <= N).all()
    ptr, col = _random_cols(M, N, lens, seed)
    return HostCSR(M, N, ptr, col, normal(len(col), val_seed), name=f"lengths_{M}")


def uniform_len_random(M: int, N: int, lo: int, hi: int, seed: int, val_seed: int) -> HostCSR:
    lens = np.empty(M, np.int32)
    _lib().syn_lens_uniform_int(M, N, int(lo), int(hi), int(seed), _p(lens))
    ptr, col = _random_cols(M, N, lens, seed)
    return HostCSR(M, N, ptr, col, normal(len(col), val_seed), name=f"uniformlen_{M}")


def _pattern(fn, M: int, N: int, a: int, b: float, seed: int, val_seed: int, name: str) -> HostCSR:
    L = _lib()
    lens = np.empty(M, np.int32)
    fn(M, N, int(a), float(b), int(seed), _p(lens), ctypes.c_void_p(0), ctypes.c_void_p(0))
    ptr, nnz = _from_lens(M, N, lens)
    col = np.empty(nnz, np.int32)
    fn(M, N, int(a), float(b), int(seed), ctypes.c_void_p(0), _p(ptr), _p(col))
    return HostCSR(M, N, ptr, col, normal(nnz, val_seed), name=name)


def banded(M: int, halfwidth: int, fill: float, seed: int, val_seed: int) -> HostCSR:
    return _pattern(_lib().syn_banded, M, M, halfwidth, fill, seed, val_seed, f"banded_{M}")


def blockdiag(M: int, block: int, density: float, seed: int, val_seed: int) -> HostCSR:
    return _pattern(_lib().syn_blockdiag, M, M, block, density, seed, val_seed, f"blockdiag_{M}")


def rmat_coo(scale: int, nedges: int, seed: int, val_seed: int, a: float = 0.57, b: float = 0.19,
             c: float = 0.19) -> HostCOO:
    M = 1 << scale
    row = np.empty(nedges, np.int32)
    col = np.empty(nedges, np.int32)
    _lib().syn_rmat(scale, nedges, a, b, c, int(seed), _p(row), _p(col))
    return HostCOO(M, M, row, col, normal(nedges, val_seed), name=f"rmat_s{scale}",
                   meta=dict(scale=scale, nedges=nedges))


def from_dense(A: np.ndarray) -> HostCSR:
    """CSR of a small dense array (test helper; row-major scan keeps columns sorted)."""
    A = np.asarray(A, dtype=np.float64)
    M, N = A.shape
    rows, cols = np.nonzero(A)
    ptr = np.zeros(M + 1, np.int32)
    np.add.at(ptr, rows + 1, 1)
    ptr = np.cumsum(ptr).astype(np.int32)
    return HostCSR(M, N, ptr, cols.astype(np.int32), A[rows, cols].copy())


def random_pattern(M: int, N: int, density: float, seed: int, integer_values: bool = False) -> HostCSR:
    """Small random CSR for brute-force tests (numpy PCG64; duplicates impossible)."""
    rng = np.random.default_rng(seed)
    mask = rng.random((M, N)) < density
    A = np.where(mask, rng.integers(-8, 9, size=(M, N)) if integer_values else rng.standard_normal((M, N)), 0.0)
    csr = from_dense(A)
    # keep explicit entries where the mask is set but the value drew zero
    rows, cols = np.nonzero(mask)
    ptr = np.zeros(M + 1, np.int64)
    np.add.at(ptr, rows + 1, 1)
    csr.ptr = np.cumsum(ptr).astype(np.int32)
    csr.col = cols.astype(np.int32)
    csr.val = A[rows, cols].astype(np.float64)
    return csr


# ----------------------------------------------------- workload recipes

def _loguniform(rng, lo, hi):
    return float(math.exp(rng.uniform(math.log(lo), math.log(hi))))


GENERATORS = ("banded", "blockdiag", "uniform", "zipf", "rmat")


def selector_spec(i: int, seed0: int = 100, kinds=GENERATORS, nnz_lo=1e5, nnz_hi=2e7,
                  rows_lo=1e4, rows_hi=2e6) -> dict:
    """Parameters of matrix i of the selector training set.  Generator kinds
    rotate, so each kind gets an equal share.  Parameters are resampled until
    the expected nnz lies in [nnz_lo, nnz_hi]."""
    if i >= N_BASE:
        return selector_spec_large(i, seed0)
    kind = kinds[i % len(kinds)]
    rng = np.random.default_rng(seed0 + i)
    for _ in range(1000):
        M = int(_loguniform(rng, rows_lo, rows_hi))
        if kind == "banded":
            hw = int(round(_loguniform(rng, 1, 256)))
            fill = float(rng.uniform(0.05, 1.0))
            exp_nnz = M * (1 + 2 * hw * fill)
            p = dict(halfwidth=hw, fill=fill)
        elif kind == "blockdiag":
            bs = int(round(_loguniform(rng, 4, 512)))
            dens = float(rng.uniform(0.1, 1.0))
            exp_nnz = M * (1 + (bs - 1) * dens)
            p = dict(block=bs, density=dens)
        elif kind == "uniform":
            mean = float(rng.uniform(2, 64))
            exp_nnz = M * mean
            p = dict(mean=mean)
        elif kind == "zipf":
            alpha = float(rng.uniform(1.5, 3.0))
            mean = float(rng.uniform(4, 64))
            lmax = int(round(_loguniform(rng, 256, 1e4)))
            lmax = min(lmax, M)
            if lmax < 2 * mean:
                continue
            exp_nnz = M * mean
            p = dict(alpha=alpha, mean=mean, lmax=lmax)
        else:  # rmat
            scale = int(round(math.log2(M)))
            M = 1 << scale
            ef = float(rng.uniform(4, 32))
            exp_nnz = M * ef * 0.9
            p = dict(scale=scale, edge_factor=ef)
        if nnz_lo <= exp_nnz <= nnz_hi:
            return dict(index=i, kind=kind, M=M, seed=seed0 + i, params=p)
    raise RuntimeError(f"could not sample spec {i}")


LARGE_KINDS = ("stencil27", "banded", "uniform", "zipf", "rmat")
N_BASE = 3000  # matrices 0..2999: the base set; from 3000 on: the large set


def selector_spec_large(i: int, seed0: int = 100) -> dict:
    """Matrix i >= N_BASE of the selector training set: the large shapes
    (2x10^7..3x10^8 nonzeros, 10^6..1.7x10^7 rows) of the benchmark matrices --
    3-D 27-point stencils on n^3 grids besides banded, uniform, Zipf and R-MAT."""
    j = i - N_BASE
    kind = LARGE_KINDS[j % len(LARGE_KINDS)]
    rng = np.random.default_rng(seed0 + i)
    for _ in range(1000):
        if kind == "stencil27":
            n = int(rng.integers(100, 221))
            return dict(index=i, kind=kind, M=n ** 3, seed=seed0 + i, params=dict(n=n))
        M = int(_loguniform(rng, 1e6, 1.7e7))
        if kind == "banded":
            hw = int(round(_loguniform(rng, 4, 64)))
            fill = float(rng.uniform(0.2, 1.0))
            exp_nnz = M * (1 + 2 * hw * fill)
            p = dict(halfwidth=hw, fill=fill)
        elif kind == "uniform":
            mean = float(rng.uniform(4, 32))
            exp_nnz = M * mean
            p = dict(mean=mean)
        elif kind == "zipf":
            alpha = float(rng.uniform(1.5, 3.0))
            mean = float(rng.uniform(8, 32))
            lmax = int(round(_loguniform(rng, 1e3, 1e4)))
            exp_nnz = M * mean
            p = dict(alpha=alpha, mean=mean, lmax=lmax)
        else:  # rmat
            scale = int(rng.integers(20, 25))
            M = 1 << scale
            ef = float(rng.uniform(4, 16))
            exp_nnz = M * ef * 0.9
            p = dict(scale=scale, edge_factor=ef)
        if 2e7 <= exp_nnz <= 3e8:
            return dict(index=i, kind=kind, M=M, seed=seed0 + i, params=p)
    raise RuntimeError(f"could not sample spec {i}")


def selector_specs(n: int = 3000, seed0: int = 100, **kw) -> list[dict]:
    return [selector_spec(i, seed0, **kw) for i in range(n)]


def make(spec: dict):
    """Build the matrix a spec describes: HostCSR, or HostCOO for R-MAT."""
    k, M, s, p = spec["kind"], spec["M"], spec["seed"], spec["params"]
    vs = s * 7919 + 1
    if k == "banded":
        return banded(M, p["halfwidth"], p["fill"], s, vs)
    if k == "blockdiag":
        return blockdiag(M, p["block"], p["density"], s, vs)
    if k == "uniform":
        return uniform_random(M, M, p["mean"], s, vs)
    if k == "uniformlen":
        return uniform_len_random(M, M, p["lo"], p["hi"], s, vs)
    if k == "zipf":
        return zipf_rows(M, M, p["alpha"], p["mean"], p["lmax"], s, vs)
    if k == "rmat":
        return rmat_coo(p["scale"], int(round(p["edge_factor"] * M)), s, vs)
    if k == "stencil27":
        return stencil27(p["n"], vs)
    raise ValueError(k)


def batch_specs(n: int = 512, seed: int = 8, rows_lo: float = 1e3, rows_hi: float = 2e5) -> list[dict]:
    """Uneven batch: rows log-uniform in [rows_lo, rows_hi]; per-row nnz mean
    uniform in {4..64}; generators round-robin over banded, block-diagonal,
    uniform and Zipf."""
    rng = np.random.default_rng(seed)
    kinds = ("banded", "blockdiag", "uniform", "zipf")
    out = []
    for i in range(n):
        M = int(_loguniform(rng, rows_lo, rows_hi))
        mean = int(rng.integers(4, 65))
        k = kinds[i % 4]
        if k == "banded":
            hw = max(1, int(round(mean / 2)))
            p = dict(halfwidth=hw, fill=min(1.0, (mean - 1) / (2 * hw)))
        elif k == "blockdiag":
            bs = max(4, mean * 2)
            p = dict(block=bs, density=min(1.0, (mean - 1) / (bs - 1)))
        elif k == "uniform":
            p = dict(mean=float(mean))
        else:
            p = dict(alpha=2.0, mean=float(mean), lmax=int(min(M, 64 * mean)))
        out.append(dict(index=i, kind=k, M=M, seed=seed * 100003 + i, params=p))
    return out


def mlp_init(seed: int, sizes=(12, 64, 64, 5)) -> list[np.ndarray]:
    """He-uniform weights U(-sqrt(6/fan_in), +sqrt(6/fan_in)), zero biases.
    Returns [W1, b1, W2, b2, W3, b3] with W_l of shape (fan_in, fan_out)."""
    out = []
    for l in range(len(sizes) - 1):
        fi, fo = sizes[l], sizes[l + 1]
        a = math.sqrt(6.0 / fi)
        W = uniform(fi * fo, seed, -a, a, stream=100 + l).reshape(fi, fo)
        out += [W, np.zeros(fo)]
    return out
