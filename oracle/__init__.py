"""CPU oracle for the SpMV format library -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports, links
or calls it.  Everything here is FP64 and plain: ``spmv_oracle.c`` (built
with -O2 -ffp-contract=off) for the formats, conversions and features, and
numpy for the MLP (``mlp.py``) and the feature transform.

Pins (what checks this oracle against something other than itself) live in
``tests/test_oracle_pins.py``: Table I's printed arrays, hand-derived
products, closed forms (Laplacian eigenvectors, stencil row sums), dense
brute force, integer-exact sums, finite differences for the MLP.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_L = None


def lib():
    global _L
    if _L is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        i64, vp, f64 = ctypes.c_int64, ctypes.c_void_p, ctypes.c_double
        sig = {
            "orc_coo_to_csr": (ctypes.c_int, [i64, i64, i64, vp, vp, vp, vp, vp, vp, vp]),
            "orc_csr_check": (ctypes.c_int, [i64, i64, i64, vp, vp]),
            "orc_csr_spmv": (None, [i64, vp, vp, vp, vp, vp]),
            "orc_csr_spmv_omp": (ctypes.c_int, [i64, vp, vp, vp, vp, vp, ctypes.c_int]),
            "orc_csr_absspmv": (None, [i64, vp, vp, vp, vp, vp]),
            "orc_csr_spmm": (None, [i64, vp, vp, vp, i64, vp, i64, vp, i64]),
            "orc_max_row_len": (i64, [i64, vp]),
            "orc_csr_to_ell": (None, [i64, vp, vp, vp, i64, vp, vp]),
            "orc_ell_spmv": (None, [i64, i64, vp, vp, vp, vp]),
            "orc_ell_to_csr": (i64, [i64, i64, vp, vp, vp, vp, vp]),
            "orc_sell_layout": (i64, [i64, i64, i64, vp, vp, vp, vp]),
            "orc_csr_to_sell": (None, [i64, i64, vp, vp, vp, vp, vp, vp, vp, vp]),
            "orc_sell_spmv": (None, [i64, i64, vp, vp, vp, vp, vp, vp, vp]),
            "orc_sell_to_csr": (i64, [i64, i64, vp, vp, vp, vp, vp, vp, vp, vp]),
            "orc_hyb_k_rule": (i64, [i64, vp]),
            "orc_hyb_coo_count": (i64, [i64, vp, i64]),
            "orc_csr_to_hyb": (None, [i64, vp, vp, vp, i64, vp, vp, vp, vp, vp]),
            "orc_hyb_spmv": (None, [i64, i64, vp, vp, i64, vp, vp, vp, vp, vp]),
            "orc_hyb_to_csr": (i64, [i64, i64, vp, vp, i64, vp, vp, vp, vp, vp, vp]),
            "orc_csr5_ntiles": (i64, [i64, i64, i64]),
            "orc_csr_to_csr5": (None, [i64, i64, vp, vp, vp, i64, i64, vp, vp, vp, vp, vp, vp]),
            "orc_csr5_spmv": (None, [i64, i64, vp, i64, i64, vp, vp, vp, vp, vp, vp, vp, vp]),
            "orc_csr5_to_csr": (None, [i64, i64, i64, vp, vp, vp, vp, vp, vp]),
            "orc_features": (None, [i64, i64, vp, vp, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _L = L
    return _L


def _p(a):
    if a is None:
        return ctypes.c_void_p(0)
    assert a.flags["C_CONTIGUOUS"], "oracle needs contiguous arrays"
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr_for(M):
    return np.zeros(M + 1, np.int32)


# ------------------------------------------------------------------ CSR

def coo_to_csr(M, N, row, col, val):
    """Stable (row, col) sort, duplicates summed in input order.  -> (ptr, col, val)."""
    row, col, val = _i32(row), _i32(col), _f64(val)
    n = len(row)
    ptr = _ptr_for(M)
    oc = np.empty(max(n, 1), np.int32)
    ov = np.empty(max(n, 1), np.float64)
    nn = ctypes.c_int64(0)
    rc = lib().orc_coo_to_csr(M, N, n, _p(row), _p(col), _p(val), _p(ptr), _p(oc), _p(ov), ctypes.byref(nn))
    if rc != 0:
        raise ValueError(f"coo_to_csr failed ({rc})")
    return ptr, oc[: nn.value].copy(), ov[: nn.value].copy()


def csr_check(M, N, ptr, col):
    ptr, col = _i32(ptr), _i32(col)
    return lib().orc_csr_check(M, N, int(ptr[-1]) if M >= 0 else 0, _p(ptr), _p(col))


def csr_spmv(M, ptr, col, val, x):
    y = np.empty(M, np.float64)
    lib().orc_csr_spmv(M, _p(_i32(ptr)), _p(_i32(col)), _p(_f64(val)), _p(_f64(x)), _p(y))
    return y


def csr_spmv_omp(M, ptr, col, val, x, nthreads):
    """Returns (y, threads_used)."""
    y = np.empty(M, np.float64)
    used = lib().orc_csr_spmv_omp(M, _p(ptr), _p(col), _p(val), _p(x), _p(y), int(nthreads))
    return y, used


def csr_absspmv(M, ptr, col, val, x):
    y = np.empty(M, np.float64)
    lib().orc_csr_absspmv(M, _p(_i32(ptr)), _p(_i32(col)), _p(_f64(val)), _p(_f64(x)), _p(y))
    return y


def csr_spmm(M, ptr, col, val, X):
    X = _f64(X)
    k = X.shape[1]
    Y = np.empty((M, k), np.float64)
    lib().orc_csr_spmm(M, _p(_i32(ptr)), _p(_i32(col)), _p(_f64(val)), k, _p(X), k, _p(Y), k)
    return Y


def rows_spmv(ptr, col, val, x, rows):
    """y_i for selected rows only (plain loop per row, for sampled checks at full size)."""
    out = np.empty(len(rows), np.float64)
    den = np.empty(len(rows), np.float64)
    for j, i in enumerate(rows):
        a, b = int(ptr[i]), int(ptr[i + 1])
        c = col[a:b]
        sub_p = np.array([0, b - a], np.int32)
        out[j] = csr_spmv(1, sub_p, c, val[a:b], x)[0]
        den[j] = csr_absspmv(1, sub_p, c, val[a:b], x)[0]
    return out, den


# ------------------------------------------------------------------ ELL

def max_row_len(M, ptr):
    return int(lib().orc_max_row_len(M, _p(_i32(ptr))))


def csr_to_ell(M, ptr, col, val, K=None):
    ptr, col, val = _i32(ptr), _i32(col), _f64(val)
    if K is None:
        K = max_row_len(M, ptr)
    ec = np.empty(M * K, np.int32)
    ev = np.empty(M * K, np.float64)
    lib().orc_csr_to_ell(M, _p(ptr), _p(col), _p(val), K, _p(ec), _p(ev))
    return K, ec, ev


def ell_spmv(M, K, ec, ev, x):
    y = np.empty(M, np.float64)
    lib().orc_ell_spmv(M, K, _p(_i32(ec)), _p(_f64(ev)), _p(_f64(x)), _p(y))
    return y


def ell_to_csr(M, K, ec, ev):
    ptr = _ptr_for(M)
    c = np.empty(max(M * K, 1), np.int32)
    v = np.empty(max(M * K, 1), np.float64)
    n = lib().orc_ell_to_csr(M, K, _p(_i32(ec)), _p(_f64(ev)), _p(ptr), _p(c), _p(v))
    return ptr, c[:n].copy(), v[:n].copy()


# ----------------------------------------------------------------- SELL

def sell_layout(M, C, sigma, ptr):
    nch = (M + C - 1) // C
    perm = np.empty(nch * C, np.int32)
    widths = np.empty(max(nch, 1), np.int32)[:nch]
    cs = np.empty(nch + 1, np.int64)
    lib().orc_sell_layout(M, C, sigma, _p(_i32(ptr)), _p(perm), _p(widths) if nch else ctypes.c_void_p(0), _p(cs))
    return perm, widths, cs


def csr_to_sell(M, ptr, col, val, C, sigma):
    ptr, col, val = _i32(ptr), _i32(col), _f64(val)
    perm, widths, cs = sell_layout(M, C, sigma, ptr)
    n = int(cs[-1])
    sc = np.empty(n, np.int32)
    sv = np.empty(n, np.float64)
    lib().orc_csr_to_sell(M, C, _p(ptr), _p(col), _p(val), _p(perm), _p(widths), _p(cs), _p(sc), _p(sv))
    return dict(perm=perm, widths=widths, cs=cs, col=sc, val=sv)


def sell_spmv(M, C, s, x):
    y = np.empty(M, np.float64)
    lib().orc_sell_spmv(M, C, _p(s["perm"]), _p(s["widths"]), _p(s["cs"]), _p(s["col"]), _p(_f64(s["val"])),
                        _p(_f64(x)), _p(y))
    return y


def sell_to_csr(M, C, s):
    ptr = _ptr_for(M)
    n = len(s["col"])
    c = np.empty(max(n, 1), np.int32)
    v = np.empty(max(n, 1), np.float64)
    nn = lib().orc_sell_to_csr(M, C, _p(s["perm"]), _p(s["widths"]), _p(s["cs"]), _p(s["col"]), _p(_f64(s["val"])),
                               _p(ptr), _p(c), _p(v))
    return ptr, c[:nn].copy(), v[:nn].copy()


# ------------------------------------------------------------------ HYB

def hyb_k_rule(M, ptr):
    return int(lib().orc_hyb_k_rule(M, _p(_i32(ptr))))


def csr_to_hyb(M, ptr, col, val, K=None):
    ptr, col, val = _i32(ptr), _i32(col), _f64(val)
    if K is None:
        K = hyb_k_rule(M, ptr)
    n = int(lib().orc_hyb_coo_count(M, _p(ptr), K))
    ec = np.empty(M * K, np.int32)
    ev = np.empty(M * K, np.float64)
    cr = np.empty(n, np.int32)
    cc = np.empty(n, np.int32)
    cv = np.empty(n, np.float64)
    lib().orc_csr_to_hyb(M, _p(ptr), _p(col), _p(val), K, _p(ec), _p(ev), _p(cr), _p(cc), _p(cv))
    return dict(K=K, ell_col=ec, ell_val=ev, coo_row=cr, coo_col=cc, coo_val=cv)


def hyb_spmv(M, h, x):
    y = np.empty(M, np.float64)
    lib().orc_hyb_spmv(M, h["K"], _p(h["ell_col"]), _p(_f64(h["ell_val"])), len(h["coo_row"]), _p(h["coo_row"]),
                       _p(h["coo_col"]), _p(_f64(h["coo_val"])), _p(_f64(x)), _p(y))
    return y


def hyb_to_csr(M, h):
    ptr = _ptr_for(M)
    n = M * h["K"] + len(h["coo_row"])
    c = np.empty(max(n, 1), np.int32)
    v = np.empty(max(n, 1), np.float64)
    nn = lib().orc_hyb_to_csr(M, h["K"], _p(h["ell_col"]), _p(_f64(h["ell_val"])), len(h["coo_row"]),
                              _p(h["coo_row"]), _p(h["coo_col"]), _p(_f64(h["coo_val"])), _p(ptr), _p(c), _p(v))
    return ptr, c[:nn].copy(), v[:nn].copy()


# ----------------------------------------------------------------- CSR5

def csr_to_csr5(M, ptr, col, val, omega, sigma):
    ptr, col, val = _i32(ptr), _i32(col), _f64(val)
    nnz = int(ptr[-1])
    T = nnz // (omega * sigma)
    tp = np.empty(T + 1, np.int32)
    fl = np.empty(T * omega, np.uint32)
    yo = np.empty(T * omega, np.int32)
    so = np.empty(T * omega, np.int32)
    tc = np.empty(T * omega * sigma, np.int32)
    tv = np.empty(T * omega * sigma, np.float64)
    lib().orc_csr_to_csr5(M, nnz, _p(ptr), _p(col), _p(val), omega, sigma, _p(tp), _p(fl), _p(yo), _p(so),
                          _p(tc), _p(tv))
    t0 = T * omega * sigma
    return dict(omega=omega, sigma=sigma, ntiles=T, tile_ptr=tp, bit_flag=fl, y_off=yo, seg_off=so,
                col=tc, val=tv, tail_col=col[t0:].copy(), tail_val=val[t0:].copy())


def csr5_spmv(M, ptr, c5, x):
    ptr = _i32(ptr)
    nnz = int(ptr[-1])
    y = np.empty(M, np.float64)
    lib().orc_csr5_spmv(M, nnz, _p(ptr), c5["omega"], c5["sigma"], _p(c5["tile_ptr"]), _p(c5["bit_flag"]),
                        _p(c5["col"]), _p(_f64(c5["val"])), _p(c5["tail_col"]), _p(_f64(c5["tail_val"])),
                        _p(_f64(x)), _p(y))
    return y


def csr5_to_csr(nnz, c5):
    c = np.empty(max(nnz, 1), np.int32)
    v = np.empty(max(nnz, 1), np.float64)
    lib().orc_csr5_to_csr(nnz, c5["omega"], c5["sigma"], _p(c5["col"]), _p(_f64(c5["val"])), _p(c5["tail_col"]),
                          _p(_f64(c5["tail_val"])), _p(c), _p(v))
    return c[:nnz].copy(), v[:nnz].copy()


# ------------------------------------------------------------- features

FEATURE_NAMES = ("n_rows", "n_cols", "nnz", "nnz_frac", "nnz_min", "nnz_max", "nnz_avg", "nnz_std",
                 "variation", "ell_pad", "bandwidth", "gini")


def features(M, N, ptr, col):
    f = np.empty(12, np.float64)
    lib().orc_features(M, N, _p(_i32(ptr)), _p(_i32(col)), _p(f))
    return f


from .mlp import (feature_transform, mlp_forward, mlp_loss_and_grads, adam_step,  # noqa: E402
                  minmax_fit, minmax_apply)
