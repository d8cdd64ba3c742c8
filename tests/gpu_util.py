"""Helpers shared by the GPU parity tests: oracle references and the
row-wise error criterion.  (Tests only; the library never imports this.)"""
import numpy as np

import oracle

TOL = {0: 1e-12, 1: 1e-5}  # FP64, FP32: max row-wise relative error


def as_dtype(A, dt):
    """Values as the device will hold them (FP32 rounds once)."""
    return A.val.astype(np.float32).astype(np.float64) if dt == 1 else A.val


def reference(A, x64, dt):
    """Oracle y and row-wise denominators sum_j |a_ij x_j| for the values as stored."""
    val = as_dtype(A, dt)
    y = oracle.csr_spmv(A.M, A.ptr, A.col, val, x64)
    den = oracle.csr_absspmv(A.M, A.ptr, A.col, val, x64)
    return y, den


def rowwise_err(y, yref, den):
    y = np.asarray(y, np.float64)
    e = np.abs(y - yref)
    z = den == 0
    if np.any(z) and np.any(e[z] != 0):
        return np.inf
    nz = ~z
    return float(np.max(e[nz] / den[nz])) if np.any(nz) else 0.0


def device_vec(x64, dt):
    import torch
    return torch.from_numpy(x64.astype(np.float32) if dt == 1 else x64.copy()).cuda()


FORMAT_CONFIGS = [
    ("csr", {}),
    ("csr", {"csr_lanes_per_row": 1}),
    ("csr", {"csr_lanes_per_row": 4}),
    ("csr", {"csr_lanes_per_row": 64}),
    ("csr", {"flags": 2}),
    ("csr", {"flags": 4}),
    ("csr", {"flags": 16}),
    ("csr", {"flags": 32}),
    ("csr", {"bands": 3}),
    ("csr", {"bands": 4, "flags": 32}),
    ("csr", {"bands": 2, "csr_lanes_per_row": 4}),
    ("csr5", {}),
    ("csr5", {"csr5_sigma": 4}),
    ("csr5", {"csr5_sigma": 32}),
    ("csr5", {"csr5_omega": 16, "csr5_sigma": 3}),
    ("csr5", {"bands": 3}),
    ("csr5", {"csr5_sigma": 4, "bands": 8}),
    ("csr5", {"csr5_sigma": 32, "bands": 2}),
    ("csr5", {"csr5_sigma": 8, "bands": 2}),
    ("csr5", {"csr5_sigma": 5, "bands": 2}),
    ("ell", {}),
    ("ell", {"flags": 4}),
    ("ell", {"flags": 64}),
    ("ell", {"flags": 64 | 4}),
    ("sell", {}),
    ("sell", {"flags": 8}),
    ("sell", {"sell_C": 64, "sell_sigma": 1}),
    ("sell", {"sell_C": 8, "sell_sigma": 64}),
    ("sell", {"sell_C": 64, "sell_sigma": 16384}),
    ("sell", {"sell_C": 64, "sell_sigma": 1, "flags": 64}),
    ("sell", {"sell_C": 64, "sell_sigma": 1 << 30, "flags": 64}),
    ("sell", {"sell_C": 64, "sell_sigma": 1, "flags": 128}),
    ("sell", {"sell_C": 64, "sell_sigma": 1 << 30, "flags": 128 | 64}),
    ("sell", {"sell_C": 64, "sell_sigma": 1, "flags": 128, "bands": 2}),
    ("sell", {"sell_C": 64, "sell_sigma": 1 << 30, "bands": 3}),
    ("sell", {"sell_C": 8, "sell_sigma": 1, "bands": 8}),
    ("sell", {"sell_C": 32, "sell_sigma": 64, "bands": 2, "flags": 8}),
    ("hyb", {}),
    ("hyb", {"hyb_K": 0}),
    ("hyb", {"hyb_K": 2}),
    ("hyb", {"hyb_K": 2, "flags": 64}),
    ("hyb", {"bands": 3}),
    ("hyb", {"hyb_K": 1, "bands": 2}),
    ("hyb", {"hyb_K": 0, "bands": 4}),
]
