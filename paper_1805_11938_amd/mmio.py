"""Matrix Market (coordinate) input, the file format of the paper's
evaluation set (Sec. III-D, Alg. 1: matrices are read from Matrix Market files
into COO, then converted).

Reads the `%%MatrixMarket matrix coordinate <field> <symmetry>` header with
field real, integer or pattern and symmetry general, symmetric,
skew-symmetric; array (dense) files are rejected.  Symmetric storage is
expanded (the mirror of an off-diagonal entry is added; skew-symmetric
negates it).  Returns 0-based triplets in file order, which the device
canonicalises (spmv_mat_from_coo: sort, duplicates summed in input order).
"""
from __future__ import annotations

import numpy as np

from .synth import HostCOO


def read(path: str) -> HostCOO:
    with open(path, "r") as f:
        header = f.readline().split()
        if len(header) < 5 or header[0].lower() != "%%matrixmarket" or header[1].lower() != "matrix":
            raise ValueError(f"{path}: not a Matrix Market matrix file")
        fmt, field, sym = header[2].lower(), header[3].lower(), header[4].lower()
        if fmt != "coordinate":
            raise ValueError(f"{path}: only coordinate files are supported (got {fmt})")
        if field not in ("real", "integer", "pattern"):
            raise ValueError(f"{path}: unsupported field {field}")
        if sym not in ("general", "symmetric", "skew-symmetric"):
            raise ValueError(f"{path}: unsupported symmetry {sym}")
        line = f.readline()
        while line.startswith("%") or not line.strip():
            line = f.readline()
            if not line:
                raise ValueError(f"{path}: missing size line")
        M, N, nz = (int(v) for v in line.split()[:3])
        cols = 2 if field == "pattern" else 3
        body = np.loadtxt(f, ndmin=2, max_rows=nz) if nz else np.zeros((0, cols))
    if body.shape != (nz, cols) and not (nz == 0):
        raise ValueError(f"{path}: expected {nz} entries of {cols} fields, got {body.shape}")
    row = body[:, 0].astype(np.int64) - 1
    col = body[:, 1].astype(np.int64) - 1
    val = np.ones(nz) if field == "pattern" else body[:, 2].astype(np.float64)
    if nz and (row.min() < 0 or col.min() < 0 or row.max() >= M or col.max() >= N):
        raise ValueError(f"{path}: index out of range")
    if sym != "general":
        off = row != col
        sign = -1.0 if sym == "skew-symmetric" else 1.0
        row, col, val = (np.concatenate([row, col[off]]), np.concatenate([col, row[off]]),
                         np.concatenate([val, sign * val[off]]))
    return HostCOO(M, N, row.astype(np.int32), col.astype(np.int32), val, name=path)


def write(path: str, M: int, N: int, row, col, val=None, comment: str = "") -> None:
    """Write 0-based triplets as a general coordinate file (real or pattern)."""
    row = np.asarray(row)
    col = np.asarray(col)
    field = "pattern" if val is None else "real"
    with open(path, "w") as f:
        f.write(f"%%MatrixMarket matrix coordinate {field} general\n")
        if comment:
            f.write(f"% {comment}\n")
        f.write(f"{M} {N} {len(row)}\n")
        for i in range(len(row)):
            if val is None:
                f.write(f"{row[i] + 1} {col[i] + 1}\n")
            else:
                f.write(f"{row[i] + 1} {col[i] + 1} {float(val[i])!r}\n")
