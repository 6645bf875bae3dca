"""ctypes front-end of the CPU oracle (``oracle/amgs_ref.c``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg.  Nothing in the GPU library imports this file.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "amgs_ref.c")
_LIB_PATH = os.path.join(_HERE, "libamgs_ref.so")

VARIANTS = {"naive": 0, "ha": 1, "hp": 2}
ORIENT = {"col": 0, "row": 1, "panel": 2, "cgs": 3, "panel8": 4, "panel16": 5}
PRECISION = {"fp64": 0, "fp32": 1}

CFLAGS = ["-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-std=c11", "-Wall"]


def build(src: str = _SRC, out: str = _LIB_PATH, extra=()) -> str:
    """Compile the oracle with gcc (plain C, OpenMP)."""
    cmd = ["gcc", *CFLAGS, *extra, src, "-o", out, "-lm"]
    subprocess.run(cmd, check=True)
    return out


_lib = None


def load(path: Optional[str] = None):
    global _lib
    if path is None and _lib is not None:
        return _lib
    p = path or _LIB_PATH
    if path is None and (not os.path.exists(p) or os.path.getmtime(p) < os.path.getmtime(_SRC)):
        build(out=p)   # missing, or older than its source
    lib = C.CDLL(p)
    i64, dp, ip = C.c_int64, C.POINTER(C.c_double), C.POINTER(C.c_int32)
    lib.amgs_ref_qr_dense.argtypes = [i64, dp, i64, i64, dp, i64, dp, i64, dp, i64, dp, i64,
                                      C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(i64), i64]
    lib.amgs_ref_qr_dense.restype = C.c_int
    lib.amgs_ref_qr_csr.argtypes = [i64, i64, ip, ip, dp, i64, dp, i64, dp, i64, dp, i64, dp,
                                    i64, C.c_int, C.c_int, C.c_int, C.c_int, C.POINTER(i64), i64]
    lib.amgs_ref_qr_csr.restype = C.c_int
    lib.amgs_ref_mv_csr.argtypes = [i64, ip, ip, dp, dp, dp, C.c_int]
    lib.amgs_ref_num_threads.restype = C.c_int
    if path is None:
        _lib = lib
    return lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


class Result:
    def __init__(self, Q, R, P, info, mv_calls, mv_cols):
        self.Q, self.R, self.P, self.info = Q, R, P, info
        self.mv_calls, self.mv_cols = mv_calls, mv_cols


def qr(Z: np.ndarray, dense: Optional[np.ndarray] = None, csr=None, variant: str = "ha",
       orientation: str = "col", reorth=False, precision: str = "fp64",
       lib=None, first: int = 0, Q0=None, P0=None, R0=None) -> Result:
    """Run the oracle.  ``dense`` is an m x m symmetric matrix; ``csr`` is an
    object with ``m, row_ptr, col_idx, vals``.  Returns Q, R, P = AQ, info.
    first > 0: Q0, P0, R0 hold the final leading columns (successive
    orthogonalisation).  reorth: False / True (the second pass per column) or
    2 (the blocked second pass of the "panel8" orientation)."""
    lib = lib or load()
    Z = np.asfortranarray(Z, dtype=np.float64)
    m, n = Z.shape
    Q = np.zeros((m, n), dtype=np.float64, order="F")
    R = np.zeros((n, n), dtype=np.float64, order="F")
    P = np.zeros((m, n), dtype=np.float64, order="F")
    if first:
        Q[:, :first] = Q0[:, :first]
        P[:, :first] = P0[:, :first]
        R[:first, :first] = R0[:first, :first]
    stats = (C.c_int64 * 2)()
    ld = max(m, 1)
    args = (n, _d(Z), ld, _d(Q), ld, _d(R), max(n, 1), _d(P), ld, VARIANTS[variant],
            ORIENT[orientation], int(reorth), PRECISION[precision], stats, int(first))
    if dense is not None:
        A = np.asfortranarray(dense, dtype=np.float64)
        info = lib.amgs_ref_qr_dense(m, _d(A), max(m, 1), *args)
    else:
        rp = np.ascontiguousarray(csr.row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(csr.col_idx, dtype=np.int32)
        va = np.ascontiguousarray(csr.vals, dtype=np.float64)
        info = lib.amgs_ref_qr_csr(m, int(rp[-1]), _i(rp), _i(ci), _d(va), *args)
    if info < 0:
        raise ValueError("oracle rejected its arguments")
    return Result(Q, R, P, int(info), int(stats[0]), int(stats[1]))


def qr_problem(prob, **kw) -> Result:
    return qr(prob.Z, dense=prob.dense, csr=prob.csr, **kw)


def mv_csr(csr, v: np.ndarray, precision: str = "fp64") -> np.ndarray:
    lib = load()
    rp = np.ascontiguousarray(csr.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(csr.col_idx, dtype=np.int32)
    va = np.ascontiguousarray(csr.vals, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    y = np.zeros(csr.m)
    lib.amgs_ref_mv_csr(csr.m, _i(rp), _i(ci), _d(va), _d(v), _d(y), PRECISION[precision])
    return y


def num_threads() -> int:
    return int(load().amgs_ref_num_threads())


# ----------------------------------------------------------- error metrics
def orth_loss(Q: np.ndarray, dense: Optional[np.ndarray] = None, csr=None) -> float:
    """||Q^T A Q - I||_2 evaluated in binary64."""
    AQ = dense @ Q if dense is not None else _csr_matmat(csr, Q)
    G = Q.T @ AQ
    return float(np.linalg.norm(G - np.eye(Q.shape[1]), 2))


def residual(Z: np.ndarray, Q: np.ndarray, R: np.ndarray) -> float:
    """||Z - QR||_F / ||Z||_F."""
    return float(np.linalg.norm(Z - Q @ np.triu(R)) / np.linalg.norm(Z))


def _csr_matmat(csr, V: np.ndarray) -> np.ndarray:
    import scipy.sparse as sp
    S = sp.csr_matrix((csr.vals, csr.col_idx, csr.row_ptr), shape=(csr.m, csr.m))
    return np.asarray(S @ V)
