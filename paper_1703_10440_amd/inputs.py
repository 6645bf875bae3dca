"""Seeded synthetic inputs for A-orthonormalising thin QR (Z = QR, Q^T A Q = I).

This module only *builds inputs*: spd matrices A (CSR or dense, column-major)
and tall matrices Z.  It contains none of the orthogonalisation arithmetic and
is the one module shared by the CPU oracle's tests and the GPU path.

Random numbers come from numpy's ``Generator(MT19937(seed))``; the paper drew
its test matrices with a Mersenne twister as well (Section 4, experiments I
and II).  Every array is returned as numpy (host) data; callers copy the same
bits to the device.

Workloads (sizes follow the paper's Section 4 shapes where it gives them):

* ``dense_gram``      A = B B^T / m + I, B m x m Gaussian, symmetrised exactly
                      (random dense spd A of experiment I-a), Z Gaussian.
* ``laplacian_graded`` 7-point 3-D Laplacian on an N^3 grid (Dirichlet,
                      unscaled stencil 6/-1) plus shift*I in CSR, with
                      Z = G diag(logspace(0, -d, n)) W, W Haar orthogonal.
* ``pentadiag_batch`` many independent instances: A spd pentadiagonal
                      (off-diagonals U[-1,0], diagonal 4.5 + U[0,1]),
                      m ~ U[64, 4096], n ~ U[4, 64], Z Gaussian.
* ``exp2_problem``    the accuracy test matrices of experiment II:
                      A = V D V^T with log-spaced eigenvalues, Z = U E W^T.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


def rng(seed: int) -> np.random.Generator:
    """Mersenne-twister generator for a given seed."""
    return np.random.Generator(np.random.MT19937(seed))


# --------------------------------------------------------------------------
# Containers
# --------------------------------------------------------------------------
@dataclass
class CSR:
    """Symmetric sparse matrix in CSR form, column indices ascending per row."""
    m: int
    row_ptr: np.ndarray  # int32, m+1
    col_idx: np.ndarray  # int32, nnz
    vals: np.ndarray     # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.m, self.m), dtype=np.float64, order="F")
        rows = np.repeat(np.arange(self.m), np.diff(self.row_ptr))
        d[rows, self.col_idx] = self.vals
        return d

    def astype(self, dtype) -> "CSR":
        return CSR(self.m, self.row_ptr, self.col_idx, self.vals.astype(dtype))


@dataclass
class Problem:
    """One A-orthonormalisation problem: spd A (``csr`` or ``dense``) and Z."""
    name: str
    Z: np.ndarray                        # m x n, float64, Fortran order
    csr: Optional[CSR] = None
    dense: Optional[np.ndarray] = None   # m x m, float64, Fortran order, symmetric
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.Z.shape[0]

    @property
    def n(self) -> int:
        return self.Z.shape[1]


@dataclass
class Batch:
    """Independent instances; instance k has its own CSR A_k and Z_k."""
    name: str
    problems: List[Problem]
    meta: dict = field(default_factory=dict)


# --------------------------------------------------------------------------
# Matrix builders
# --------------------------------------------------------------------------
def laplacian7(N: int, shift: float) -> CSR:
    """7-point Laplacian on an N x N x N grid, Dirichlet boundary, plus shift*I.

    Rows are numbered k = x + N*y + N*N*z; the stencil is 6 on the diagonal and
    -1 for each of the (up to) six grid neighbours, so the diagonal entry is
    6 + shift and nnz = 7 N^3 - 6 N^2.  Columns are stored ascending.
    """
    m = N * N * N
    k = np.arange(m, dtype=np.int64)
    x = k % N
    y = (k // N) % N
    z = k // (N * N)
    # candidate neighbours in ascending column order
    offs = [(-N * N, z > 0), (-N, y > 0), (-1, x > 0), (0, np.ones(m, bool)),
            (1, x < N - 1), (N, y < N - 1), (N * N, z < N - 1)]
    valid = np.stack([v for _, v in offs], axis=1)          # m x 7
    cols = np.stack([k + o for o, _ in offs], axis=1)       # m x 7
    vals = np.where(np.arange(7)[None, :] == 3, 6.0 + shift, -1.0)
    vals = np.broadcast_to(vals, (m, 7))
    counts = valid.sum(axis=1)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = cols[valid].astype(np.int32)
    v = vals[valid].astype(np.float64)
    assert row_ptr[-1] == 7 * N ** 3 - 6 * N ** 2
    return CSR(m, row_ptr.astype(np.int32), col_idx, np.ascontiguousarray(v))


def laplacian7_kappa(N: int, shift: float) -> float:
    """Closed-form 2-norm condition number of ``laplacian7(N, shift)``."""
    c = np.cos(np.pi / (N + 1))
    return (6.0 * (1.0 + c) + shift) / (6.0 * (1.0 - c) + shift)


def haar_orthogonal(g: np.random.Generator, n: int) -> np.ndarray:
    """Haar-distributed orthogonal n x n matrix: QR of a Gaussian, sign-fixed."""
    G = g.standard_normal((n, n))
    Qh, Rh = np.linalg.qr(G)
    return Qh * np.sign(np.diag(Rh))[None, :]


def graded_columns(g: np.random.Generator, m: int, n: int, decades: float) -> np.ndarray:
    """Z = G diag(logspace(0, -decades, n)) W: kappa(Z) ~ 10**decades."""
    G = g.standard_normal((m, n))
    s = np.logspace(0.0, -decades, n)
    W = haar_orthogonal(g, n)
    return np.asfortranarray((G * s[None, :]) @ W)


def gram_spd(g: np.random.Generator, m: int, device: Optional[str] = None) -> np.ndarray:
    """A = B B^T / m + I with B m x m standard normal, symmetrised exactly.

    The product may be formed on a torch device (input preparation only); the
    upper triangle is then mirrored so that A is bitwise symmetric.
    """
    B = g.standard_normal((m, m))
    if device is None or device == "cpu":
        A = B @ B.T
    else:
        import torch
        Bt = torch.from_numpy(B).to(device)
        A = (Bt @ Bt.T).cpu().numpy()
        del Bt
    del B
    A /= m
    A[np.diag_indices(m)] += 1.0
    iu = np.triu_indices(m, 1)
    A.T[iu] = A[iu]          # lower := upper  (A.T[i,j] is A[j,i])
    return np.asfortranarray(A)


def pentadiag_spd(g: np.random.Generator, m: int) -> CSR:
    """Symmetric pentadiagonal spd matrix: off-diagonals U[-1,0], diagonal 4.5+U[0,1].

    The diagonal exceeds the sum of |off-diagonals| in each row (at most 4),
    so A is strictly diagonally dominant with positive diagonal, hence spd.
    """
    d = 4.5 + g.random(m)
    o1 = -g.random(m - 1)
    o2 = -g.random(m - 2)
    rows, cols, vals = [], [], []
    for off, band in ((-2, o2), (-1, o1), (0, d), (1, o1), (2, o2)):
        lo = max(0, -off)
        idx = np.arange(lo, lo + band.size)
        rows.append(idx)
        cols.append(idx + off)
        vals.append(band)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    v = np.concatenate(vals)
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.add.at(row_ptr, r + 1, 1)
    np.cumsum(row_ptr, out=row_ptr)
    assert row_ptr[-1] == 5 * m - 6
    return CSR(m, row_ptr.astype(np.int32), c.astype(np.int32), v.astype(np.float64))


def csr_from_dense(A: np.ndarray, drop_zeros: bool = True) -> CSR:
    m = A.shape[0]
    mask = A != 0 if drop_zeros else np.ones_like(A, bool)
    rows, cols = np.nonzero(mask)          # row-major order: rows asc, cols asc
    counts = np.bincount(rows, minlength=m)
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSR(m, row_ptr.astype(np.int32), cols.astype(np.int32),
               np.ascontiguousarray(A[rows, cols], dtype=np.float64))


# --------------------------------------------------------------------------
# The workloads
# --------------------------------------------------------------------------
def dense_gram_problem(m: int = 512, n: int = 32, seed: int = 1,
                       device: Optional[str] = None) -> Problem:
    """Dense spd A = B B^T/m + I and Gaussian Z (draw order: B, then Z)."""
    g = rng(seed)
    A = gram_spd(g, m, device)
    Z = np.asfortranarray(g.standard_normal((m, n)))
    return Problem(f"dense_gram_m{m}_n{n}", Z, dense=A,
                   meta={"seed": seed, "kind": "dense"})


def laplacian_graded_problem(N: int = 64, n: int = 64, decades: float = 6.0,
                             shift: float = 1e-2, seed: int = 2) -> Problem:
    """CSR 7-point Laplacian N^3 + shift*I with graded Z (kappa(Z) ~ 10**decades)."""
    g = rng(seed)
    A = laplacian7(N, shift)
    Z = graded_columns(g, A.m, n, decades)
    return Problem(f"laplacian{N}^3_n{n}_kz1e{decades:g}", Z, csr=A,
                   meta={"seed": seed, "kind": "csr", "N": N,
                         "kappa_A": laplacian7_kappa(N, shift),
                         "decades": decades})


def random_csr_problem(m: int, n: int, nnz_per_row: int, seed: int,
                       decades: float = 0.0) -> Problem:
    """Random symmetric, strictly diagonally dominant CSR (spd) with a given
    average row length, for ragged/irregular SpMV shapes."""
    g = rng(seed)
    half = max(0, (nnz_per_row - 1) // 2)
    r = np.repeat(np.arange(m), half)
    c = g.integers(0, m, size=r.size)
    keep = r != c
    r, c = r[keep], c[keep]
    v = -g.random(r.size)
    rr = np.concatenate([r, c])
    cc = np.concatenate([c, r])
    vv = np.concatenate([v, v])
    # merge duplicates
    key = rr.astype(np.int64) * m + cc
    uk, inv = np.unique(key, return_inverse=True)
    uv = np.zeros(uk.size)
    np.add.at(uv, inv, vv)
    rr = (uk // m).astype(np.int64)
    cc = (uk % m).astype(np.int64)
    rowsum = np.zeros(m)
    np.add.at(rowsum, rr, np.abs(uv))
    diag = rowsum + 1.0 + g.random(m)
    rr = np.concatenate([rr, np.arange(m)])
    cc = np.concatenate([cc, np.arange(m)])
    uv = np.concatenate([uv, diag])
    order = np.lexsort((cc, rr))
    rr, cc, uv = rr[order], cc[order], uv[order]
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.add.at(row_ptr, rr + 1, 1)
    np.cumsum(row_ptr, out=row_ptr)
    A = CSR(m, row_ptr.astype(np.int32), cc.astype(np.int32), uv.astype(np.float64))
    if decades > 0:
        Z = graded_columns(g, m, n, decades)
    else:
        Z = np.asfortranarray(g.standard_normal((m, n)))
    return Problem(f"randcsr_m{m}_n{n}_r{nnz_per_row}", Z, csr=A,
                   meta={"seed": seed, "kind": "csr"})


def random_dense_problem(m: int, n: int, seed: int, decades: float = 0.0) -> Problem:
    """Small dense spd A = B B^T/m + I with Gaussian (or graded) Z."""
    g = rng(seed)
    A = gram_spd(g, m)
    if decades > 0:
        Z = graded_columns(g, m, n, decades)
    else:
        Z = np.asfortranarray(g.standard_normal((m, n)))
    return Problem(f"randdense_m{m}_n{n}", Z, dense=A, meta={"seed": seed, "kind": "dense"})


def pentadiag_batch(batch: int = 2048, m_lo: int = 64, m_hi: int = 4096,
                    n_lo: int = 4, n_hi: int = 64, seed: int = 5) -> Batch:
    """Independent pentadiagonal instances.  The master seed draws all m, then
    all n (inclusive bounds); instance k then uses seed 1_000_000 + k, drawing
    its diagonal, first and second off-diagonals, then Z."""
    g = rng(seed)
    ms = g.integers(m_lo, m_hi, size=batch, endpoint=True)
    ns = g.integers(n_lo, n_hi, size=batch, endpoint=True)
    probs = []
    for k in range(batch):
        gk = rng(1_000_000 + k)
        m, n = int(ms[k]), int(ns[k])
        A = pentadiag_spd(gk, m)
        Z = np.asfortranarray(gk.standard_normal((m, n)))
        probs.append(Problem(f"penta{k}", Z, csr=A, meta={"seed": 1_000_000 + k}))
    return Batch(f"pentadiag_batch{batch}", probs,
                 meta={"seed": seed, "m_range": (m_lo, m_hi), "n_range": (n_lo, n_hi)})


def exp2_problem(m: int, n: int, kappa_A: float, kappa_Z: float, case: int,
                 seed: int) -> Problem:
    """Accuracy test problem of experiment II.

    A = V D V^T with d_i = 10**(alpha (i-1)), alpha = log10(kappa_A)/(m-1);
    Z = U E W^T with e_i = 10**(beta (i-1)), beta = log10(kappa_Z)/(n-1) and U
    the eigenvectors of the n largest (case 1) or n smallest (case 2)
    eigenvalues.  V and W are Haar orthogonal.
    """
    g = rng(seed)
    V = haar_orthogonal(g, m)
    W = haar_orthogonal(g, n)
    alpha = np.log10(kappa_A) / (m - 1)
    d = 10.0 ** (alpha * np.arange(m))
    A = (V * d[None, :]) @ V.T
    A = 0.5 * (A + A.T)
    beta = np.log10(kappa_Z) / (n - 1)
    e = 10.0 ** (beta * np.arange(n))
    U = V[:, m - n:][:, ::-1] if case == 1 else V[:, :n]
    Z = np.asfortranarray((U * e[None, :]) @ W.T)
    return Problem(f"exp2_case{case}", Z, dense=np.asfortranarray(A),
                   meta={"seed": seed, "kappa_A": kappa_A, "kappa_Z": kappa_Z,
                         "case": case})


# Named workloads ----------------------------------------------------------
WORKLOADS = {
    # dense spd 512 x 512, Z 512 x 32
    "dense512_n32": lambda: dense_gram_problem(512, 32, seed=1),
    # 7-point Laplacian 64^3 + 1e-2 I, Z 262144 x 64, kappa(Z) ~ 1e6
    "lap64_n64": lambda: laplacian_graded_problem(64, 64, 6.0, 1e-2, seed=2),
    # 7-point Laplacian 128^3 + 1e-2 I, Z 2097152 x 128, kappa(Z) ~ 1e4
    "lap128_n128": lambda: laplacian_graded_problem(128, 128, 4.0, 1e-2, seed=3),
}


def dense16k_problem(device: Optional[str] = None) -> Problem:
    """Dense spd 16384 x 16384 (B B^T/m + I), Z 16384 x 256 Gaussian."""
    return dense_gram_problem(16384, 256, seed=4, device=device)
