"""Seeded input generators: structure and closed-form facts."""
import numpy as np

from paper_1703_10440_amd import inputs


def test_laplacian_structure_and_kappa():
    for N in (4, 6):
        A = inputs.laplacian7(N, 0.01)
        assert A.nnz == 7 * N ** 3 - 6 * N ** 2
        D = A.to_dense()
        assert np.array_equal(D, D.T)
        assert np.all(np.diff(A.col_idx[A.row_ptr[0]:A.row_ptr[1]]) > 0)
        w = np.linalg.eigvalsh(D)
        assert abs(w[-1] / w[0] - inputs.laplacian7_kappa(N, 0.01)) < 1e-9 * w[-1] / w[0]
    # the two large grids: closed-form values
    assert abs(inputs.laplacian7_kappa(64, 0.01) - 705.78) < 0.01
    assert abs(inputs.laplacian7_kappa(128, 0.01) - 1019.44) < 0.01


def test_graded_columns_condition():
    g = inputs.rng(5)
    Z = inputs.graded_columns(g, 4000, 16, 6.0)
    s = np.linalg.svd(Z, compute_uv=False)
    assert 1e5 < s[0] / s[-1] < 1e7


def test_gram_spd_symmetric_and_seeded():
    a = inputs.dense_gram_problem(64, 8, seed=1)
    b = inputs.dense_gram_problem(64, 8, seed=1)
    assert np.array_equal(a.dense, b.dense) and np.array_equal(a.Z, b.Z)
    assert np.array_equal(a.dense, a.dense.T)
    assert np.linalg.eigvalsh(a.dense)[0] > 1.0 - 1e-12


def test_pentadiag_batch():
    b = inputs.pentadiag_batch(batch=16, seed=5)
    for p in b.problems:
        assert 64 <= p.m <= 4096 and 4 <= p.n <= 64
        assert p.csr.nnz == 5 * p.m - 6
        D = p.csr.to_dense()
        assert np.array_equal(D, D.T)
        off = np.abs(D).sum(axis=1) - np.abs(np.diag(D))
        assert np.all(np.diag(D) > off)          # strictly diagonally dominant


def test_exp2_problem_conditioning():
    p = inputs.exp2_problem(100, 20, 1e6, 1e3, 2, 1)
    w = np.linalg.eigvalsh(p.dense)
    assert abs(np.log10(w[-1] / w[0]) - 6) < 1e-6
    s = np.linalg.svd(p.Z, compute_uv=False)
    assert abs(np.log10(s[0] / s[-1]) - 3) < 1e-6
