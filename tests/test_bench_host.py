"""Host-side behaviour of bench.py that needs no GPU: the one-GPU contract
and the byte model behind the batched line's roofline."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1703_10440_amd import inputs  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_batch_size_classes():
    # 4 ranges of m (<= 512, <= 1024, <= 2048, larger) times n <= 16 or not
    assert bench.batch_size_class(64, 4) == 0
    assert bench.batch_size_class(512, 16) == 0
    assert bench.batch_size_class(512, 17) == 1
    assert bench.batch_size_class(513, 4) == 2
    assert bench.batch_size_class(2048, 64) == 5
    assert bench.batch_size_class(4096, 64) == 7


def test_batch_requested_bytes_counts_each_pass():
    """One instance, counted by hand: m = 100, n = 8, tridiagonal A."""
    m, n = 100, 8
    D = np.diag(np.full(m, 4.0)) + np.diag(np.full(m - 1, -1.0), 1) + np.diag(np.full(m - 1, -1.0), -1)
    p = inputs.Problem("tri", np.asfortranarray(np.ones((m, n))), csr=inputs.csr_from_dense(D))
    nnz = 3 * m - 2
    w = 8
    col = m * w
    A = 4 * (m + 1) + nnz * (4 + w)
    R = 8 * n * n + 8 * n * (n + 1) / 2
    for B, earlier in ((1, sum(range(8))), (4, 0 + 4), (8, 0)):
        tiles = [B] * 8
        ha = R + n * col + 2 * n * col + 2 * earlier * col + n * A
        assert bench.batch_requested_bytes([p], tiles, "ha", w) == ha
        naive = ha + n * A
        assert bench.batch_requested_bytes([p], tiles, "naive", w) == naive
        hp = ha - n * A + n * (A + 2 * col) + n * col
        assert bench.batch_requested_bytes([p], tiles, "hp", w) == hp
    # wider blocks read the earlier columns fewer times
    assert (bench.batch_requested_bytes([p], [8] * 8, "ha", w)
            < bench.batch_requested_bytes([p], [1] * 8, "ha", w))


def test_batch_model_bytes_by_hand():
    """The method's byte model and compulsory floor for one instance, counted
    by hand: m = 100, n = 8, tridiagonal A, binary64 and binary32."""
    m, n = 100, 8
    D = np.diag(np.full(m, 4.0)) + np.diag(np.full(m - 1, -1.0), 1) + np.diag(np.full(m - 1, -1.0), -1)
    p = inputs.Problem("tri", np.asfortranarray(np.ones((m, n))), csr=inputs.csr_from_dense(D))
    nnz = 3 * m - 2
    for w in (8, 4):
        A = 4 * (m + 1) + nnz * (4 + w)
        io = 2 * m * n * w + 8 * n * n
        proj = m * n * (n - 1) * w
        S1 = A + 2 * m * w
        want = {"naive": 2 * n * S1 + proj + io, "ha": n * S1 + proj + io,
                "hp": A + 2 * m * n * w + proj + io}
        for v, b in want.items():
            alg, floor = bench.batch_model_bytes([p], v, w)
            assert alg == b, (v, w)
            assert floor == A + io
