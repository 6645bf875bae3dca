"""The CPU oracle against facts fixed by the paper and by mathematics."""
import pytest

import pins
from conftest import read_golden


@pytest.fixture(scope="module")
def lib(oracle):
    return oracle.load()


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(lib, pin):
    if pin is pins.pin_hand_example:
        fails = pin(lib, read_golden("hand_example.txt"))
    else:
        fails = pin(lib)
    assert not fails, "\n".join(fails[:20])


def test_high_precision_cholesky(oracle):
    """R against the Cholesky factor of Z^T A Z evaluated with 60 significant
    digits (mpmath), on a tiny problem: the oracle must agree to a few units
    in the last place of binary64."""
    mpmath = pytest.importorskip("mpmath")
    import numpy as np
    from paper_1703_10440_amd import inputs
    mpmath.mp.dps = 60
    p = inputs.random_dense_problem(8, 4, 5)
    Zm = mpmath.matrix(p.Z.tolist())
    Am = mpmath.matrix(p.dense.tolist())
    G = Zm.T * Am * Zm
    L = mpmath.cholesky(G)
    Rexact = np.array([[float(L[j, i]) for j in range(4)] for i in range(4)])
    for v in ("naive", "ha", "hp"):
        for o in ("col", "row"):
            r = oracle.qr_problem(p, variant=v, orientation=o)
            err = np.abs(np.triu(r.R) - Rexact).max() / np.abs(Rexact).max()
            assert err < 1e-14, (v, o, err)


def test_mv_matches_scipy(oracle):
    import numpy as np
    import scipy.sparse as sp
    from paper_1703_10440_amd import inputs
    A = inputs.laplacian7(7, 0.01)
    v = inputs.rng(3).standard_normal(A.m)
    S = sp.csr_matrix((A.vals, A.col_idx, A.row_ptr), shape=(A.m, A.m))
    assert np.allclose(oracle.mv_csr(A, v), S @ v, rtol=1e-14, atol=1e-14)
