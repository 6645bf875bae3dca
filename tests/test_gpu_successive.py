"""Successive orthogonalisation (opts.first): the columns before `first` are
final in Q, P and R; the rest are A-orthonormalised against them and each
other.  The GPU result must equal the GPU's own one-call result on all
columns bit for bit (same kernels, same per-column arithmetic, same order of
projections), and match the oracle's successive run (pinned to the one-call
oracle run bit for bit, tests/pins.py, pin_successive) within the usual
tolerance.
"""
import numpy as np
import pytest

from oracle import ref
from paper_1703_10440_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1703_10440_amd import amgs  # noqa: E402

DEV = torch.device("cuda:0")
VARIANTS = ("naive", "ha", "hp")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _call(prob, variant, cgs, reorth, precision, Zt, **kw):
    print(f"[gpu] successive {prob.name} m={prob.m} n={prob.n} {variant} cgs={cgs} "
          f"reorth={reorth} {precision} first={kw.get('first', 0)}", flush=True)
    args = dict(variant=variant, precision=precision, reorth=reorth, cgs=cgs, **kw)
    if prob.csr is not None:
        out = amgs.qr_csr(torch.from_numpy(prob.csr.row_ptr).to(DEV),
                          torch.from_numpy(prob.csr.col_idx).to(DEV),
                          torch.from_numpy(prob.csr.vals).to(DEV), Zt, **args)
    else:
        out = amgs.qr_dense(torch.from_numpy(np.ascontiguousarray(prob.dense)).to(DEV), Zt,
                            **args)
    torch.cuda.synchronize()
    return out


PROBS = [
    inputs.laplacian_graded_problem(N=12, n=21, decades=2.0, seed=17),   # CSR, m = 1728
    inputs.random_dense_problem(333, 19, seed=18),                      # dense, ragged
]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("reorth", [False, True])
@pytest.mark.parametrize("cgs", [False, True])
@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("pi", range(len(PROBS)), ids=[p.name for p in PROBS])
def test_successive_equals_one_call(pi, variant, cgs, reorth, precision):
    p = PROBS[pi]
    Zt = torch.from_numpy(np.ascontiguousarray(p.Z)).to(DEV)
    full = _call(p, variant, cgs, reorth, precision, Zt, return_p=True)
    assert int(full.info.item()) == 0
    for k in (3, 9):   # 9 > 8: the blocked HP recurrence crosses the split
        part = _call(p, variant, cgs, reorth, precision, Zt[:, :k].contiguous(), return_p=True)
        assert int(part.info.item()) == 0
        m, n = p.Z.shape
        dt = full.Q.dtype
        Q = amgs.empty_colmajor(m, n, dt, DEV)
        P = amgs.empty_colmajor(m, n, dt, DEV)
        R = amgs.empty_colmajor(n, n, torch.float64, DEV)
        Q[:, :k] = part.Q
        P[:, :k] = part.P
        R.zero_()
        R[:k, :k] = part.R
        succ = _call(p, variant, cgs, reorth, precision, Zt, Q=Q, P=P, R=R, first=k)
        assert int(succ.info.item()) == 0
        assert torch.equal(succ.Q[:, k:], full.Q[:, k:]), k
        assert torch.equal(succ.R, full.R), k
        assert torch.equal(P[:, k:], full.P[:, k:]), k
        if precision == "fp64":
            o = ref.qr(p.Z, dense=p.dense, csr=p.csr, variant=variant,
                       orientation="cgs" if cgs else "col", reorth=reorth, first=k,
                       Q0=part.Q.double().cpu().numpy(), P0=part.P.double().cpu().numpy(),
                       R0=part.R.cpu().numpy())
            e = _rel(succ.R.cpu().numpy(), o.R)
            print(f"  first={k}: R vs oracle {e:.2e}")
            assert e <= 1e-10


def test_successive_edges_and_errors():
    p = PROBS[0]
    Zt = torch.from_numpy(np.ascontiguousarray(p.Z)).to(DEV)
    full = _call(p, "ha", False, False, "fp64", Zt, return_p=True)
    m, n = p.Z.shape
    # first = n: nothing to do, nothing written
    Q, P, R = full.Q.clone(), full.P.clone(), full.R.clone()
    out = _call(p, "ha", False, False, "fp64", Zt, Q=Q, P=P, R=R, first=n)
    assert torch.equal(Q, full.Q) and torch.equal(R, full.R) and torch.equal(P, full.P)
    assert int(out.info.item()) == 0
    # first > 0 needs P; first > n; panel schedule
    for kw, want in ((dict(first=2), "invalid argument"), (dict(first=n + 1, P=P), "invalid argument"),
                     (dict(first=2, P=P, panel=4), "unsupported")):
        with pytest.raises(RuntimeError, match=want):
            _call(p, "ha", False, False, "fp64", Zt, Q=full.Q.clone(), **kw)
