"""A whole single-problem call captured in a HIP graph and replayed.

amgs_qr_csr / amgs_qr_dense only enqueue kernels on the caller's stream (no
allocation, synchronisation or memset inside), so a captured call must
reproduce the eager call bit for bit on every replay: the reductions are
deterministic.  Between replays the outputs are overwritten with NaN and an
unrelated eager call runs on the same workspace, with synchronisations, so a
replay that depended on state left over from the capture or from an earlier
replay would be caught.
"""
import numpy as np
import pytest

from paper_1703_10440_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1703_10440_amd import amgs  # noqa: E402

DEV = torch.device("cuda:0")


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    return t if dtype is None else t.to(dtype)


def _colmajor(m, n, dtype):
    return torch.empty((n, m), dtype=dtype, device=DEV).t()


def _call(prob, A, Z, variant, panel, Q, R, P, work, precision="fp64", reorth=False):
    kw = dict(variant=variant, panel=panel, Q=Q, R=R, P=P, work=work, precision=precision,
              reorth=reorth)
    if prob.csr is not None:
        rp, ci, va = A
        return amgs.qr_csr(rp, ci, va, Z, **kw)
    return amgs.qr_dense(A, Z, **kw)


@pytest.mark.parametrize("panel", [0, 4, 8, 16])
@pytest.mark.parametrize("variant", ["naive", "ha", "hp"])
@pytest.mark.parametrize("kind", ["csr", "dense"])
def test_captured_call_replays_bitwise(kind, variant, panel):
    if panel == 16 and variant == "hp":
        pytest.skip("the three-level schedule has no HP form")
    _replay_check(kind, variant, panel, "fp64", False)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("variant", ["naive", "ha", "hp"])
@pytest.mark.parametrize("kind", ["csr", "dense"])
def test_captured_blocked_second_pass_replays_bitwise(kind, variant, precision):
    """The blocked second pass (two-level schedule) enqueues kernels only."""
    _replay_check(kind, variant, 8, precision, 2)


@pytest.mark.parametrize("form", ["fp32", "fp64_reorth", "fp32_reorth"])
@pytest.mark.parametrize("panel", [0, 4, 8, 16])
@pytest.mark.parametrize("variant", ["naive", "ha", "hp"])
@pytest.mark.parametrize("kind", ["csr", "dense"])
def test_captured_call_replays_bitwise_other_forms(kind, variant, panel, form):
    """The binary32 form and the second pass also enqueue kernels only."""
    if panel == 16 and variant == "hp":
        pytest.skip("the three-level schedule has no HP form")
    _replay_check(kind, variant, panel, form[:4], form.endswith("reorth"))


def _replay_check(kind, variant, panel, precision, reorth):
    dt = torch.float64 if precision == "fp64" else torch.float32
    if kind == "csr":
        prob = inputs.laplacian_graded_problem(N=12, n=13, decades=2.0, seed=7)
        A = (_dev(prob.csr.row_ptr), _dev(prob.csr.col_idx), _dev(prob.csr.vals, dt))
        other = inputs.random_csr_problem(3001, 11, 5, seed=12)
        A_other = (_dev(other.csr.row_ptr), _dev(other.csr.col_idx), _dev(other.csr.vals, dt))
    else:
        prob = inputs.random_dense_problem(333, 21, seed=10)
        A = _dev(prob.dense, dt)
        other = inputs.dense_gram_problem(512, 32, seed=1)
        A_other = _dev(other.dense, dt)
    print(f"[gpu] graph {kind} {prob.name} {variant} panel={panel} {precision} "
          f"reorth={reorth}", flush=True)
    m, n = prob.Z.shape
    Z = _dev(prob.Z, dt)
    Q = _colmajor(m, n, dt)
    P = _colmajor(m, n, dt)
    R = _colmajor(n, n, torch.float64)
    work = torch.empty(1 << 26, dtype=torch.uint8, device=DEV)
    call = lambda pr, a, z, q, r, p: _call(pr, a, z, variant, panel, q, r, p, work,  # noqa: E731
                                           precision, reorth)

    # eager reference
    eager = call(prob, A, Z, Q, R, P)
    torch.cuda.synchronize()
    assert int(eager.info.item()) == 0
    Qe, Re, Pe = Q.clone(), R.clone(), P.clone()

    # capture on a side stream after a warm-up there
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        call(prob, A, Z, Q, R, P)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        cap = call(prob, A, Z, Q, R, P)

    Zo = _dev(other.Z, dt)
    for rep in range(3):
        Q.fill_(float("nan"))
        R.fill_(float("nan"))
        P.fill_(float("nan"))
        # unrelated eager work on the same workspace between replays
        call(other, A_other, Zo, None, None, None)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(cap.info.item()) == 0
        assert torch.equal(Q, Qe), f"replay {rep}: Q differs"
        assert torch.equal(R, Re), f"replay {rep}: R differs"
        assert torch.equal(P, Pe), f"replay {rep}: P differs"
