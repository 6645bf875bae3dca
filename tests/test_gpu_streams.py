"""Calls enqueued on a side stream give the same bits as calls on torch's
current stream: the binding makes the side stream wait for the current one
(the inputs are complete), prepares outputs and workspace on the side
stream, and keeps the caller's tensors alive for it.  Two passes of one
batched plan launched on different streams are ordered by the library."""
import numpy as np
import pytest

from paper_1703_10440_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover - CPU container
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1703_10440_amd import amgs  # noqa: E402

DEV = torch.device("cuda:0")


@pytest.mark.parametrize("raw", [False, True], ids=["torch_stream", "raw_handle"])
@pytest.mark.parametrize("variant,panel", [("ha", 0), ("hp", 0), ("ha", 4), ("ha", 16)])
def test_side_stream_single(variant, panel, raw):
    p = inputs.laplacian_graded_problem(N=24, n=12, decades=3.0, seed=31)
    print(f"[gpu] side stream {variant} panel={panel} raw={raw}", flush=True)
    rp = torch.from_numpy(p.csr.row_ptr).to(DEV)
    ci = torch.from_numpy(p.csr.col_idx).to(DEV)
    va = torch.from_numpy(p.csr.vals).to(DEV)
    Z = torch.from_numpy(np.ascontiguousarray(p.Z)).to(DEV)
    ref_out = amgs.qr_csr(rp, ci, va, Z, variant=variant, panel=panel, return_p=True)
    torch.cuda.synchronize()
    side = torch.cuda.Stream(device=DEV)
    # inputs produced on the current stream right before the call: the side
    # stream must wait for them
    Z2 = torch.empty_like(Z)
    Z2.copy_(Z)
    out = amgs.qr_csr(rp, ci, va, Z2, variant=variant, panel=panel, return_p=True,
                      stream=side.cuda_stream if raw else side)
    del Z2   # the binding keeps it alive for the side stream
    side.synchronize()
    assert torch.equal(out.R, ref_out.R) and torch.equal(out.Q, ref_out.Q)
    assert torch.equal(out.P, ref_out.P) and int(out.info.item()) == 0


def test_side_stream_batched():
    g = inputs.rng(5)
    probs = []
    for k in range(12):
        m = int(g.integers(64, 900))
        n = int(g.integers(1, 20))
        gk = inputs.rng(2000 + k)
        probs.append((inputs.pentadiag_spd(gk, m), np.asfortranarray(gk.standard_normal((m, n)))))
    inst = [(torch.from_numpy(A.row_ptr).to(DEV), torch.from_numpy(A.col_idx).to(DEV),
             torch.from_numpy(A.vals).to(DEV), torch.from_numpy(np.ascontiguousarray(Z)).to(DEV))
            for A, Z in probs]
    print("[gpu] side stream batched", flush=True)
    Qs, Rs, info, plan, keep = amgs.qr_batched(inst, variant="ha")
    torch.cuda.synchronize()
    want = [R.clone() for R in Rs]
    side = torch.cuda.Stream(device=DEV)
    Qs2, Rs2, info2, _, keep2 = amgs.qr_batched(inst, variant="ha", stream=side)
    side.synchronize()
    assert int(info2.abs().max().item()) == 0
    for a, b in zip(want, Rs2):
        assert torch.equal(a, b)
    # passes of one plan alternate between two streams with no host
    # synchronisation in between: each waits for the previous one
    items, desc, work = keep
    other = torch.cuda.Stream(device=DEV)
    for rep in range(4):
        for R in Rs:
            R.fill_(-1.0)
        info.fill_(-9)
        plan.run(desc, work, info, stream=side if rep % 2 else other)
    torch.cuda.synchronize()
    assert int(info.abs().max().item()) == 0
    for a, b in zip(want, Rs):
        assert torch.equal(a, b)
