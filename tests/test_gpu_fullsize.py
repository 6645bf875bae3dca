"""Parity at the full sizes of the measured workloads, in the launch
configurations bench.py times (same sizes, so the same kernels, tiles and
grids), against the oracle run on the whole problem.

Every result, panel schedule included, is gated against the paper's column
algorithm (Alg. 3 / 5 / 6; the oracle's "col" orientation, or its classical
form for CGS); panel results are also compared with the oracle's panel
orientation as an extra check.

* Laplacian 64^3 + 1e-2 I, Z 262144 x 64, kappa(Z) ~ 1e6 (no R bound
  applies): residual and ||Q^T A Q - I||_2 within max(floor, 10x) the
  oracle's -- naive, HA, HP in binary64; the second pass in binary64 and in
  the binary32 form; CGS and CGS2 (column schedule only).  At this m
  the column and second-pass kernels hold four rows per thread, the
  configuration the measured second-pass and CGS figures run.
* dense 16384 x 16384, Z 16384 x 256, kappa(Z) ~ 1.3: HP in binary64 (R, Q
  within 1e-10) and in the binary32 form (R within 64 u_32 kappa(R) sqrt(n)
  of the oracle's binary32 emulation, the 128 x 128 binary32 matrix-core
  tiles).
* Laplacian 128^3 + 1e-2 I, Z 2097152 x 128, kappa(Z) ~ 1e4: HA and HP in
  the binary32 form against the oracle's binary32 emulation on the same
  binary32 inputs (residual and orthogonality within 10x), and in binary64
  (residual and orthogonality within max(floor, 10x)).

Every case but CGS runs in the column schedule and in the one- and two-level
panel schedules (panels of four; panels of eight taken apart as panels of
four); the three-level schedule (panels of sixteen taken apart as panels of
eight) runs HA and naive on lap64 (with and without the second pass), HA on
lap128 in both precisions, and at lap128 also naive and HA with the
per-column second pass in both precisions.
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
U32 = 2.0 ** -24


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _run(prob, variant, precision, panel, reorth=False, cgs=False):
    print(f"[gpu] full size {prob.name} m={prob.m} n={prob.n} {variant} {precision} "
          f"panel={panel} reorth={reorth} cgs={cgs}", flush=True)
    Zt = torch.from_numpy(np.ascontiguousarray(prob.Z)).to(DEV)
    kw = dict(variant=variant, precision=precision, panel=panel, reorth=reorth, cgs=cgs)
    if prob.csr is not None:
        out = amgs.qr_csr(torch.from_numpy(prob.csr.row_ptr).to(DEV),
                          torch.from_numpy(prob.csr.col_idx).to(DEV),
                          torch.from_numpy(prob.csr.vals).to(DEV), Zt, **kw)
    else:
        out = amgs.qr_dense(torch.from_numpy(np.ascontiguousarray(prob.dense)).to(DEV), Zt, **kw)
    torch.cuda.synchronize()
    Q, R, info = out.Q.double().cpu().numpy(), out.R.cpu().numpy(), int(out.info.item())
    del out, Zt
    torch.cuda.empty_cache()
    return Q, R, info


def _oracles(prob, variant, precision, panel, reorth=False, cgs=False):
    """The column (or classical) algorithm, and for the panel schedule also
    the panel orientation."""
    kw = dict(variant=variant, precision=precision, reorth=reorth)
    outs = [("column algorithm",
             ref.qr_problem(prob, orientation="cgs" if cgs else "col", **kw))]
    if panel:
        outs.append(("panel orientation",
                     ref.qr_problem(prob, orientation={4: "panel", 8: "panel8", 16: "panel16"}[panel],
                                    **kw)))
    return outs


def _at_oracle_level(prob, Q, R, outs, floors=(1e-12, 1e-13)):
    """Residual and A-orthogonality of the GPU result within max(floor, 10x)
    of each oracle result in outs."""
    res_g = ref.residual(prob.Z, Q, R)
    o_g = ref.orth_loss(Q, csr=prob.csr, dense=prob.dense)
    for what, want in outs:
        assert want.info == 0, what
        res_o = ref.residual(prob.Z, want.Q, want.R)
        o_o = ref.orth_loss(want.Q, csr=prob.csr, dense=prob.dense)
        print(f"  vs {what}: residual {res_g:.2e} (oracle {res_o:.2e}) orth {o_g:.2e} "
              f"(oracle {o_o:.2e}) R rel {_rel(R, want.R):.2e}")
        assert res_g <= max(floors[0], 10 * res_o), (what, res_g, res_o)
        assert o_g <= max(floors[1], 10 * o_o), (what, o_g, o_o)


def _fp32_problem(p):
    """The same problem with every input rounded to binary32 (the oracle's
    binary32 emulation and the GPU then start from identical values)."""
    Z32 = np.asfortranarray(p.Z.astype(np.float32).astype(np.float64))
    if p.csr is not None:
        return inputs.Problem(p.name, Z32, csr=inputs.CSR(
            p.m, p.csr.row_ptr, p.csr.col_idx, p.csr.vals.astype(np.float32).astype(np.float64)))
    return inputs.Problem(p.name, Z32, dense=np.asfortranarray(
        p.dense.astype(np.float32).astype(np.float64)))


# ------------------------------------------------------------------- lap64
@pytest.fixture(scope="module")
def lap64():
    return inputs.WORKLOADS["lap64_n64"]()


@pytest.fixture(scope="module")
def lap64_fp32(lap64):
    return _fp32_problem(lap64)


@pytest.mark.parametrize("panel", [0, 4, 8])
@pytest.mark.parametrize("variant", ["hp", "ha", "naive"])
def test_lap64_full(lap64, variant, panel):
    p = lap64
    Q, R, info = _run(p, variant, "fp64", panel)
    assert info == 0
    _at_oracle_level(p, Q, R, _oracles(p, variant, "fp64", panel))


@pytest.mark.parametrize("panel", [0, 4, 8])
@pytest.mark.parametrize("variant", ["hp", "ha", "naive"])
def test_lap64_second_pass_fp64(lap64, variant, panel):
    p = lap64
    Q, R, info = _run(p, variant, "fp64", panel, reorth=True)
    assert info == 0
    _at_oracle_level(p, Q, R, _oracles(p, variant, "fp64", panel, reorth=True))


@pytest.mark.parametrize("panel", [0, 4, 8])
@pytest.mark.parametrize("variant", ["hp", "ha", "naive"])
def test_lap64_second_pass_fp32(lap64_fp32, variant, panel):
    p = lap64_fp32
    Q, R, info = _run(p, variant, "fp32", panel, reorth=True)
    assert info == 0
    _at_oracle_level(p, Q, R, _oracles(p, variant, "fp32", panel, reorth=True), floors=(0.0, 0.0))


@pytest.mark.parametrize("reorth", [False, True], ids=["cgs", "cgs2"])
@pytest.mark.parametrize("variant", ["hp", "ha", "naive"])
def test_lap64_cgs_fp64(lap64, variant, reorth):
    p = lap64
    Q, R, info = _run(p, variant, "fp64", 0, reorth=reorth, cgs=True)
    assert info == 0
    _at_oracle_level(p, Q, R, _oracles(p, variant, "fp64", 0, reorth=reorth, cgs=True))


@pytest.mark.parametrize("reorth", [False, True], ids=["cgs", "cgs2"])
def test_lap64_cgs_fp32(lap64_fp32, reorth):
    p = lap64_fp32
    Q, R, info = _run(p, "ha", "fp32", 0, reorth=reorth, cgs=True)
    assert info == 0
    _at_oracle_level(p, Q, R, _oracles(p, "ha", "fp32", 0, reorth=reorth, cgs=True), floors=(0.0, 0.0))


# ---------------------------------------------------------------- dense16k
@pytest.fixture(scope="module")
def dense16k():
    return inputs.dense16k_problem(device="cuda:0")


@pytest.mark.parametrize("panel", [0, 4, 8])
def test_dense16k_full(dense16k, panel):
    p = dense16k
    Q, R, info = _run(p, "hp", "fp64", panel)
    assert info == 0
    for what, want in _oracles(p, "hp", "fp64", panel):
        assert want.info == 0
        eR, eQ = _rel(R, want.R), _rel(Q, want.Q)
        print(f"  vs {what}: R {eR:.2e} Q {eQ:.2e}")
        assert eR <= 1e-10 and eQ <= 1e-10, what


@pytest.mark.parametrize("panel", [0, 4, 8])
def test_dense16k_fp32_full(dense16k, panel):
    p = _fp32_problem(dense16k)
    Q, R, info = _run(p, "hp", "fp32", panel)
    assert info == 0
    outs = _oracles(p, "hp", "fp32", panel)
    kappa = np.linalg.cond(outs[0][1].R)
    tol = 64 * U32 * kappa * np.sqrt(p.n)
    for what, want in outs:
        assert want.info == 0
        eR = _rel(R, want.R)
        o_g, o_o = ref.orth_loss(Q, dense=p.dense), ref.orth_loss(want.Q, dense=p.dense)
        print(f"  vs {what} (binary32 emulation): R {eR:.2e} tol {tol:.2e} orth {o_g:.2e} "
              f"(oracle {o_o:.2e})")
        assert eR <= tol, what
        assert o_g <= max(10 * o_o, 1e-6), what


# ------------------------------------------------------------------ lap128
@pytest.fixture(scope="module")
def lap128_fp64():
    return inputs.WORKLOADS["lap128_n128"]()


@pytest.fixture(scope="module")
def lap128_fp32(lap128_fp64):
    return _fp32_problem(lap128_fp64)


@pytest.mark.parametrize("panel", [0, 4, 8])
@pytest.mark.parametrize("variant", ["hp", "ha"])
def test_lap128_fp32_full(lap128_fp32, variant, panel):
    p = lap128_fp32
    Q, R, info = _run(p, variant, "fp32", panel)
    assert info == 0
    _at_oracle_level(p, Q, R, _oracles(p, variant, "fp32", panel), floors=(0.0, 0.0))


@pytest.mark.parametrize("panel", [0, 4, 8])
@pytest.mark.parametrize("variant", ["hp", "ha"])
def test_lap128_fp64_full(lap128_fp64, variant, panel):
    p = lap128_fp64
    Q, R, info = _run(p, variant, "fp64", panel)
    assert info == 0
    _at_oracle_level(p, Q, R, _oracles(p, variant, "fp64", panel))


@pytest.mark.parametrize("variant", ["hp", "ha"])
def test_lap128_fp32_blocked_second_pass(lap128_fp32, variant):
    """The binary32 form with the blocked second pass (reorth = 2, two-level
    schedule): residual and orthogonality at the level of the oracle's
    blocked pass on the same binary32 inputs."""
    p = lap128_fp32
    Q, R, info = _run(p, variant, "fp32", 8, reorth=2)
    assert info == 0
    want = ref.qr_problem(p, variant=variant, orientation="panel8", precision="fp32", reorth=2)
    _at_oracle_level(p, Q, R, [("panel8 orientation, blocked pass", want)], floors=(0.0, 0.0))


# ------------------------------------------- three-level schedule (panel 16)
@pytest.mark.parametrize("reorth", [False, True])
@pytest.mark.parametrize("variant", ["ha", "naive"])
def test_lap64_three_level(lap64, variant, reorth):
    p = lap64
    Q, R, info = _run(p, variant, "fp64", 16, reorth=reorth)
    assert info == 0
    _at_oracle_level(p, Q, R, _oracles(p, variant, "fp64", 16, reorth=reorth))


@pytest.mark.parametrize("variant", ["ha", "naive"])
def test_lap64_three_level_fp32_second_pass(lap64_fp32, variant):
    p = lap64_fp32
    Q, R, info = _run(p, variant, "fp32", 16, reorth=True)
    assert info == 0
    _at_oracle_level(p, Q, R, _oracles(p, variant, "fp32", 16, reorth=True), floors=(0.0, 0.0))


def test_lap128_three_level_fp64(lap128_fp64):
    p = lap128_fp64
    Q, R, info = _run(p, "ha", "fp64", 16)
    assert info == 0
    _at_oracle_level(p, Q, R, _oracles(p, "ha", "fp64", 16))


@pytest.mark.parametrize("variant,reorth", [("naive", False), ("ha", True)],
                         ids=["naive", "ha_second_pass"])
def test_lap128_three_level_other_forms(lap128_fp64, variant, reorth):
    """The naive form and HA with the per-column second pass at the headline
    size and schedule (both reported by bench.py's variants)."""
    p = lap128_fp64
    Q, R, info = _run(p, variant, "fp64", 16, reorth=reorth)
    assert info == 0
    _at_oracle_level(p, Q, R, _oracles(p, variant, "fp64", 16, reorth=reorth))


@pytest.mark.parametrize("variant,reorth", [("naive", False), ("ha", True)],
                         ids=["naive", "ha_second_pass"])
def test_lap128_three_level_other_forms_fp32(lap128_fp32, variant, reorth):
    p = lap128_fp32
    Q, R, info = _run(p, variant, "fp32", 16, reorth=reorth)
    assert info == 0
    _at_oracle_level(p, Q, R, _oracles(p, variant, "fp32", 16, reorth=reorth), floors=(0.0, 0.0))


def test_lap128_three_level_fp32(lap128_fp32):
    p = lap128_fp32
    Q, R, info = _run(p, "ha", "fp32", 16)
    assert info == 0
    _at_oracle_level(p, Q, R, _oracles(p, "ha", "fp32", 16), floors=(0.0, 0.0))


@pytest.mark.parametrize("variant", ["hp", "ha", "naive"])
def test_lap64_blocked_second_pass_fp64(lap64, variant):
    p = lap64
    Q, R, info = _run(p, variant, "fp64", 8, reorth=2)
    assert info == 0
    outs = [("column algorithm, per-column pass",
             ref.qr_problem(p, variant=variant, orientation="col", reorth=True)),
            ("panel8 orientation, blocked pass",
             ref.qr_problem(p, variant=variant, orientation="panel8", reorth=2))]
    _at_oracle_level(p, Q, R, outs)
