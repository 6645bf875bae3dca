"""Panel schedules of the GPU path against the oracle: one level (opts.panel
= 4, panels of four columns), two levels (opts.panel = 8, panels of eight
columns each taken apart as two panels of four) and three levels
(opts.panel = 16, panels of sixteen taken apart as two of eight; naive and
HA only).

Every GPU panel result is gated against the paper's column algorithms
(Alg. 3/5/6, the oracle's "col" orientation), with the tolerances of the
column schedule (tests/test_gpu_parity.py): R, Q, P within 1e-10 (relative,
Frobenius) for kappa(Z) <= 1e3; for kappa(Z) > 1e3 the residual and
||Q^T A Q - I||_2 within max(floor, 10x) the column oracle's; the binary32
form within 64 u_32 kappa(A^{1/2} Z) sqrt(n) of the column oracle's binary32
emulation, orthogonality within 10x.  As an extra check the same bounds are
applied against the oracle's panel orientation of the same schedule ("panel",
"panel8" or "panel16"), which performs the same regrouped operations step by
step (pinned in tests/pins.py, pin_panel, pin_panel8 and pin_panel16).
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
U32 = 2.0 ** -24
PANELS = (4, 8, 16)
ORIENT = {4: "panel", 8: "panel8", 16: "panel16"}


def variants_for(panel):
    """The three-level schedule has no HP form (AMGS_ERR_UNSUPPORTED)."""
    return ("naive", "ha") if panel == 16 else VARIANTS


def need(variant, panel):
    if variant not in variants_for(panel):
        pytest.skip("the three-level schedule has no HP form")


def _rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb else 1.0))


def gpu_run(prob, variant, precision="fp64", panel=4, reorth=False):
    Zt = torch.from_numpy(np.ascontiguousarray(prob.Z)).to(DEV)
    print(f"[gpu] panel={panel} {prob.name} m={prob.m} n={prob.n} {variant} {precision} "
          f"reorth={reorth}", flush=True)
    if prob.csr is not None:
        out = amgs.qr_csr(torch.from_numpy(prob.csr.row_ptr).to(DEV),
                          torch.from_numpy(prob.csr.col_idx).to(DEV),
                          torch.from_numpy(prob.csr.vals).to(DEV), Zt, variant=variant,
                          precision=precision, return_p=True, panel=panel, reorth=reorth)
    else:
        out = amgs.qr_dense(torch.from_numpy(np.ascontiguousarray(prob.dense)).to(DEV), Zt,
                            variant=variant, precision=precision, return_p=True, panel=panel,
                            reorth=reorth)
    torch.cuda.synchronize()
    return (out.Q.double().cpu().numpy(), out.R.cpu().numpy(), out.P.double().cpu().numpy(),
            int(out.info.item()), out.stats)


def oracle(prob, variant, precision="fp64", reorth=False, panel=4):
    return ref.qr_problem(prob, variant=variant, orientation=ORIENT[panel], precision=precision,
                          reorth=reorth)


def oracle_col(prob, variant, precision="fp64", reorth=False):
    """The paper's column algorithm (Alg. 3 / 5 / 6)."""
    return ref.qr_problem(prob, variant=variant, orientation="col", precision=precision,
                          reorth=reorth)


def close_1e10(R, Q, P, want, what):
    eR, eQ = _rel(R, want.R), _rel(Q, want.Q)
    eP = _rel(P, want.P) if P is not None else 0.0
    print(f"  vs {what}: R {eR:.2e} Q {eQ:.2e} P {eP:.2e}")
    assert eR <= 1e-10 and eQ <= 1e-10 and eP <= 1e-10, (what, eR, eQ, eP)


def at_oracle_level(prob, Q, R, want, what):
    """kappa(Z) > 1e3: residual and A-orthogonality at the oracle's level."""
    res_g, res_o = ref.residual(prob.Z, Q, R), ref.residual(prob.Z, want.Q, want.R)
    o_g, o_o = orth(prob, Q), orth(prob, want.Q)
    print(f"  vs {what}: residual {res_g:.2e} (oracle {res_o:.2e}) orth {o_g:.2e} "
          f"(oracle {o_o:.2e})")
    assert res_g <= max(1e-12, 10 * res_o), (what, res_g, res_o)
    assert o_g <= max(1e-13, 10 * o_o), (what, o_g, o_o)


def orth(prob, Q):
    return ref.orth_loss(Q, dense=prob.dense, csr=prob.csr)


def small_problems():
    return [
        inputs.laplacian_graded_problem(N=12, n=13, decades=2.0, seed=7),   # m=1728, 4 panels
        inputs.random_csr_problem(3001, 17, 40, seed=8),                    # 4 lanes/row
        inputs.random_csr_problem(2003, 9, 220, seed=9),                    # 32 lanes/row
        inputs.dense_gram_problem(512, 32, seed=1),                         # dense, 8 panels
        inputs.random_dense_problem(333, 21, seed=10),                      # ragged
    ]


SMALL = small_problems()


@pytest.mark.parametrize("panel", PANELS)
@pytest.mark.parametrize("reorth", [False, True])
@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("pi", range(len(SMALL)), ids=[p.name for p in SMALL])
def test_panel_fp64_parity(pi, variant, reorth, panel):
    need(variant, panel)
    p = SMALL[pi]
    col = oracle_col(p, variant, reorth=reorth)
    want = oracle(p, variant, reorth=reorth, panel=panel)
    Q, R, P, info, st = gpu_run(p, variant, reorth=reorth, panel=panel)
    assert info == 0 and want.info == 0 and col.info == 0
    print(f"  |Q^TAQ-I| {orth(p, Q):.2e}")
    close_1e10(R, Q, P, col, "column algorithm")
    close_1e10(R, Q, P, want, "panel orientation")
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)
    assert st.mv_calls == {"naive": 2 * p.n, "ha": p.n, "hp": 1}[variant]


@pytest.mark.parametrize("panel", PANELS)
@pytest.mark.parametrize("reorth", [False, True])
@pytest.mark.parametrize("variant", VARIANTS)
def test_panel_graded_ill_conditioned(variant, reorth, panel):
    """kappa(Z) ~ 1e6, 6 panels of four (3 of eight): residual and
    orthogonality at the oracle's level."""
    need(variant, panel)
    p = inputs.laplacian_graded_problem(N=16, n=24, decades=6.0, seed=11)
    col = oracle_col(p, variant, reorth=reorth)
    want = oracle(p, variant, reorth=reorth, panel=panel)
    Q, R, P, info, _ = gpu_run(p, variant, reorth=reorth, panel=panel)
    assert info == 0
    at_oracle_level(p, Q, R, col, "column algorithm")
    at_oracle_level(p, Q, R, want, "panel orientation")


@pytest.mark.parametrize("panel", PANELS)
@pytest.mark.parametrize("reorth", [False, True])
@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("pi", [0, 1, 3], ids=[SMALL[i].name for i in (0, 1, 3)])
def test_panel_fp32_form(pi, variant, reorth, panel):
    need(variant, panel)
    p = SMALL[pi]
    Z32 = np.asfortranarray(p.Z.astype(np.float32).astype(np.float64))
    if p.csr is not None:
        p32 = inputs.Problem(p.name, Z32, csr=inputs.CSR(
            p.m, p.csr.row_ptr, p.csr.col_idx, p.csr.vals.astype(np.float32).astype(np.float64)))
    else:
        p32 = inputs.Problem(p.name, Z32, dense=np.asfortranarray(
            p.dense.astype(np.float32).astype(np.float64)))
    kappa = np.linalg.cond(oracle_col(p32, variant).R)
    Q, R, P, info, _ = gpu_run(p32, variant, precision="fp32", reorth=reorth, panel=panel)
    assert info == 0
    tol = 64 * U32 * kappa * np.sqrt(p.n)
    o_g = orth(p32, Q)
    for what, want32 in (("column algorithm", oracle_col(p32, variant, "fp32", reorth=reorth)),
                         ("panel orientation", oracle(p32, variant, "fp32", reorth=reorth,
                                                      panel=panel))):
        e32 = _rel(R, want32.R)
        o_o = orth(p32, want32.Q)
        print(f"  R vs fp32 {what} {e32:.2e} tol {tol:.2e} orth {o_g:.2e} (oracle {o_o:.2e})")
        assert e32 <= tol, what
        assert o_g <= max(10 * o_o, 1e-6), what


@pytest.mark.parametrize("panel", PANELS)
@pytest.mark.parametrize("variant", VARIANTS)
def test_panel_many_workgroups_deterministic(variant, panel):
    """m = 64000, n = 40: the sweeps after each panel run hundreds of row
    chunks and several column groups; parity and bit-identical repeats."""
    need(variant, panel)
    p = inputs.laplacian_graded_problem(N=40, n=40, decades=2.0, seed=14)
    Q, R, P, info, _ = gpu_run(p, variant, panel=panel)
    Q2, R2, _, _, _ = gpu_run(p, variant, panel=panel)
    assert info == 0
    assert np.array_equal(R, R2) and np.array_equal(Q, Q2)
    print(f"  orth {orth(p, Q):.2e}")
    close_1e10(R, Q, P, oracle_col(p, variant), "column algorithm")
    close_1e10(R, Q, P, oracle(p, variant, panel=panel), "panel orientation")


@pytest.mark.parametrize("panel", PANELS)
def test_panel_edges(panel):
    """Panel boundaries: n = 1, 4 (one full panel), 5 (a one-column last
    panel), 8 (one outer panel), 9 (an outer panel and one column), 12, 16
    (one sixteen-panel), 17, 24 (a sixteen-panel and one eight-panel), 33;
    square and tiny m; dense and CSR."""
    g = inputs.rng(15)
    for m, n in ((700, 1), (300, 4), (300, 5), (200, 8), (300, 9), (300, 12), (300, 16),
                 (300, 17), (300, 24), (300, 33), (40, 40), (5, 3)):
        A = inputs.gram_spd(g, m)
        Z = np.asfortranarray(g.standard_normal((m, n)))
        for prob in (inputs.Problem(f"edge{m}x{n}", Z, dense=A),
                     inputs.Problem(f"edgecsr{m}x{n}", Z, csr=inputs.csr_from_dense(A))):
            for v in variants_for(panel):
                Q, R, P, info, _ = gpu_run(prob, v, panel=panel)
                assert info == 0
                for what, want in (("column", oracle_col(prob, v)),
                                   ("panel", oracle(prob, v, panel=panel))):
                    assert _rel(R, want.R) <= 1e-10, (prob.name, v, what, _rel(R, want.R))
                    assert _rel(Q, want.Q) <= 1e-10, (prob.name, v, what, _rel(Q, want.Q))


@pytest.mark.parametrize("panel", PANELS)
def test_panel_breakdown_reports_column(panel):
    """A zero column in the second panel (column 6) and a NaN in the third
    (column 10) stop at the right index; earlier columns stay valid."""
    g = inputs.rng(16)
    m, n = 300, 12
    A = inputs.gram_spd(g, m)
    Z = np.asfortranarray(g.standard_normal((m, n)))
    Zc = Z.copy(order="F")
    Zc[:, 5] = 0.0
    Zn = Z.copy(order="F")
    Zn[7, 9] = np.nan
    for v in variants_for(panel):
        _, R, _, info, _ = gpu_run(inputs.Problem("zero", Zc, dense=A), v, panel=panel)
        want = oracle(inputs.Problem("zero", Zc, dense=A), v, panel=panel)
        col = oracle_col(inputs.Problem("zero", Zc, dense=A), v)
        assert info == 6 and want.info == 6 and col.info == 6
        assert _rel(R[:5, :5], want.R[:5, :5]) <= 1e-10
        assert _rel(R[:5, :5], col.R[:5, :5]) <= 1e-10
        _, _, _, info, _ = gpu_run(inputs.Problem("nan", Zn, csr=inputs.csr_from_dense(A)), v,
                                   panel=panel)
        assert info == 10


@pytest.mark.parametrize("panel", PANELS)
def test_panel_breakdown_in_a_later_panel(panel):
    """n = 40: a zero column in the second sixteen-panel (column 21) and a NaN
    in the third (column 35), so the block sweeps between panels (and, with
    three levels, the update-only and dots-only sweeps) run before the
    breakdown.  The reported column is the oracle's; the columns before it
    agree with both oracles."""
    g = inputs.rng(18)
    m, n = 300, 40
    A = inputs.gram_spd(g, m)
    Z = np.asfortranarray(g.standard_normal((m, n)))
    Zc = Z.copy(order="F")
    Zc[:, 20] = 0.0
    Zn = Z.copy(order="F")
    Zn[7, 34] = np.nan
    for v in variants_for(panel):
        pz = inputs.Problem("zero40", Zc, dense=A)
        _, R, _, info, _ = gpu_run(pz, v, panel=panel)
        want, col = oracle(pz, v, panel=panel), oracle_col(pz, v)
        assert info == 21 and want.info == 21 and col.info == 21, (v, info)
        assert _rel(R[:20, :20], want.R[:20, :20]) <= 1e-10
        assert _rel(R[:20, :20], col.R[:20, :20]) <= 1e-10
        pn = inputs.Problem("nan40", Zn, csr=inputs.csr_from_dense(A))
        _, R, _, info, _ = gpu_run(pn, v, panel=panel)
        want = oracle(pn, v, panel=panel)
        assert info == 35 and want.info == 35, (v, info, want.info)
        assert _rel(R[:34, :34], want.R[:34, :34]) <= 1e-10


def test_panel_argument_errors():
    h = amgs.handle(0)
    import ctypes as C
    info = torch.zeros(1, dtype=torch.int32, device=DEV)
    Z = torch.zeros(10, 4, dtype=torch.float64, device=DEV)
    work = torch.empty(1 << 20, dtype=torch.uint8, device=DEV)
    # panel values other than 4, 8 and 16 are invalid; the panel schedules
    # with classical Gram-Schmidt are not supported (with the second pass they
    # are), nor the three-level one with HP (variant 2)
    for panel, cgs, var, want in ((3, 0, 1, -1), (12, 0, 1, -1), (32, 0, 1, -1), (4, 1, 1, -4),
                                  (8, 1, 1, -4), (16, 1, 1, -4), (16, 0, 2, -4)):
        opts = amgs.Opts(0, panel, cgs, 0)
        st = amgs.amgs_qr_dense(h, 10, Z.data_ptr(), 10, 4, Z.data_ptr(), 10, Z.data_ptr(), 10,
                                Z.data_ptr(), 4, None, 0, var, 0, C.byref(opts), work.data_ptr(),
                                work.numel(), info.data_ptr(), None)
        assert st == want, (panel, cgs, var, st)
    assert amgs.amgs_workspace_bytes(h, 10, 4, 1, 1, 0, 0, amgs.Opts(0, 3, 0, 0)) == 0
    assert amgs.amgs_workspace_bytes(h, 10, 4, 1, 2, 0, 0, amgs.Opts(0, 16, 0, 0)) == 0
    for panel in (4, 8, 16):
        assert amgs.amgs_workspace_bytes(h, 10, 4, 1, 1, 0, 0, amgs.Opts(0, panel, 0, 0)) > 0


# ----------------------------------------------- blocked second pass (reorth=2)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("pi", [0, 1, 3, 4], ids=[SMALL[i].name for i in (0, 1, 3, 4)])
def test_blocked_second_pass(pi, variant, precision):
    """opts.reorth = 2 in the two-level schedule against the oracle's blocked
    pass and against the per-column pass of the column algorithm: binary64
    within 1e-10 (kappa(Z) <= 1e3 here), the binary32 form within the
    binary32 bound and at the oracle's orthogonality."""
    p = SMALL[pi]
    if precision == "fp32":
        Z32 = np.asfortranarray(p.Z.astype(np.float32).astype(np.float64))
        if p.csr is not None:
            p = inputs.Problem(p.name, Z32, csr=inputs.CSR(
                p.m, p.csr.row_ptr, p.csr.col_idx, p.csr.vals.astype(np.float32).astype(np.float64)))
        else:
            p = inputs.Problem(p.name, Z32, dense=np.asfortranarray(
                p.dense.astype(np.float32).astype(np.float64)))
    Q, R, P, info, _ = gpu_run(p, variant, precision=precision, panel=8, reorth=2)
    assert info == 0
    blk = ref.qr_problem(p, variant=variant, orientation="panel8", precision=precision, reorth=2)
    col = ref.qr_problem(p, variant=variant, orientation="col", precision=precision, reorth=True)
    assert blk.info == 0 and col.info == 0
    if precision == "fp64":
        close_1e10(R, Q, P, col, "column algorithm, per-column pass")
        close_1e10(R, Q, P, blk, "panel8 orientation, blocked pass")
    else:
        kappa = np.linalg.cond(oracle_col(p, variant).R)
        tol = 64 * U32 * kappa * np.sqrt(p.n)
        o_g = orth(p, Q)
        for what, want in (("column algorithm, per-column pass", col),
                           ("panel8 orientation, blocked pass", blk)):
            e32, o_o = _rel(R, want.R), orth(p, want.Q)
            print(f"  R vs fp32 {what} {e32:.2e} tol {tol:.2e} orth {o_g:.2e} (oracle {o_o:.2e})")
            assert e32 <= tol, what
            assert o_g <= max(10 * o_o, 1e-6), what


@pytest.mark.parametrize("variant", ["naive", "ha"])
def test_blocked_second_pass_ill_conditioned(variant):
    """kappa(Z) ~ 1e6, three outer panels, binary32 form: the blocked pass
    restores A-orthogonality to the per-column pass's level."""
    p0 = inputs.laplacian_graded_problem(N=16, n=24, decades=6.0, seed=11)
    Z32 = np.asfortranarray(p0.Z.astype(np.float32).astype(np.float64))
    p = inputs.Problem(p0.name, Z32, csr=inputs.CSR(
        p0.m, p0.csr.row_ptr, p0.csr.col_idx, p0.csr.vals.astype(np.float32).astype(np.float64)))
    Q0, _, _, _, _ = gpu_run(p, variant, precision="fp32", panel=8)
    Q, R, _, info, _ = gpu_run(p, variant, precision="fp32", panel=8, reorth=2)
    assert info == 0
    blk = ref.qr_problem(p, variant=variant, orientation="panel8", precision="fp32", reorth=2)
    o0, o_g, o_o = orth(p, Q0), orth(p, Q), orth(p, blk.Q)
    print(f"  orth without pass {o0:.2e}, blocked pass {o_g:.2e} (oracle {o_o:.2e})")
    assert o_g <= max(10 * o_o, 1e-6) and o_g < 1e-2 * o0
    assert ref.residual(p.Z, Q, R) <= 10 * ref.residual(p.Z, blk.Q, blk.R) + 1e-7


def test_blocked_second_pass_needs_two_levels():
    h = amgs.handle(0)
    import ctypes as C
    info = torch.zeros(1, dtype=torch.int32, device=DEV)
    Z = torch.zeros(10, 4, dtype=torch.float64, device=DEV)
    work = torch.empty(1 << 20, dtype=torch.uint8, device=DEV)
    for reorth, panel, want in ((2, 0, -4), (2, 4, -4), (3, 8, -1)):
        opts = amgs.Opts(reorth, panel, 0, 0)
        st = amgs.amgs_qr_dense(h, 10, Z.data_ptr(), 10, 4, Z.data_ptr(), 10, Z.data_ptr(), 10,
                                Z.data_ptr(), 4, None, 0, 1, 0, C.byref(opts), work.data_ptr(),
                                work.numel(), info.data_ptr(), None)
        assert st == want, (reorth, panel, st)
    assert amgs.amgs_workspace_bytes(h, 10, 4, 1, 1, 0, 0, amgs.Opts(2, 8, 0, 0)) > 0
    assert amgs.amgs_workspace_bytes(h, 10, 4, 1, 1, 0, 0, amgs.Opts(2, 4, 0, 0)) == 0


WIDE = [inputs.random_csr_problem(3001, 45, 40, seed=17),
        inputs.dense_gram_problem(512, 40, seed=18)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("case", [(8, 1), (8, 3), (16, 0), (16, 1)],
                         ids=["8-" + SMALL[1].name, "8-" + SMALL[3].name, "16-" + WIDE[0].name,
                              "16-" + WIDE[1].name])
def test_two_level_working_copy(case, variant, precision):
    """Two- and three-level schedules: only the first two eight-panels (the
    first sixteen-panel) are copied from Z before the call's work; the block
    sweep after the second eight-panel reads the later columns from Z (three
    levels: the update-only sweep before the second sixteen-panel reads its
    columns from Z, the sweep after it the later ones).  Out of place, Z must
    come back untouched; in place (Q aliases Z) the result must equal the
    out-of-place one bit for bit.  Every problem has n > 2 x the panel width,
    so the later columns take the Z path."""
    panel, pi = case
    need(variant, panel)
    p = SMALL[pi] if panel == 8 else WIDE[pi]
    assert p.n > 2 * panel
    dt = torch.float64 if precision == "fp64" else torch.float32
    Z0 = amgs.colmajor(torch.from_numpy(np.ascontiguousarray(p.Z)).to(DEV).to(dt))
    Zc = Z0.clone()

    def run(Zt, Q=None):
        print(f"[gpu] working copy panel={panel} {p.name} {variant} {precision} "
              f"inplace={Q is not None}",
              flush=True)
        kw = dict(variant=variant, precision=precision, return_p=True, panel=panel, Q=Q)
        if p.csr is not None:
            return amgs.qr_csr(torch.from_numpy(p.csr.row_ptr).to(DEV),
                               torch.from_numpy(p.csr.col_idx).to(DEV),
                               torch.from_numpy(p.csr.vals).to(DEV).to(dt), Zt, **kw)
        return amgs.qr_dense(torch.from_numpy(np.ascontiguousarray(p.dense)).to(DEV).to(dt),
                             Zt, **kw)

    a = run(Z0)
    torch.cuda.synchronize()
    assert torch.equal(Z0, Zc), "Z modified by an out-of-place call"
    b = run(Zc, Q=Zc)
    torch.cuda.synchronize()
    assert int(a.info.item()) == 0 and int(b.info.item()) == 0
    assert torch.equal(a.Q, Zc) and torch.equal(a.R, b.R) and torch.equal(a.P, b.P)
    want = oracle_col(p, variant, precision=precision)
    if precision == "fp64":
        close_1e10(a.R.cpu().numpy(), a.Q.cpu().numpy(), a.P.cpu().numpy(), want,
                   "column algorithm")
