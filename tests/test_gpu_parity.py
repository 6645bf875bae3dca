"""GPU path (HIP library through the C ABI) against the CPU oracle.

Tolerances:
* binary64, kappa(Z) <= 1e3: ||R_gpu - R_ref||_F / ||R_ref||_F <= 1e-10, the
  same for Q and P = AQ;
* binary64, kappa(Z) > 1e3: no R tolerance applies (R's error grows with
  kappa); the residual ||Z - QR||_F/||Z||_F must stay at the oracle's level
  (<= max(1e-12, 10x oracle)) and ||Q^T A Q - I||_2 <= max(1e-13, 10x oracle);
* binary32 form: against the oracle's binary32 emulation on the same
  binary32 inputs, R within 64 u_32 kappa(A^{1/2} Z) sqrt(n) (first-order
  rounding bound of the projections, u_32 = 2^-24), and the A-orthogonality
  within 10x the oracle's.
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


def _rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb else 1.0))


def gpu_run(prob, variant, precision="fp64", reorth=False, Z=None, **kw):
    Z = prob.Z if Z is None else Z
    Zt = torch.from_numpy(np.ascontiguousarray(Z)).to(DEV)
    print(f"[gpu] {prob.name} m={prob.m} n={Z.shape[1]} {variant} {precision} "
          f"reorth={reorth}", flush=True)
    if prob.csr is not None:
        vals = prob.csr.vals
        out = amgs.qr_csr(torch.from_numpy(prob.csr.row_ptr).to(DEV),
                          torch.from_numpy(prob.csr.col_idx).to(DEV),
                          torch.from_numpy(vals).to(DEV), Zt, variant=variant,
                          precision=precision, reorth=reorth, return_p=True, **kw)
    else:
        out = amgs.qr_dense(torch.from_numpy(np.ascontiguousarray(prob.dense)).to(DEV), Zt,
                            variant=variant, precision=precision, reorth=reorth,
                            return_p=True, **kw)
    torch.cuda.synchronize()
    return (out.Q.double().cpu().numpy(), out.R.cpu().numpy(), out.P.double().cpu().numpy(),
            int(out.info.item()), out.stats)


def A_dense(prob):
    return prob.dense if prob.dense is not None else prob.csr.to_dense()


def orth(prob, Q):
    return ref.orth_loss(Q, dense=prob.dense, csr=prob.csr)


# Small problems spanning several tiles with ragged tails --------------------
def small_problems():
    return [
        inputs.laplacian_graded_problem(N=12, n=13, decades=2.0, seed=7),   # m=1728
        inputs.random_csr_problem(3001, 17, 40, seed=8),                    # 4 lanes/row
        inputs.random_csr_problem(2003, 9, 220, seed=9),                    # 32 lanes/row
        inputs.dense_gram_problem(512, 32, seed=1),                         # dense 512 x 32
        inputs.random_dense_problem(333, 21, seed=10),                      # ragged GEMM tiles
        inputs.random_csr_problem(3001, 11, 5, seed=12),                    # short rows, some past K
    ]


SMALL = small_problems()


@pytest.mark.parametrize("reorth", [False, True])
@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("pi", range(len(SMALL)), ids=[p.name for p in SMALL])
def test_fp64_parity_small(pi, variant, reorth):
    p = SMALL[pi]
    want = ref.qr_problem(p, variant=variant, reorth=reorth)
    Q, R, P, info, st = gpu_run(p, variant, reorth=reorth)
    assert info == 0 and want.info == 0
    eR, eQ, eP = _rel(R, want.R), _rel(Q, want.Q), _rel(P, want.P)
    loss = orth(p, Q)
    print(f"  R {eR:.2e} Q {eQ:.2e} P {eP:.2e} |Q^TAQ-I| {loss:.2e}")
    assert eR <= 1e-10 and eQ <= 1e-10 and eP <= 1e-10
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)
    exp_calls = {"naive": 2 * p.n, "ha": p.n, "hp": 1}[variant]
    assert st.mv_calls == exp_calls


@pytest.mark.parametrize("variant", VARIANTS)
def test_fp64_graded_ill_conditioned(variant):
    """kappa(Z) ~ 1e6: residual and orthogonality at the oracle's level."""
    p = inputs.laplacian_graded_problem(N=16, n=24, decades=6.0, seed=11)
    want = ref.qr_problem(p, variant=variant)
    Q, R, P, info, _ = gpu_run(p, variant)
    assert info == 0
    res_g, res_o = ref.residual(p.Z, Q, R), ref.residual(p.Z, want.Q, want.R)
    o_g, o_o = orth(p, Q), orth(p, want.Q)
    print(f"  residual {res_g:.2e} (oracle {res_o:.2e}) orth {o_g:.2e} (oracle {o_o:.2e}) "
          f"R {_rel(R, want.R):.2e}")
    assert res_g <= max(1e-12, 10 * res_o)
    assert o_g <= max(1e-13, 10 * o_o)


@pytest.mark.parametrize("reorth", [False, True])
@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("pi", [0, 1, 3], ids=[SMALL[i].name for i in (0, 1, 3)])
def test_fp32_form_parity(pi, variant, reorth):
    p = SMALL[pi]
    Z32 = np.asfortranarray(p.Z.astype(np.float32).astype(np.float64))
    if p.csr is not None:
        A32 = inputs.CSR(p.m, p.csr.row_ptr, p.csr.col_idx,
                         p.csr.vals.astype(np.float32).astype(np.float64))
        p32 = inputs.Problem(p.name, Z32, csr=A32)
    else:
        p32 = inputs.Problem(p.name, Z32, dense=np.asfortranarray(
            p.dense.astype(np.float32).astype(np.float64)))
    want32 = ref.qr_problem(p32, variant=variant, reorth=reorth, precision="fp32")
    want64 = ref.qr_problem(p32, variant=variant, reorth=reorth, precision="fp64")
    Q, R, P, info, _ = gpu_run(p32, variant, precision="fp32", reorth=reorth)
    assert info == 0
    kappa = np.linalg.cond(want64.R)
    tol = 64 * U32 * kappa * np.sqrt(p.n)
    e32, e64 = _rel(R, want32.R), _rel(R, want64.R)
    o_g, o_o = orth(p32, Q), orth(p32, want32.Q)
    print(f"  R vs fp32-oracle {e32:.2e} vs fp64 {e64:.2e} tol {tol:.2e} orth {o_g:.2e} "
          f"(oracle fp32 {o_o:.2e})")
    assert e32 <= tol
    assert o_g <= max(10 * o_o, 1e-6)


def test_determinism_and_inplace():
    p = SMALL[0]
    a = gpu_run(p, "ha")
    b = gpu_run(p, "ha")
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[0], b[0])
    # in place: Q aliases Z
    Zt = amgs.colmajor(torch.from_numpy(np.ascontiguousarray(p.Z)).to(DEV))
    out = amgs.qr_csr(torch.from_numpy(p.csr.row_ptr).to(DEV),
                      torch.from_numpy(p.csr.col_idx).to(DEV),
                      torch.from_numpy(p.csr.vals).to(DEV), Zt, variant="ha", Q=Zt)
    torch.cuda.synchronize()
    assert np.array_equal(Zt.cpu().numpy(), a[0])
    assert np.array_equal(out.R.cpu().numpy(), a[1])


def test_edge_shapes():
    g = inputs.rng(12)
    # n = 1, square m = n, tiny m
    for m, n in ((700, 1), (40, 40), (5, 3)):
        A = inputs.gram_spd(g, m)
        Z = np.asfortranarray(g.standard_normal((m, n)))
        p = inputs.Problem(f"edge{m}x{n}", Z, dense=A)
        pc = inputs.Problem(f"edgecsr{m}x{n}", Z, csr=inputs.csr_from_dense(A))
        for prob in (p, pc):
            for v in VARIANTS:
                want = ref.qr_problem(prob, variant=v)
                Q, R, P, info, _ = gpu_run(prob, v)
                assert info == 0
                assert _rel(R, want.R) <= 1e-10, (prob.name, v, _rel(R, want.R))


def test_breakdown_reports_column():
    g = inputs.rng(13)
    m, n = 300, 6
    A = inputs.gram_spd(g, m)
    Z = np.asfortranarray(g.standard_normal((m, n)))
    Zc = Z.copy(order="F")
    Zc[:, 3] = 0.0
    for v in VARIANTS:
        _, R, _, info, _ = gpu_run(inputs.Problem("zero", Zc, dense=A), v)
        assert info == 4
        want = ref.qr(Zc, dense=A, variant=v)
        assert _rel(R[:3, :3], want.R[:3, :3]) <= 1e-10
        _, _, _, info, _ = gpu_run(inputs.Problem("neg", Z, csr=inputs.csr_from_dense(-A)), v)
        assert info == 1
        Zn = Z.copy(order="F")
        Zn[5, 2] = np.nan
        _, _, _, info, _ = gpu_run(inputs.Problem("nan", Zn, dense=A), v)
        assert info == 3


def test_csr_check():
    p = SMALL[0]
    rp = torch.from_numpy(p.csr.row_ptr).to(DEV)
    ci = torch.from_numpy(p.csr.col_idx).to(DEV)
    assert amgs.csr_check(rp, ci, p.m)
    bad = ci.clone()
    bad[17] = p.m  # out of range index
    assert not amgs.csr_check(rp, bad, p.m)


def test_argument_errors():
    h = amgs.handle(0)
    import ctypes as C
    info = torch.zeros(1, dtype=torch.int32, device=DEV)
    Z = torch.zeros(10, 4, dtype=torch.float64, device=DEV)
    # m < n
    st = amgs.amgs_qr_dense(h, 3, Z.data_ptr(), 3, 4, Z.data_ptr(), 3, Z.data_ptr(), 3,
                            Z.data_ptr(), 4, None, 0, 1, 0, None, Z.data_ptr(), 1 << 20,
                            info.data_ptr(), None)
    assert st == -1
    # workspace too small
    st = amgs.amgs_qr_dense(h, 10, Z.data_ptr(), 10, 4, Z.data_ptr(), 10, Z.data_ptr(), 10,
                            Z.data_ptr(), 4, None, 0, 1, 0, None, Z.data_ptr(), 8,
                            info.data_ptr(), None)
    assert st == -2
    # n = 0 is a no-op
    st = amgs.amgs_qr_dense(h, 10, Z.data_ptr(), 10, 0, Z.data_ptr(), 10, Z.data_ptr(), 10,
                            Z.data_ptr(), 1, None, 0, 1, 0, None, None, 0, info.data_ptr(), None)
    assert st == 0


@pytest.mark.parametrize("variant", VARIANTS)
def test_padded_leading_dimensions(variant):
    """Z, Q, P and R given with leading dimensions larger than their row
    counts: the results equal those of unpadded buffers bit for bit, and the
    padding rows are left untouched."""
    for p in (SMALL[0], SMALL[3]):
        m, n = p.Z.shape
        ref_run = gpu_run(p, variant)

        def padded(rows, cols, pad, dtype=torch.float64):
            buf = torch.full((cols, rows + pad), float("nan"), dtype=dtype, device=DEV).t()
            return buf, buf[:rows, :]

        zb, Zv = padded(m, n, 7)
        Zv.copy_(torch.from_numpy(np.ascontiguousarray(p.Z)))
        qb, Qv = padded(m, n, 3)
        pb, Pv = padded(m, n, 5)
        rb, Rv = padded(n, n, 2)
        kw = dict(variant=variant, Q=Qv, P=Pv, R=Rv)
        print(f"[gpu] padded {p.name} {variant}", flush=True)
        if p.csr is not None:
            out = amgs.qr_csr(torch.from_numpy(p.csr.row_ptr).to(DEV),
                              torch.from_numpy(p.csr.col_idx).to(DEV),
                              torch.from_numpy(p.csr.vals).to(DEV), Zv, **kw)
        else:
            out = amgs.qr_dense(torch.from_numpy(np.ascontiguousarray(p.dense)).to(DEV), Zv, **kw)
        torch.cuda.synchronize()
        assert int(out.info.item()) == 0
        assert np.array_equal(Qv.cpu().numpy(), ref_run[0])
        assert np.array_equal(Rv.cpu().numpy(), ref_run[1])
        assert np.array_equal(Pv.cpu().numpy(), ref_run[2])
        for buf, rows in ((qb, m), (pb, m), (rb, n)):
            assert torch.isnan(buf[rows:, :]).all()


def _arrow(m):
    """Row and column 0 full, diagonal m+1 there and 3 elsewhere: strictly
    diagonally dominant, so spd.  Mean row length ~3, one row of m entries."""
    rows, cols, vals = [], [], []
    for i in range(m):
        if i == 0:
            rows += [0] * m
            cols += list(range(m))
            vals += [m + 1.0] + [-1.0] * (m - 1)
        else:
            rows += [i, i]
            cols += [0, i]
            vals += [-1.0, 3.0]
    row_ptr = np.zeros(m + 1, dtype=np.int64)
    np.add.at(row_ptr, np.array(rows) + 1, 1)
    return inputs.CSR(m, np.cumsum(row_ptr).astype(np.int32), np.array(cols, dtype=np.int32),
                      np.array(vals))


@pytest.mark.parametrize("variant", ["naive", "ha"])
def test_short_rows_with_long_tails(variant):
    """The column MV for short rows reads the first K entries of each row
    from a padded copy and the rest from CSR: one row of every entry (arrow
    matrix, K = 3), and rows of exactly K and K + 1 entries."""
    g = inputs.rng(21)
    for A in (_arrow(2500), _arrow(513)):
        Z = np.asfortranarray(g.standard_normal((A.m, 7)))
        p = inputs.Problem(f"arrow{A.m}", Z, csr=A)
        want = ref.qr_problem(p, variant=variant)
        Q, R, P, info, _ = gpu_run(p, variant)
        assert info == 0 and want.info == 0
        eR, eQ, eP = _rel(R, want.R), _rel(Q, want.Q), _rel(P, want.P)
        print(f"  {p.name}: R {eR:.2e} Q {eQ:.2e} P {eP:.2e}")
        assert eR <= 1e-10 and eQ <= 1e-10 and eP <= 1e-10
    # tridiagonal (K = 3, rows of 2 and 3) with a few rows of 4 entries
    m = 1500
    D = np.diag(np.full(m, 4.0)) + np.diag(np.full(m - 1, -1.0), 1) + np.diag(np.full(m - 1, -1.0), -1)
    for i in (5, 700, 1499):
        j = (i + 37) % m
        D[i, j] = D[j, i] = -0.5
    Z = np.asfortranarray(g.standard_normal((m, 9)))
    p = inputs.Problem("tri_plus", Z, csr=inputs.csr_from_dense(D))
    want = ref.qr_problem(p, variant=variant)
    Q, R, P, info, _ = gpu_run(p, variant)
    assert info == 0 and want.info == 0
    assert _rel(R, want.R) <= 1e-10 and _rel(Q, want.Q) <= 1e-10 and _rel(P, want.P) <= 1e-10


@pytest.mark.parametrize("variant", ["naive", "ha"])
def test_short_rows_several_tiles_per_workgroup(variant):
    """Laplacian 96^3 (884,736 rows): 1728 tiles of the short-row column MV
    over at most 512 workgroups, so each thread takes rows of two tiles at
    once, and the last pair of some workgroups has one tile."""
    p = inputs.laplacian_graded_problem(N=96, n=6, decades=1.0, seed=23)
    want = ref.qr_problem(p, variant=variant)
    Q, R, P, info, _ = gpu_run(p, variant)
    assert info == 0 and want.info == 0
    eR, eQ, eP = _rel(R, want.R), _rel(Q, want.Q), _rel(P, want.P)
    print(f"  R {eR:.2e} Q {eQ:.2e} P {eP:.2e}")
    assert eR <= 1e-10 and eQ <= 1e-10 and eP <= 1e-10


@pytest.mark.parametrize("per_row", [10, 20, 40, 80, 150, 300, 500])
def test_hp_block_product_lane_widths(per_row):
    """HP's block product X = AZ for CSR picks a thread per row (mean row
    length <= 12) or L = 2 .. 64 lanes per row from the mean row length, and
    takes Z in groups of 8 columns: every lane width, n = 11 (a ragged last
    group), against the oracle."""
    p = inputs.random_csr_problem(1500, 11, per_row, seed=30 + per_row)
    want = ref.qr_problem(p, variant="hp")
    Q, R, P, info, _ = gpu_run(p, "hp")
    assert info == 0 and want.info == 0
    eR, eQ, eP = _rel(R, want.R), _rel(Q, want.Q), _rel(P, want.P)
    print(f"  mean row length {p.csr.nnz / p.m:.1f}: R {eR:.2e} Q {eQ:.2e} P {eP:.2e}")
    assert eR <= 1e-10 and eQ <= 1e-10 and eP <= 1e-10


def _align256(x):
    return (x + 255) // 256 * 256


@pytest.mark.parametrize("panel", [0, 4])
@pytest.mark.parametrize("variant", ["naive", "ha"])
def test_workspace_without_padded_copy(variant, panel):
    """A workspace without room for the padded copy of A is accepted; the
    column MV then reads CSR directly, in the same stored order, so Q, R and
    P equal the full-workspace call bit for bit.  One byte less is refused."""
    for p in (SMALL[0], SMALL[5]):
        m, n = p.Z.shape
        rp = torch.from_numpy(p.csr.row_ptr).to(DEV)
        ci = torch.from_numpy(p.csr.col_idx).to(DEV)
        va = torch.from_numpy(p.csr.vals).to(DEV)
        Z = torch.from_numpy(np.ascontiguousarray(p.Z)).to(DEV)
        h = amgs.handle(0)
        opts = amgs.Opts(0, panel, 0, 0)
        full = amgs.amgs_workspace_bytes(h, m, n, 0, amgs.VARIANTS[variant],
                                         amgs.PRECISIONS["fp64"], 1, opts)   # P passed
        # the padded copy: 32-bit columns, values, per-tile flags, 16-bit
        # column offsets and the offsets' flag, last in the workspace
        copy = (_align256(8 * m * 4) + _align256(8 * m * 8) + _align256((m + 511) // 512 * 4)
                + _align256(8 * m * 2) + _align256(4))
        base = full - copy
        print(f"[gpu] workspace {p.name} {variant} panel={panel}: full {full} base {base}",
              flush=True)
        ref_out = amgs.qr_csr(rp, ci, va, Z, variant=variant, panel=panel, return_p=True)
        small = torch.empty(base, dtype=torch.uint8, device=DEV)
        out = amgs.qr_csr(rp, ci, va, Z, variant=variant, panel=panel, return_p=True, work=small)
        torch.cuda.synchronize()
        assert int(out.info.item()) == 0
        assert torch.equal(out.Q, ref_out.Q) and torch.equal(out.R, ref_out.R)
        assert torch.equal(out.P, ref_out.P)
        too_small = torch.empty(base - 1, dtype=torch.uint8, device=DEV)
        with pytest.raises(amgs.AmgsError):
            amgs.qr_csr(rp, ci, va, Z, variant=variant, panel=panel, return_p=True,
                        work=too_small)


def test_size_limits():
    """Row counts beyond int32, and entry counts within 1024 of 2^31 (the
    kernels step entry positions up to 512 past a row's end in int32), are
    rejected before any memory is touched."""
    h = amgs.handle(0)
    info = torch.zeros(1, dtype=torch.int32, device=DEV)
    Z = torch.zeros(16, dtype=torch.float64, device=DEV)
    big = (1 << 31) + 1
    ptr = Z.data_ptr()
    st = amgs.amgs_qr_csr(h, big, 10, ptr, ptr, ptr, 4, ptr, big, ptr, big, ptr, 4, None, 0,
                          1, 0, None, ptr, 1 << 20, info.data_ptr(), None)
    assert st == -1
    for nnz in (big, (1 << 31) - 1, (1 << 31) - 1024):
        st = amgs.amgs_qr_csr(h, 100, nnz, ptr, ptr, ptr, 4, ptr, 100, ptr, 100, ptr, 4, None, 0,
                              1, 0, None, ptr, 1 << 20, info.data_ptr(), None)
        assert st == -1, nnz


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("variant", VARIANTS)
def test_second_pass_many_workgroups(variant, precision):
    """The second pass on a problem large enough that its kernels run
    hundreds of workgroups per grid row and several grid rows of
    coefficient groups (m = 64000, n = 40): parity with the oracle and
    bit-identical repeated runs (a read/write race between workgroups would
    show in either)."""
    p = inputs.laplacian_graded_problem(N=40, n=40, decades=2.0, seed=14)
    if precision == "fp32":
        p = inputs.Problem(p.name, np.asfortranarray(p.Z.astype(np.float32).astype(np.float64)),
                           csr=inputs.CSR(p.m, p.csr.row_ptr, p.csr.col_idx,
                                          p.csr.vals.astype(np.float32).astype(np.float64)))
    want = ref.qr_problem(p, variant=variant, reorth=True, precision=precision)
    Q, R, P, info, _ = gpu_run(p, variant, precision=precision, reorth=True)
    Q2, R2, _, _, _ = gpu_run(p, variant, precision=precision, reorth=True)
    assert info == 0
    assert np.array_equal(R, R2) and np.array_equal(Q, Q2)
    o_g, o_o = orth(p, Q), orth(p, want.Q)
    if precision == "fp64":
        e = _rel(R, want.R)
        print(f"  R {e:.2e} orth {o_g:.2e} (oracle {o_o:.2e})")
        assert e <= 1e-10
        assert o_g <= max(1e-13, 10 * o_o)
    else:
        kappa = np.linalg.cond(ref.qr_problem(p, variant=variant).R)
        tol = 64 * U32 * kappa * np.sqrt(p.n)
        e = _rel(R, want.R)
        print(f"  R vs fp32 oracle {e:.2e} tol {tol:.2e} orth {o_g:.2e} (oracle {o_o:.2e})")
        assert e <= tol
        assert o_g <= max(10 * o_o, 1e-6)


@pytest.mark.parametrize("panel", [0, 4])
@pytest.mark.parametrize("form", ["fp64_reorth", "fp32", "fp32_reorth"])
def test_edge_shapes_other_forms(form, panel):
    """The edge shapes (n = 1, a one-column last panel, square m = n, m
    below one wave) in the binary32 form and with the second pass, in both
    schedules, dense and CSR, against the oracle in the matching
    orientation and precision."""
    precision = "fp32" if form.startswith("fp32") else "fp64"
    reorth = form.endswith("reorth")
    orient = "panel" if panel else "col"
    g = inputs.rng(17)
    for m, n in ((700, 1), (300, 5), (40, 40), (5, 3)):
        A = inputs.gram_spd(g, m)
        Z = np.asfortranarray(g.standard_normal((m, n)))
        if precision == "fp32":
            A = np.asfortranarray(A.astype(np.float32).astype(np.float64))
            Z = np.asfortranarray(Z.astype(np.float32).astype(np.float64))
        for prob in (inputs.Problem(f"edge{m}x{n}", Z, dense=A),
                     inputs.Problem(f"edgecsr{m}x{n}", Z, csr=inputs.csr_from_dense(A))):
            for v in VARIANTS:
                want = ref.qr_problem(prob, variant=v, orientation=orient, precision=precision,
                                      reorth=reorth)
                Q, R, P, info, _ = gpu_run(prob, v, precision=precision, reorth=reorth,
                                           panel=panel)
                assert info == 0 and want.info == 0
                if precision == "fp64":
                    assert _rel(R, want.R) <= 1e-10, (prob.name, v, _rel(R, want.R))
                    assert _rel(Q, want.Q) <= 1e-10, (prob.name, v, _rel(Q, want.Q))
                else:
                    kappa = np.linalg.cond(want.R)
                    tol = 64 * U32 * kappa * np.sqrt(n)
                    assert _rel(R, want.R) <= tol, (prob.name, v, _rel(R, want.R), tol)
                    assert orth(prob, Q) <= max(10 * orth(prob, want.Q), 1e-6), (prob.name, v)


def test_binding_rejects_bad_buffers_before_launch():
    """Output buffers of the wrong dtype, shape or layout would be written past
    their end by the kernels; the binding refuses them before any launch."""
    p = SMALL[0]
    m, n = p.Z.shape
    rp = torch.from_numpy(p.csr.row_ptr).to(DEV)
    ci = torch.from_numpy(p.csr.col_idx).to(DEV)
    va = torch.from_numpy(p.csr.vals).to(DEV)
    Z = torch.from_numpy(np.ascontiguousarray(p.Z)).to(DEV)
    print(f"[gpu] binding checks {p.name}", flush=True)
    cases = (
        (dict(Q=amgs.empty_colmajor(m, n, torch.float32, DEV)), "Q must be torch.float64"),
        (dict(Q=amgs.empty_colmajor(m, n - 1, torch.float64, DEV)), "Q must be"),
        (dict(P=torch.empty(m, n, dtype=torch.float64, device=DEV)), "P must be column-major"),
        (dict(R=amgs.empty_colmajor(n, n, torch.float32, DEV)), "R must be torch.float64"),
        (dict(Q=amgs.empty_colmajor(m, n, torch.float64, DEV), precision="fp32"),
         "Q must be torch.float32"),
        (dict(work=torch.empty(1 << 20, dtype=torch.uint8, device=DEV)[::2]), "contiguous"),
    )
    for kw, msg in cases:
        with pytest.raises(ValueError, match=msg):
            amgs.qr_csr(rp, ci, va, Z, variant="ha", **kw)
    with pytest.raises(ValueError, match="Q must be"):
        amgs.qr_dense(torch.eye(m, dtype=torch.float64, device=DEV), Z, variant="hp",
                      Q=amgs.empty_colmajor(m + 1, n, torch.float64, DEV))
    torch.cuda.synchronize()


@pytest.mark.parametrize("panel", [0, 8])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("variant", ["naive", "ha"])
def test_padded_copy_wide_and_narrow_offsets(variant, precision, panel):
    """The short-row MV reads the padded copy's 16-bit column offsets when
    every |col - row| fits, else the 32-bit columns.  A random sparse matrix
    with m = 70001 has offsets far beyond 32767 (32-bit path); the graded
    Laplacian 20^3 has offsets of at most 400 (16-bit path).  Both against
    the column algorithm of the oracle: R, Q and P within 1e-10 in binary64,
    orthogonality within 10x the oracle's binary32 emulation in binary32."""
    probs = (inputs.random_csr_problem(70001, 8, 5, seed=21),
             inputs.laplacian_graded_problem(N=20, n=12, decades=2.0, seed=22))
    for p in probs:
        offs = np.abs(p.csr.col_idx.astype(np.int64)
                      - np.repeat(np.arange(p.m), np.diff(p.csr.row_ptr)))
        print(f"  {p.name}: largest |col - row| {offs.max()}")
        Q, R, P, info, st = gpu_run(p, variant, precision=precision, panel=panel)
        want = ref.qr_problem(p if precision == "fp64" else _as32(p), variant=variant,
                              precision=precision)
        assert info == 0 and want.info == 0
        if precision == "fp64":
            for got, ref_, what in ((R, want.R, "R"), (Q, want.Q, "Q"), (P, want.P, "P")):
                assert _rel(got, ref_) <= 1e-10, (p.name, what, _rel(got, ref_))
        else:
            o_g, o_o = orth(p, Q), orth(p, want.Q)
            print(f"  orth {o_g:.2e} (oracle {o_o:.2e})")
            assert o_g <= max(10 * o_o, 1e-6)


def _as32(p):
    """The problem with its data rounded to binary32 (the binary32 form's input)."""
    return inputs.Problem(p.name + "_f32", np.asfortranarray(p.Z.astype(np.float32).astype(np.float64)),
                          csr=inputs.CSR(p.m, p.csr.row_ptr, p.csr.col_idx,
                                         p.csr.vals.astype(np.float32).astype(np.float64)))
