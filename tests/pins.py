"""Checks that pin the CPU oracle to facts other than itself.

Each check takes the oracle's ctypes library (so the mutation tests can run
the same checks against deliberately broken builds of the oracle) and
returns a list of failure messages (empty = pass).  The facts come from the
paper and from mathematics:

* eq. (1): Z = QR, Q^T A Q = I  =>  Z^T A Z = R^T R, so R is the unique
  Cholesky factor of Z^T A Z (positive diagonal) and Q = Z R^{-1};
* for A = I the problem is the ordinary thin QR (Section 1), so LAPACK's
  Householder QR gives Q and R up to column signs;
* for A = L L^T, Q^T A Q = I  <=>  (L^T Q)^T (L^T Q) = I, so the QR of L^T Z
  gives R (sign-normalised);
* a hand-derived exact example (tests/golden/hand_example.txt);
* Section 2.1: column and row orientations perform the same operations and
  give identical numbers;
* Section 2: naive needs 2n MV, HA n MV, HP one block product A Z;
* Section 3 (eq. (11)): the representation error is O(u) for every variant;
* power-of-two scalings commute with rounding.
"""
from __future__ import annotations

import math

import numpy as np

from oracle import ref
from paper_1703_10440_amd import inputs

VARIANTS = ("naive", "ha", "hp")
ORIENTS = ("col", "row")


def _chol_R(Z, Adense):
    G = Z.T @ Adense @ Z
    return np.linalg.cholesky(0.5 * (G + G.T)).T


def _rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def pin_hand_example(lib, golden) -> list:
    fails = []
    A, Z = golden["A"], golden["Z"]
    csr = inputs.csr_from_dense(A)
    for v in VARIANTS:
        for o in ORIENTS + ("panel", "panel8", "panel16", "cgs"):
            for prec in ("fp64", "fp32"):
                for re_ in ((False, True) if o not in ("panel", "panel8", "panel16") else (False,)):
                    for kind in ("dense", "csr"):
                        kw = dict(dense=A) if kind == "dense" else dict(csr=csr)
                        r = ref.qr(Z, variant=v, orientation=o, reorth=re_, precision=prec,
                                   lib=lib, **kw)
                        tag = f"{v}/{o}/{prec}/reorth={re_}/{kind}"
                        if r.info != 0:
                            fails.append(f"hand {tag}: info {r.info}")
                            continue
                        for name, got in (("R", r.R), ("Q", r.Q), ("P", r.P)):
                            if not np.array_equal(got, golden[name]):
                                fails.append(f"hand {tag}: {name} {got.tolist()}")
    return fails


def pin_cholesky(lib, seeds=(11, 12)) -> list:
    """R equals chol(Z^T A Z) on well-conditioned dense and CSR problems."""
    fails = []
    for seed in seeds:
        probs = [inputs.random_dense_problem(60, 9, seed),
                 inputs.random_csr_problem(300, 12, 9, seed)]
        for p in probs:
            Ad = p.dense if p.dense is not None else p.csr.to_dense()
            Rc = _chol_R(p.Z, Ad)
            for v in VARIANTS:
                for o in ORIENTS:
                    for re_ in (False, True):
                        r = ref.qr(p.Z, dense=p.dense, csr=p.csr, variant=v, orientation=o,
                                   reorth=re_, lib=lib)
                        e = _rel(np.triu(r.R), Rc)
                        if r.info != 0 or not e <= 1e-13:
                            fails.append(f"chol {p.name} {v}/{o}/reorth={re_}: rel {e} info {r.info}")
                        # Q = Z R^{-1}
                        eq = _rel(r.Q, np.linalg.solve(Rc.T, p.Z.T).T)
                        if not eq <= 1e-12:
                            fails.append(f"Q=ZR^-1 {p.name} {v}/{o}: rel {eq}")
                        # P = A Q (auxiliary vectors)
                        ep = _rel(r.P, Ad @ r.Q)
                        if not ep <= 1e-12:
                            fails.append(f"P=AQ {p.name} {v}/{o}: rel {ep}")
    return fails


def pin_identity_householder(lib) -> list:
    """A = I: Householder QR (LAPACK via numpy), sign-normalised; the three
    variants coincide bit for bit because p_i = q_i and x_j = z_j exactly."""
    fails = []
    g = inputs.rng(21)
    m, n = 200, 15
    Z = np.asfortranarray(g.standard_normal((m, n)))
    eye = inputs.CSR(m, np.arange(m + 1, dtype=np.int32), np.arange(m, dtype=np.int32),
                     np.ones(m))
    Qh, Rh = np.linalg.qr(Z)
    D = np.sign(np.diag(Rh))
    Qh, Rh = Qh * D[None, :], Rh * D[:, None]
    outs = {}
    for v in VARIANTS:
        r = ref.qr(Z, csr=eye, variant=v, lib=lib)
        outs[v] = r
        if _rel(np.triu(r.R), Rh) > 1e-14 or _rel(r.Q, Qh) > 1e-13:
            fails.append(f"identity {v}: R {_rel(np.triu(r.R), Rh)} Q {_rel(r.Q, Qh)}")
    for v in ("ha", "hp"):
        if not (np.array_equal(outs[v].R, outs["naive"].R)
                and np.array_equal(outs[v].Q, outs["naive"].Q)):
            fails.append(f"identity: {v} differs bitwise from naive")
    return fails


def pin_cholesky_factor(lib) -> list:
    """A = L L^T: R = R_qr(L^T Z) (sign-normalised) and Q = L^{-T} Q_qr."""
    fails = []
    g = inputs.rng(31)
    m, n = 80, 10
    L = np.tril(g.standard_normal((m, m))) * 0.1 + np.diag(1.0 + g.random(m))
    A = np.asfortranarray(L @ L.T)
    A = 0.5 * (A + A.T)
    Z = np.asfortranarray(g.standard_normal((m, n)))
    Qh, Rh = np.linalg.qr(L.T @ Z)
    D = np.sign(np.diag(Rh))
    Qh, Rh = Qh * D[None, :], Rh * D[:, None]
    Qexp = np.linalg.solve(L.T, Qh)
    for v in VARIANTS:
        for o in ORIENTS:
            r = ref.qr(Z, dense=A, variant=v, orientation=o, lib=lib)
            e1, e2 = _rel(np.triu(r.R), Rh), _rel(r.Q, Qexp)
            if e1 > 1e-12 or e2 > 1e-11:
                fails.append(f"LL^T {v}/{o}: R {e1} Q {e2}")
    return fails


def pin_col_row_bitwise(lib) -> list:
    """Section 2.1: column and row versions give exactly the same numbers."""
    fails = []
    p = inputs.random_csr_problem(500, 10, 7, 41, decades=5.0)
    d = inputs.random_dense_problem(90, 8, 42, decades=3.0)
    for prob in (p, d):
        for v in VARIANTS:
            for prec in ("fp64", "fp32"):
                for re_ in (False, True):
                    a = ref.qr(prob.Z, dense=prob.dense, csr=prob.csr, variant=v,
                               orientation="col", reorth=re_, precision=prec, lib=lib)
                    b = ref.qr(prob.Z, dense=prob.dense, csr=prob.csr, variant=v,
                               orientation="row", reorth=re_, precision=prec, lib=lib)
                    if not (np.array_equal(a.R, b.R) and np.array_equal(a.Q, b.Q)
                            and np.array_equal(a.P, b.P)):
                        fails.append(f"col!=row {prob.name} {v} {prec} reorth={re_}")
    return fails


def pin_mv_counts(lib) -> list:
    """naive: 2n MV; HA: n MV; HP: one block product over n columns."""
    fails = []
    p = inputs.random_csr_problem(100, 7, 5, 51)
    exp = {"naive": (14, 14), "ha": (7, 7), "hp": (1, 7)}
    for v in VARIANTS:
        for o in ORIENTS:
            r = ref.qr_problem(p, variant=v, orientation=o, lib=lib)
            if (r.mv_calls, r.mv_cols) != exp[v]:
                fails.append(f"mv count {v}/{o}: {(r.mv_calls, r.mv_cols)}")
    return fails


def pin_scaling(lib) -> list:
    """A -> 4A gives R -> 2R, Q -> Q/2; Z -> 2Z gives R -> 2R, Q unchanged;
    exactly, because power-of-two scalings commute with rounding."""
    fails = []
    p = inputs.random_dense_problem(70, 9, 61, decades=2.0)
    for v in VARIANTS:
        for prec in ("fp64", "fp32"):
            base = ref.qr(p.Z, dense=p.dense, variant=v, precision=prec, lib=lib)
            a4 = ref.qr(p.Z, dense=4.0 * p.dense, variant=v, precision=prec, lib=lib)
            z2 = ref.qr(2.0 * p.Z, dense=p.dense, variant=v, precision=prec, lib=lib)
            if not (np.array_equal(a4.R, 2 * base.R) and np.array_equal(a4.Q, base.Q / 2)):
                fails.append(f"scale A {v} {prec}")
            if not (np.array_equal(z2.R, 2 * base.R) and np.array_equal(z2.Q, base.Q)):
                fails.append(f"scale Z {v} {prec}")
    return fails


def pin_first_column(lib) -> list:
    """Column 1 (r_11, q_1) is computed identically by every variant."""
    fails = []
    p = inputs.random_csr_problem(400, 6, 9, 71)
    outs = [ref.qr_problem(p, variant=v, lib=lib) for v in VARIANTS]
    for o in outs[1:]:
        if o.R[0, 0] != outs[0].R[0, 0] or not np.array_equal(o.Q[:, 0], outs[0].Q[:, 0]):
            fails.append("first column differs between variants")
    return fails


def pin_residual_and_reorth(lib) -> list:
    """Eq. (11): ||Z - QR|| = O(u) for all variants even when Z is badly
    conditioned; with the second pass the A-orthogonality improves and the
    residual stays O(u) (the pass must add s_i into R)."""
    fails = []
    p = inputs.random_csr_problem(2000, 16, 7, 81, decades=12.0)
    for v in VARIANTS:
        r0 = ref.qr_problem(p, variant=v, lib=lib)
        r1 = ref.qr_problem(p, variant=v, reorth=True, lib=lib)
        for tag, r in (("plain", r0), ("reorth", r1)):
            res = ref.residual(p.Z, r.Q, r.R)
            if r.info != 0 or not res < 1e-14:
                fails.append(f"residual {v} {tag}: {res} info {r.info}")
        o0, o1 = ref.orth_loss(r0.Q, csr=p.csr), ref.orth_loss(r1.Q, csr=p.csr)
        # naive and HA hold P = AQ to O(u), so a second pass restores
        # A-orthogonality to O(u).  HP's P comes from the recurrence of
        # eq. (5), which cancels when Z is ill-conditioned; the pass then
        # only reduces the loss.
        limit = 1e-13 if v != "hp" else 0.1 * o0
        if not (o1 < limit and o1 < o0):
            fails.append(f"reorth orthogonality {v}: {o0} -> {o1}")
    # An ill-conditioned A (experiment II, case 2) makes the first pass lose
    # A-orthogonality while z_j^{(j-1)} stays comparable to z_j^{(0)}: the
    # second-pass coefficients are then large enough that Z = QR needs them.
    q = inputs.exp2_problem(100, 20, 1e10, 1e3, 2, 7)
    for v in VARIANTS:
        r1 = ref.qr_problem(q, variant=v, reorth=True, lib=lib)
        res = ref.residual(q.Z, r1.Q, r1.R)
        if r1.info != 0 or not res < 1e-14:
            fails.append(f"residual exp2 reorth {v}: {res}")
    return fails


def _kappa(M):
    s = np.linalg.svd(M, compute_uv=False)
    return float(s[0] / s[-1])


def pin_exp2_accuracy(lib) -> list:
    """Experiment II/III (Section 4): the loss of A-orthogonality of all three
    variants stays below a small multiple of delta_1 = u kappa(A)
    kappa(A^{1/2} Z); in case 2 with A and Z both ill-conditioned HA is far
    more accurate than naive, and HP tracks naive."""
    fails = []
    u = 2.0 ** -53
    for ka, kz in ((1e4, 1e4), (1e8, 1e6), (1e6, 1e8)):
        p = inputs.exp2_problem(100, 20, ka, kz, 2, 3)
        w, V = np.linalg.eigh(p.dense)
        kA = float(w[-1] / w[0])
        kAZ = _kappa((V * np.sqrt(w)[None, :]) @ V.T @ p.Z)
        d1 = u * kA * kAZ
        loss = {}
        for v in VARIANTS:
            r = ref.qr_problem(p, variant=v, lib=lib)
            loss[v] = ref.orth_loss(r.Q, dense=p.dense)
            if r.info != 0 or not loss[v] <= 10 * d1:
                fails.append(f"exp2 {ka:g},{kz:g} {v}: loss {loss[v]} > 10 delta1 {d1}")
        if ka >= 1e8 and not loss["ha"] < 1e-2 * loss["naive"]:
            fails.append(f"exp2 {ka:g},{kz:g}: HA {loss['ha']} not << naive {loss['naive']}")
        if not loss["hp"] < 100 * loss["naive"] + 1e-14:
            fails.append(f"exp2 {ka:g},{kz:g}: HP {loss['hp']} far above naive {loss['naive']}")
    return fails


def pin_fp32_accumulation(lib) -> list:
    """FP32-storage form: r_ij accumulates in binary32 while the squared
    A-norm accumulates in binary64 (values worked out by hand).

    Norm: A = I, z = (1 + 2^-12) * ones(4096).  Each z_k^2 = 1 + 2^-11 + 2^-24 is
    exact in binary64, so z^T z = 4098 + 2^-12 exactly and r_11 must be the
    correctly rounded sqrt of that; in binary32 the 2^-24 terms would vanish.
    Projection: A = I, z_1 = (1,1,1,1) so p_1 = q_1 = (1/2,...);
    z_2 = (2, 2^-23, 2^-23, 0) gives products (1, 2^-24, 2^-24, 0), whose
    left-to-right binary32 sum rounds (ties to even) to exactly 1, while the
    binary64 sum is 1 + 2^-23.
    """
    fails = []
    m = 4096
    eye = inputs.CSR(m, np.arange(m + 1, dtype=np.int32), np.arange(m, dtype=np.int32),
                     np.ones(m))
    z = np.full((m, 1), 1.0 + 2.0 ** -12, order="F")
    for v in VARIANTS:
        r = ref.qr(z, csr=eye, variant=v, precision="fp32", lib=lib)
        want = math.sqrt(4098.0 + 2.0 ** -12)
        if r.R[0, 0] != want:
            fails.append(f"fp32 norm {v}: {r.R[0, 0]!r} != {want!r}")
        qv = float(np.float32((1.0 + 2.0 ** -12) / want))
        if not np.all(r.Q[:, 0] == qv):
            fails.append(f"fp32 q rounding {v}")
    eye4 = inputs.CSR(4, np.arange(5, dtype=np.int32), np.arange(4, dtype=np.int32), np.ones(4))
    Z = np.asfortranarray(np.array([[1, 2], [1, 2.0 ** -23], [1, 2.0 ** -23], [1, 0]], float))
    for v in VARIANTS:
        r32 = ref.qr(Z, csr=eye4, variant=v, precision="fp32", lib=lib)
        r64 = ref.qr(Z, csr=eye4, variant=v, precision="fp64", lib=lib)
        if r32.R[0, 1] != 1.0 or r64.R[0, 1] != 1.0 + 2.0 ** -23:
            fails.append(f"fp32 dot accumulation {v}: {r32.R[0, 1]!r} {r64.R[0, 1]!r}")
    return fails


def pin_fp32_mv_axpy_rounding(lib) -> list:
    """Binary32 form: the MV sums each row left to right in binary32, and the
    projection update z -= r q rounds the product and then the difference to
    binary32 (two roundings).  Both worked out by hand on exact values.

    MV: A = [[1, e, e], [e, 1, 0], [e, 0, 1]] with e = 2^-24 (spd, values
    exact in binary32), z = (1, 1, 1), n = 1.  Row 0 in stored order:
    1 + 2^-24 is a tie and rounds to 1 (even), and again for the second e,
    so x_0 = 1; rows 1 and 2 give 1 + 2^-24 -> 1.  Hence z^T x = 3 exactly
    and r_11 = sqrt(3).  A row sum accumulated in binary64 and rounded once
    gives x_0 = 1 + 2^-23 and r_11 = sqrt(3 + 2^-23); summed from the right,
    e + e = 2^-23 and x_0 = 1 + 2^-23 as well.

    AXPY: A = I_2, z_1 = (3, 4), z_2 = (1, -27).  r_11 = 5, q_1 = p_1 =
    (fl(3/5), fl(4/5)) = (10066330, 13421773) 2^-24.  r_12 = p_1^T z_2 in
    binary32: fl(13421773 * 2^-24 * -27) = -11324621 * 2^-19, and
    10066330 * 2^-24 - 11324621 * 2^-19 = -352321542 * 2^-24 rounds to -21
    exactly.  Second entry of z_2 - r_12 q_1: the product 21 q_12 =
    281857233 * 2^-24 rounds to 8808039 * 2^-19, and -27 + 8808039 * 2^-19 =
    -10695474 * 2^-20 is exact; one binary64 rounding of -27 + 21 q_12 =
    -171127599 * 2^-24 would instead give -10695475 * 2^-20.  The first entry,
    1 + 21 q_11 -> 1 + 13212058 * 2^-20 = 14260634 * 2^-20, is the same either
    way.  Then r_22 = sqrt(z'^T z') in binary64 and q_2 = z' / r_22 rounded
    to binary32; every variant agrees (A = I)."""
    fails = []
    e = 2.0 ** -24
    A = np.asfortranarray(np.array([[1, e, e], [e, 1, 0], [e, 0, 1]], float))
    z = np.asfortranarray(np.ones((3, 1)))
    want = math.sqrt(3.0)
    for v in VARIANTS:
        for kind, kw in (("csr", dict(csr=inputs.csr_from_dense(A))), ("dense", dict(dense=A))):
            r = ref.qr(z, variant=v, precision="fp32", lib=lib, **kw)
            if r.info != 0 or r.R[0, 0] != want:
                fails.append(f"fp32 MV row sum {v}/{kind}: r_11 {r.R[0, 0]!r} != sqrt(3)")
            qv = float(np.float32(1.0 / want))
            if not np.all(r.Q[:, 0] == qv):
                fails.append(f"fp32 MV row sum {v}/{kind}: q_1 {r.Q[:, 0].tolist()}")
    I2 = np.asfortranarray(np.eye(2))
    Z = np.asfortranarray(np.array([[3.0, 1.0], [4.0, -27.0]]))
    zp = np.array([14260634 * 2.0 ** -20, -10695474 * 2.0 ** -20])
    r22 = math.sqrt(zp[0] * zp[0] + zp[1] * zp[1])
    q2 = np.array([float(np.float32(zp[k] / r22)) for k in range(2)])
    for v in VARIANTS:
        for kind, kw in (("csr", dict(csr=inputs.csr_from_dense(I2))), ("dense", dict(dense=I2))):
            for o in ORIENTS:
                r = ref.qr(Z, variant=v, orientation=o, precision="fp32", lib=lib, **kw)
                tag = f"{v}/{kind}/{o}"
                if r.info != 0 or r.R[0, 0] != 5.0 or r.R[0, 1] != -21.0:
                    fails.append(f"fp32 axpy {tag}: R[0, :] {r.R[0].tolist()}")
                if r.R[1, 1] != r22:
                    fails.append(f"fp32 axpy {tag}: r_22 {r.R[1, 1]!r} != {r22!r}")
                if not np.array_equal(r.Q[:, 1], q2):
                    fails.append(f"fp32 axpy {tag}: q_2 {r.Q[:, 1].tolist()} != {q2.tolist()}")
    return fails


def pin_fp32_vs_fp64(lib) -> list:
    """The binary32 form agrees with binary64 to the accuracy binary32 allows
    on a well-conditioned problem (inputs rounded to binary32 first)."""
    fails = []
    p = inputs.random_csr_problem(3000, 12, 7, 91)
    csr32 = inputs.CSR(p.m, p.csr.row_ptr, p.csr.col_idx,
                       p.csr.vals.astype(np.float32).astype(np.float64))
    Z32 = np.asfortranarray(p.Z.astype(np.float32).astype(np.float64))
    for v in VARIANTS:
        a = ref.qr(Z32, csr=csr32, variant=v, precision="fp32", lib=lib)
        b = ref.qr(Z32, csr=csr32, variant=v, precision="fp64", lib=lib)
        e = _rel(a.R, b.R)
        if not (1e-9 < e < 1e-5):
            fails.append(f"fp32 vs fp64 {v}: {e}")
    return fails


def pin_breakdown(lib) -> list:
    """Breakdown convention: the 1-based index of the first column whose
    squared A-norm is not positive and finite."""
    fails = []
    g = inputs.rng(101)
    m, n = 50, 5
    Z = np.asfortranarray(g.standard_normal((m, n)))
    A = inputs.gram_spd(g, m)
    Zc = Z.copy(order="F")
    Zc[:, 2] = 0.0
    for v in VARIANTS:
        if ref.qr(Zc, dense=A, variant=v, lib=lib).info != 3:
            fails.append(f"zero column {v}")
        if ref.qr(Z, dense=-A, variant=v, lib=lib).info != 1:
            fails.append(f"negative definite {v}")
        Zn = Z.copy(order="F")
        Zn[7, 3] = np.nan
        if ref.qr(Zn, dense=A, variant=v, lib=lib).info != 4:
            fails.append(f"nan column {v}")
    return fails


def pin_panel(lib) -> list:
    """Panel schedule (orientation "panel", panels of 4 columns): the
    regrouped projections give, in exact arithmetic, the column algorithm's
    coefficients, so the same facts hold -- R = chol(Z^T A Z), Q = Z R^{-1},
    P = AQ on well-conditioned problems with several panels and a ragged last
    panel; Householder QR for A = I with the three variants equal bit for
    bit; the hand example exactly; one panel (n <= 4) is the column
    algorithm bit for bit; MV counts 2n / n / one block; and on an
    experiment-II problem (case 2, kappa(A) = kappa(Z) = 1e8) the loss of
    A-orthogonality stays within a small factor of the column algorithm's
    and below 10 delta_1 (a block step without the triangular correction
    loses orders of magnitude there)."""
    fails = []
    for seed in (11, 12):
        for p in (inputs.random_dense_problem(60, 9, seed), inputs.random_csr_problem(300, 14, 9, seed)):
            Ad = p.dense if p.dense is not None else p.csr.to_dense()
            Rc = _chol_R(p.Z, Ad)
            for v in VARIANTS:
                r = ref.qr(p.Z, dense=p.dense, csr=p.csr, variant=v, orientation="panel", lib=lib)
                e, eq, ep = (_rel(np.triu(r.R), Rc), _rel(r.Q, np.linalg.solve(Rc.T, p.Z.T).T),
                             _rel(r.P, Ad @ r.Q))
                if r.info != 0 or not (e <= 1e-13 and eq <= 1e-12 and ep <= 1e-12):
                    fails.append(f"panel chol {p.name} {v}: R {e} Q {eq} P {ep} info {r.info}")
                want_calls = {"naive": 2 * p.n, "ha": p.n, "hp": 1}[v]
                if r.mv_calls != want_calls:
                    fails.append(f"panel MV count {p.name} {v}: {r.mv_calls} != {want_calls}")
    g = inputs.rng(22)
    m, n = 150, 11
    Z = np.asfortranarray(g.standard_normal((m, n)))
    eye = inputs.CSR(m, np.arange(m + 1, dtype=np.int32), np.arange(m, dtype=np.int32), np.ones(m))
    Qh, Rh = np.linalg.qr(Z)
    D = np.sign(np.diag(Rh))
    Qh, Rh = Qh * D[None, :], Rh * D[:, None]
    outs = {v: ref.qr(Z, csr=eye, variant=v, orientation="panel", lib=lib) for v in VARIANTS}
    for v, r in outs.items():
        if _rel(np.triu(r.R), Rh) > 1e-14 or _rel(r.Q, Qh) > 1e-13:
            fails.append(f"panel identity {v}: R {_rel(np.triu(r.R), Rh)} Q {_rel(r.Q, Qh)}")
        if not (np.array_equal(r.R, outs["naive"].R) and np.array_equal(r.Q, outs["naive"].Q)):
            fails.append(f"panel identity: {v} differs bitwise from naive")
    p = inputs.random_dense_problem(40, 4, 5)
    for v in VARIANTS:
        a = ref.qr(p.Z, dense=p.dense, variant=v, lib=lib)
        b = ref.qr(p.Z, dense=p.dense, variant=v, orientation="panel", lib=lib)
        if not (np.array_equal(a.R, b.R) and np.array_equal(a.Q, b.Q)):
            fails.append(f"panel single panel {v}: differs from the column algorithm")
    u = 2.0 ** -53
    p = inputs.exp2_problem(100, 20, 1e8, 1e8, 2, 7)
    w, V = np.linalg.eigh(p.dense)
    d1 = u * float(w[-1] / w[0]) * _kappa((V * np.sqrt(w)[None, :]) @ V.T @ p.Z)
    for v in ("naive", "ha"):
        lc = ref.orth_loss(ref.qr_problem(p, variant=v, lib=lib).Q, dense=p.dense)
        r = ref.qr_problem(p, variant=v, orientation="panel", lib=lib)
        lp = ref.orth_loss(r.Q, dense=p.dense)
        if r.info != 0 or not (lp <= 30 * lc and lp <= 10 * d1):
            fails.append(f"panel exp2 {v}: loss {lp} (column {lc}, 10 delta1 {10 * d1})")
    # with the second pass: the closed forms, one panel equal to the column
    # form bit for bit, and the pass restoring orthogonality in the binary32
    # form on an ill-conditioned problem
    for p in (inputs.random_dense_problem(60, 9, 13), inputs.random_csr_problem(300, 14, 9, 13)):
        Ad = p.dense if p.dense is not None else p.csr.to_dense()
        Rc = _chol_R(p.Z, Ad)
        for v in VARIANTS:
            r = ref.qr(p.Z, dense=p.dense, csr=p.csr, variant=v, orientation="panel", reorth=True,
                       lib=lib)
            e, eq = _rel(np.triu(r.R), Rc), _rel(r.Q, np.linalg.solve(Rc.T, p.Z.T).T)
            if r.info != 0 or not (e <= 1e-13 and eq <= 1e-12):
                fails.append(f"panel reorth chol {p.name} {v}: R {e} Q {eq} info {r.info}")
    p = inputs.random_dense_problem(40, 4, 5)
    for v in VARIANTS:
        a = ref.qr(p.Z, dense=p.dense, variant=v, reorth=True, lib=lib)
        b = ref.qr(p.Z, dense=p.dense, variant=v, orientation="panel", reorth=True, lib=lib)
        if not (np.array_equal(a.R, b.R) and np.array_equal(a.Q, b.Q)):
            fails.append(f"panel reorth single panel {v}: differs from the column algorithm")
    q = inputs.laplacian_graded_problem(N=10, n=12, decades=4.0, seed=3)
    for v in ("naive", "ha"):
        o0 = ref.orth_loss(ref.qr_problem(q, variant=v, orientation="panel", precision="fp32",
                                          lib=lib).Q, csr=q.csr)
        o1 = ref.orth_loss(ref.qr_problem(q, variant=v, orientation="panel", precision="fp32",
                                          reorth=True, lib=lib).Q, csr=q.csr)
        if not o1 < 1e-2 * o0:
            fails.append(f"panel reorth binary32 orthogonality {v}: {o0} -> {o1}")
    return fails


def pin_panel8(lib) -> list:
    """Two-level panel schedule (orientation "panel8": panels of 8 columns,
    each taken apart as two panels of 4).  Every regrouping gives the column
    algorithm's coefficients in exact arithmetic, so: R = chol(Z^T A Z),
    Q = Z R^{-1}, P = AQ on well-conditioned problems spanning several
    8-panels with ragged last 8- and 4-panels (n = 21 = 8 + 8 + 4 + 1), with
    and without the second pass; Householder QR for A = I with the three
    variants equal bit for bit; MV counts 2n / n / one block; with n <= 8 it
    is the one-level panel orientation bit for bit (a single 8-panel is two
    4-panels); with n > 8 it is not (the 8-panel blocks are in use) yet agrees
    to rounding level; on an experiment-II problem (case 2, kappa(A) =
    kappa(Z) = 1e8) the loss stays within a small factor of the column
    algorithm's and below 10 delta_1; and the second pass restores
    orthogonality in the binary32 form."""
    fails = []
    for seed in (31, 32):
        for p in (inputs.random_dense_problem(60, 21, seed), inputs.random_csr_problem(300, 21, 9, seed)):
            Ad = p.dense if p.dense is not None else p.csr.to_dense()
            Rc = _chol_R(p.Z, Ad)
            for v in VARIANTS:
                for re_ in (False, True):
                    r = ref.qr(p.Z, dense=p.dense, csr=p.csr, variant=v, orientation="panel8",
                               reorth=re_, lib=lib)
                    e, eq, ep = (_rel(np.triu(r.R), Rc), _rel(r.Q, np.linalg.solve(Rc.T, p.Z.T).T),
                                 _rel(r.P, Ad @ r.Q))
                    if r.info != 0 or not (e <= 1e-13 and eq <= 1e-12 and ep <= 1e-12):
                        fails.append(f"panel8 chol {p.name} {v} reorth={re_}: R {e} Q {eq} P {ep} "
                                     f"info {r.info}")
                    want_calls = {"naive": 2 * p.n, "ha": p.n, "hp": 1}[v]
                    if r.mv_calls != want_calls:
                        fails.append(f"panel8 MV count {p.name} {v}: {r.mv_calls} != {want_calls}")
                r1 = ref.qr(p.Z, dense=p.dense, csr=p.csr, variant=v, orientation="panel", lib=lib)
                r2 = ref.qr(p.Z, dense=p.dense, csr=p.csr, variant=v, orientation="panel8", lib=lib)
                if np.array_equal(r1.R, r2.R):
                    fails.append(f"panel8 {p.name} {v}: identical to the one-level form at n = 21")
                if _rel(np.triu(r2.R), np.triu(r1.R)) > 1e-13:
                    fails.append(f"panel8 {p.name} {v}: R differs from the one-level form by "
                                 f"{_rel(np.triu(r2.R), np.triu(r1.R))}")
    g = inputs.rng(23)
    m, n = 150, 19
    Z = np.asfortranarray(g.standard_normal((m, n)))
    eye = inputs.CSR(m, np.arange(m + 1, dtype=np.int32), np.arange(m, dtype=np.int32), np.ones(m))
    Qh, Rh = np.linalg.qr(Z)
    D = np.sign(np.diag(Rh))
    Qh, Rh = Qh * D[None, :], Rh * D[:, None]
    outs = {v: ref.qr(Z, csr=eye, variant=v, orientation="panel8", lib=lib) for v in VARIANTS}
    for v, r in outs.items():
        if _rel(np.triu(r.R), Rh) > 1e-14 or _rel(r.Q, Qh) > 1e-13:
            fails.append(f"panel8 identity {v}: R {_rel(np.triu(r.R), Rh)} Q {_rel(r.Q, Qh)}")
        if not (np.array_equal(r.R, outs["naive"].R) and np.array_equal(r.Q, outs["naive"].Q)):
            fails.append(f"panel8 identity: {v} differs bitwise from naive")
    for nn in (3, 7, 8):
        p = inputs.random_dense_problem(40, nn, 6)
        for v in VARIANTS:
            for re_ in (False, True):
                a = ref.qr(p.Z, dense=p.dense, variant=v, orientation="panel", reorth=re_, lib=lib)
                b = ref.qr(p.Z, dense=p.dense, variant=v, orientation="panel8", reorth=re_, lib=lib)
                if not (np.array_equal(a.R, b.R) and np.array_equal(a.Q, b.Q)
                        and np.array_equal(a.P, b.P)):
                    fails.append(f"panel8 n={nn} {v} reorth={re_}: differs from the one-level form")
    u = 2.0 ** -53
    p = inputs.exp2_problem(100, 20, 1e8, 1e8, 2, 7)
    w, V = np.linalg.eigh(p.dense)
    d1 = u * float(w[-1] / w[0]) * _kappa((V * np.sqrt(w)[None, :]) @ V.T @ p.Z)
    for v in ("naive", "ha"):
        lc = ref.orth_loss(ref.qr_problem(p, variant=v, lib=lib).Q, dense=p.dense)
        r = ref.qr_problem(p, variant=v, orientation="panel8", lib=lib)
        lp = ref.orth_loss(r.Q, dense=p.dense)
        if r.info != 0 or not (lp <= 30 * lc and lp <= 10 * d1):
            fails.append(f"panel8 exp2 {v}: loss {lp} (column {lc}, 10 delta1 {10 * d1})")
    q = inputs.laplacian_graded_problem(N=10, n=20, decades=4.0, seed=3)
    for v in ("naive", "ha"):
        o0 = ref.orth_loss(ref.qr_problem(q, variant=v, orientation="panel8", precision="fp32",
                                          lib=lib).Q, csr=q.csr)
        o1 = ref.orth_loss(ref.qr_problem(q, variant=v, orientation="panel8", precision="fp32",
                                          reorth=True, lib=lib).Q, csr=q.csr)
        if not o1 < 1e-2 * o0:
            fails.append(f"panel8 reorth binary32 orthogonality {v}: {o0} -> {o1}")
    return fails


def pin_panel16(lib) -> list:
    """Three-level panel schedule (orientation "panel16": panels of 16
    columns, each taken apart as two panels of 8, each of those as two of
    4).  As for "panel8": R = chol(Z^T A Z), Q = Z R^{-1}, P = AQ on
    well-conditioned problems spanning several 16-panels with ragged last
    16-, 8- and 4-panels (n = 37 = 16 + 16 + 4 + 1), with and without the
    second pass; Householder QR for A = I, the three variants equal bit for
    bit; MV counts 2n / n / one block; with n <= 16 it is the two-level
    orientation bit for bit (a single 16-panel is two 8-panels); with n > 16
    it is not (the 16-panel blocks are in use) yet agrees to rounding level;
    on the experiment-II problem of pin_panel8 the loss stays within a small
    factor of the column algorithm's and below 10 delta_1."""
    fails = []
    for seed in (41, 42):
        for p in (inputs.random_dense_problem(80, 37, seed), inputs.random_csr_problem(400, 37, 9, seed)):
            Ad = p.dense if p.dense is not None else p.csr.to_dense()
            Rc = _chol_R(p.Z, Ad)
            for v in VARIANTS:
                for re_ in (False, True):
                    r = ref.qr(p.Z, dense=p.dense, csr=p.csr, variant=v, orientation="panel16",
                               reorth=re_, lib=lib)
                    e, eq, ep = (_rel(np.triu(r.R), Rc), _rel(r.Q, np.linalg.solve(Rc.T, p.Z.T).T),
                                 _rel(r.P, Ad @ r.Q))
                    if r.info != 0 or not (e <= 1e-13 and eq <= 1e-12 and ep <= 1e-12):
                        fails.append(f"panel16 chol {p.name} {v} reorth={re_}: R {e} Q {eq} P {ep} "
                                     f"info {r.info}")
                    want_calls = {"naive": 2 * p.n, "ha": p.n, "hp": 1}[v]
                    if r.mv_calls != want_calls:
                        fails.append(f"panel16 MV count {p.name} {v}: {r.mv_calls} != {want_calls}")
                r1 = ref.qr(p.Z, dense=p.dense, csr=p.csr, variant=v, orientation="panel8", lib=lib)
                r2 = ref.qr(p.Z, dense=p.dense, csr=p.csr, variant=v, orientation="panel16", lib=lib)
                if np.array_equal(r1.R, r2.R):
                    fails.append(f"panel16 {p.name} {v}: identical to the two-level form at n = 37")
                if _rel(np.triu(r2.R), np.triu(r1.R)) > 1e-13:
                    fails.append(f"panel16 {p.name} {v}: R differs from the two-level form by "
                                 f"{_rel(np.triu(r2.R), np.triu(r1.R))}")
    g = inputs.rng(24)
    m, n = 150, 35
    Z = np.asfortranarray(g.standard_normal((m, n)))
    eye = inputs.CSR(m, np.arange(m + 1, dtype=np.int32), np.arange(m, dtype=np.int32), np.ones(m))
    Qh, Rh = np.linalg.qr(Z)
    D = np.sign(np.diag(Rh))
    Qh, Rh = Qh * D[None, :], Rh * D[:, None]
    outs = {v: ref.qr(Z, csr=eye, variant=v, orientation="panel16", lib=lib) for v in VARIANTS}
    for v, r in outs.items():
        if _rel(np.triu(r.R), Rh) > 1e-14 or _rel(r.Q, Qh) > 1e-13:
            fails.append(f"panel16 identity {v}: R {_rel(np.triu(r.R), Rh)} Q {_rel(r.Q, Qh)}")
        if not (np.array_equal(r.R, outs["naive"].R) and np.array_equal(r.Q, outs["naive"].Q)):
            fails.append(f"panel16 identity: {v} differs bitwise from naive")
    for nn in (5, 12, 16):
        p = inputs.random_dense_problem(40, nn, 6)
        for v in VARIANTS:
            for re_ in (False, True):
                a = ref.qr(p.Z, dense=p.dense, variant=v, orientation="panel8", reorth=re_, lib=lib)
                b = ref.qr(p.Z, dense=p.dense, variant=v, orientation="panel16", reorth=re_, lib=lib)
                if not (np.array_equal(a.R, b.R) and np.array_equal(a.Q, b.Q)
                        and np.array_equal(a.P, b.P)):
                    fails.append(f"panel16 n={nn} {v} reorth={re_}: differs from the two-level form")
    u = 2.0 ** -53
    p = inputs.exp2_problem(100, 40, 1e8, 1e8, 2, 7)
    w, V = np.linalg.eigh(p.dense)
    d1 = u * float(w[-1] / w[0]) * _kappa((V * np.sqrt(w)[None, :]) @ V.T @ p.Z)
    for v in ("naive", "ha"):
        lc = ref.orth_loss(ref.qr_problem(p, variant=v, lib=lib).Q, dense=p.dense)
        r = ref.qr_problem(p, variant=v, orientation="panel16", lib=lib)
        lp = ref.orth_loss(r.Q, dense=p.dense)
        if r.info != 0 or not (lp <= 30 * lc and lp <= 10 * d1):
            fails.append(f"panel16 exp2 {v}: loss {lp} (column {lc}, 10 delta1 {10 * d1})")
    return fails


def pin_blocked_second_pass(lib) -> list:
    """Blocked second pass (reorth = 2, orientation "panel8"): each outer
    panel's columns get the classical pass against all earlier outer panels
    at once, then the in-panel pass.  Every pass only removes components
    along earlier columns and adds the same coefficients into R, so the
    closed forms hold (n = 21: two full outer panels and a ragged one); with
    n <= 8 there is no earlier outer panel and it is the per-column pass bit
    for bit; on an experiment-II case-2 problem (the first pass loses
    orthogonality, so the pass's coefficients matter) the residual stays at
    rounding level and the loss drops below a tenth of the first pass's, to
    within 10x that of the per-column pass; in the binary32 form it restores
    orthogonality by orders of magnitude."""
    fails = []
    for p in (inputs.random_dense_problem(60, 21, 33), inputs.random_csr_problem(300, 21, 9, 33)):
        Ad = p.dense if p.dense is not None else p.csr.to_dense()
        Rc = _chol_R(p.Z, Ad)
        for v in VARIANTS:
            r = ref.qr(p.Z, dense=p.dense, csr=p.csr, variant=v, orientation="panel8", reorth=2,
                       lib=lib)
            e, eq, ep = (_rel(np.triu(r.R), Rc), _rel(r.Q, np.linalg.solve(Rc.T, p.Z.T).T),
                         _rel(r.P, Ad @ r.Q))
            if r.info != 0 or not (e <= 1e-13 and eq <= 1e-12 and ep <= 1e-12):
                fails.append(f"blocked pass chol {p.name} {v}: R {e} Q {eq} P {ep} info {r.info}")
    for nn in (5, 8):
        p = inputs.random_dense_problem(40, nn, 6)
        for v in VARIANTS:
            a = ref.qr(p.Z, dense=p.dense, variant=v, orientation="panel8", reorth=True, lib=lib)
            b = ref.qr(p.Z, dense=p.dense, variant=v, orientation="panel8", reorth=2, lib=lib)
            if not (np.array_equal(a.R, b.R) and np.array_equal(a.Q, b.Q)):
                fails.append(f"blocked pass n={nn} {v}: differs from the per-column pass")
    p = inputs.exp2_problem(100, 20, 1e8, 1e8, 2, 7)
    for v in ("naive", "ha"):
        r0 = ref.qr_problem(p, variant=v, orientation="panel8", lib=lib)
        r1 = ref.qr_problem(p, variant=v, orientation="panel8", reorth=True, lib=lib)
        r2 = ref.qr_problem(p, variant=v, orientation="panel8", reorth=2, lib=lib)
        res = ref.residual(p.Z, r2.Q, r2.R)
        o0, o1, o2 = (ref.orth_loss(r.Q, dense=p.dense) for r in (r0, r1, r2))
        if r2.info != 0 or res > 1e-14 or not (o2 <= 10 * o1 + 1e-15 and o2 < 0.1 * o0):
            fails.append(f"blocked pass exp2 {v}: residual {res} loss {o2} (per-column {o1}, "
                         f"no pass {o0})")
    q = inputs.laplacian_graded_problem(N=10, n=20, decades=4.0, seed=3)
    for v in ("naive", "ha"):
        o0 = ref.orth_loss(ref.qr_problem(q, variant=v, orientation="panel8", precision="fp32",
                                          lib=lib).Q, csr=q.csr)
        o2 = ref.orth_loss(ref.qr_problem(q, variant=v, orientation="panel8", precision="fp32",
                                          reorth=2, lib=lib).Q, csr=q.csr)
        if not o2 < 1e-2 * o0:
            fails.append(f"blocked pass binary32 orthogonality {v}: {o0} -> {o2}")
    # only with the two-level panel orientation
    try:
        ref.qr(q.Z, csr=q.csr, variant="ha", orientation="panel", reorth=2, lib=lib)
        fails.append("blocked pass accepted outside the two-level orientation")
    except ValueError:
        pass
    return fails


def pin_cgs(lib) -> list:
    """Classical Gram-Schmidt (orientation "cgs"): the closed forms on
    well-conditioned problems (with and without the second pass), Householder
    for A = I with the three variants equal bit for bit, MV counts; Section 3
    (analysis of CGS): CGS-HA loses about as much A-orthogonality as
    CGS-naive; Section 4 (experiment II): the loss of CGS grows with the
    square of kappa(A^{1/2} Z) while MGS grows linearly, so at
    kappa(A^{1/2} Z) ~ 6e5 CGS is far less accurate than MGS (and within
    10 u kappa(A) kappa(A^{1/2} Z)^2); a second classical pass (CGS2)
    restores A-orthogonality to rounding level for naive and HA."""
    fails = []
    for seed in (11, 12):
        for p in (inputs.random_dense_problem(60, 9, seed), inputs.random_csr_problem(300, 12, 9, seed)):
            Ad = p.dense if p.dense is not None else p.csr.to_dense()
            Rc = _chol_R(p.Z, Ad)
            for v in VARIANTS:
                for re_ in (False, True):
                    r = ref.qr(p.Z, dense=p.dense, csr=p.csr, variant=v, orientation="cgs",
                               reorth=re_, lib=lib)
                    e, eq, ep = (_rel(np.triu(r.R), Rc), _rel(r.Q, np.linalg.solve(Rc.T, p.Z.T).T),
                                 _rel(r.P, Ad @ r.Q))
                    if r.info != 0 or not (e <= 1e-13 and eq <= 1e-12 and ep <= 1e-12):
                        fails.append(f"cgs chol {p.name} {v}/reorth={re_}: R {e} Q {eq} P {ep}")
                    want_calls = {"naive": 2 * p.n, "ha": p.n, "hp": 1}[v]
                    if r.mv_calls != want_calls:
                        fails.append(f"cgs MV count {p.name} {v}: {r.mv_calls}")
    g = inputs.rng(23)
    m, n = 150, 9
    Z = np.asfortranarray(g.standard_normal((m, n)))
    eye = inputs.CSR(m, np.arange(m + 1, dtype=np.int32), np.arange(m, dtype=np.int32), np.ones(m))
    Qh, Rh = np.linalg.qr(Z)
    D = np.sign(np.diag(Rh))
    Qh, Rh = Qh * D[None, :], Rh * D[:, None]
    outs = {v: ref.qr(Z, csr=eye, variant=v, orientation="cgs", lib=lib) for v in VARIANTS}
    for v, r in outs.items():
        if _rel(np.triu(r.R), Rh) > 1e-13 or _rel(r.Q, Qh) > 1e-12:
            fails.append(f"cgs identity {v}: R {_rel(np.triu(r.R), Rh)} Q {_rel(r.Q, Qh)}")
        if not (np.array_equal(r.R, outs["naive"].R) and np.array_equal(r.Q, outs["naive"].Q)):
            fails.append(f"cgs identity: {v} differs bitwise from naive")
    u = 2.0 ** -53
    for ka, kz in ((1e2, 1e6), (1e4, 1e4)):
        p = inputs.exp2_problem(100, 20, ka, kz, 1, 7)
        w, V = np.linalg.eigh(p.dense)
        kA = float(w[-1] / w[0])
        kAZ = _kappa((V * np.sqrt(w)[None, :]) @ V.T @ p.Z)
        loss = {}
        for v in ("naive", "ha"):
            r = ref.qr_problem(p, variant=v, orientation="cgs", lib=lib)
            loss[v] = ref.orth_loss(r.Q, dense=p.dense)
            if r.info != 0 or not loss[v] <= 10 * u * kA * kAZ ** 2:
                fails.append(f"cgs exp2 {ka:g},{kz:g} {v}: loss {loss[v]} above the quadratic bound")
            r2 = ref.qr_problem(p, variant=v, orientation="cgs", reorth=True, lib=lib)
            l2 = ref.orth_loss(r2.Q, dense=p.dense)
            if not l2 <= 1e-13:
                fails.append(f"cgs2 exp2 {ka:g},{kz:g} {v}: loss {l2}")
        if not (0.1 <= loss["ha"] / loss["naive"] <= 10):
            fails.append(f"cgs exp2 {ka:g},{kz:g}: HA {loss['ha']} vs naive {loss['naive']}")
        if kz >= 1e6:
            lm = ref.orth_loss(ref.qr_problem(p, variant="ha", lib=lib).Q, dense=p.dense)
            if not loss["ha"] >= 1e3 * lm:
                fails.append(f"cgs exp2 {ka:g},{kz:g}: CGS {loss['ha']} not far above MGS {lm}")
    return fails


def pin_successive(lib) -> list:
    """Successive orthogonalisation (Section 2.1: the column form suits it):
    column j of the column algorithm depends only on columns before it, so
    orthonormalising the first k columns and then appending the rest
    (first = k, the k final columns passed in) must reproduce the one-call
    result bit for bit, for every variant, the classical form and the second
    pass; on a well-conditioned problem the appended result also equals the
    closed form R = chol(Z^T A Z)."""
    fails = []
    for p in (inputs.random_dense_problem(60, 11, 13), inputs.random_csr_problem(300, 10, 9, 14)):
        Ad = p.dense if p.dense is not None else p.csr.to_dense()
        Rc = _chol_R(p.Z, Ad)
        for o in ("col", "cgs"):
            for v in VARIANTS:
                for re_ in (False, True):
                    for prec in ("fp64", "fp32"):
                        kw = dict(dense=p.dense, csr=p.csr, variant=v, orientation=o, reorth=re_,
                                  precision=prec, lib=lib)
                        full = ref.qr(p.Z, **kw)
                        for k in (1, 4):
                            part = ref.qr(p.Z[:, :k], **kw)
                            succ = ref.qr(p.Z, first=k, Q0=part.Q, P0=part.P, R0=part.R, **kw)
                            tag = f"{p.name} {o}/{v}/reorth={re_}/{prec}/first={k}"
                            if succ.info != 0 or not (np.array_equal(succ.Q, full.Q)
                                                      and np.array_equal(succ.R, full.R)
                                                      and np.array_equal(succ.P, full.P)):
                                fails.append(f"successive {tag}: differs from one call")
                            if prec == "fp64" and _rel(np.triu(succ.R), Rc) > 1e-13:
                                fails.append(f"successive {tag}: R vs chol {_rel(np.triu(succ.R), Rc)}")
    return fails


ALL_PINS = [pin_hand_example, pin_cholesky, pin_identity_householder, pin_cholesky_factor,
            pin_col_row_bitwise, pin_mv_counts, pin_scaling, pin_first_column,
            pin_residual_and_reorth, pin_exp2_accuracy, pin_fp32_accumulation,
            pin_fp32_mv_axpy_rounding, pin_fp32_vs_fp64, pin_breakdown,
            pin_panel, pin_panel8, pin_panel16, pin_blocked_second_pass, pin_cgs, pin_successive]
