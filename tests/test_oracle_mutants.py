"""Plant plausible mistakes in a copy of the oracle and check that the pins
catch every one of them (the mistakes live only in temporary copies)."""
import os
import shutil
import tempfile

import pytest

import pins
from conftest import ROOT, read_golden
from oracle import ref

SRC = os.path.join(ROOT, "oracle", "amgs_ref.c")

# (name, original text, planted text)
MUTANTS = [
    ("projection uses q instead of p (standard inner product)",
     "Rc[i] = dot_st(P + i * ldp, z, m, prec);", "Rc[i] = dot_st(Q + i * ldq, z, m, prec);"),
    ("projection update sign flipped",
     "z[k] = z[k] - prod;", "z[k] = z[k] + prod;"),
    ("HP recurrence uses q instead of p",
     "axpy_st(x, st(Rc[i], prec), P + i * ldp, m, prec);",
     "axpy_st(x, st(Rc[i], prec), Q + i * ldq, m, prec);"),
    ("HP recurrence term dropped (last i)",
     "for (int64_t i = 0; i < j; ++i) axpy_st(x, st(Rc[i], prec)",
     "for (int64_t i = 0; i + 1 < j; ++i) axpy_st(x, st(Rc[i], prec)"),
    ("HA auxiliary vector from z instead of x",
     "scale(P + j * ldp, x, rjj, m, prec);", "scale(P + j * ldp, z, rjj, m, prec);"),
    ("A-norm without square root", "*rjj = sqrt(rr);", "*rjj = rr;"),
    ("row form stores r_ij transposed",
     "R[j * ldr + i] = rij;", "R[i * ldr + j] = rij;"),
    ("row HP recurrence uses the wrong column of X",
     "axpy_st(X + j * m, st(R[j * ldr + i], prec)", "axpy_st(X + i * m, st(R[j * ldr + i], prec)"),
    ("second pass does not add s_i into R",
     "Rcol[i] = Rcol[i] + s[i - i0];", "Rcol[i] = Rcol[i];"),
    ("A-norm accumulated in binary32 in the binary32 form",
     "double rr = dot_hi(z, x, m);", "double rr = dot_st(z, x, m, REF_FP32);"),
    ("binary32 projections accumulated in binary64",
     "        if (prec == REF_FP32) {\n            float s = 0.0f;\n            for (int64_t k = lo;",
     "        if (0) {\n            float s = 0.0f;\n            for (int64_t k = lo;"),
    ("dense MV walks a row of the wrong matrix (transposed operand of a non-symmetric read)",
     "const double *col = A->a + k * A->lda;", "const double *col = A->a + k;"),
    ("panel block step without the triangular correction",
     "for (int k = 0; k < i; ++k) t = t - L[i * b + k] * r[k];",
     "for (int k = 0; k < i; ++k) t = t - 0.0 * r[k];"),
    ("panel block step updates x with q instead of p",
     "axpy_st(c->X + col * m, st(r[i], c->prec), c->P + (s + i) * c->ldp, m, c->prec);",
     "axpy_st(c->X + col * m, st(r[i], c->prec), c->Q + (s + i) * c->ldq, m, c->prec);"),
    ("classical Gram-Schmidt leaves the HP x column uncorrected",
     "        /* r_ij = p_i^T z_j^{(0)} for every i < j, then one correction */\n        reorth_pass(z, xr, j,",
     "        /* r_ij = p_i^T z_j^{(0)} for every i < j, then one correction */\n        reorth_pass(z, NULL, j,"),
    ("appended columns skip the projections onto the final columns",
     "for (int64_t i = 0; i < j; ++i) {           /* projections */",
     "for (int64_t i = first; i < j; ++i) {           /* projections */"),
    ("binary32 CSR MV row sum accumulated in binary64 and rounded once",
     "                float s = 0.0f;\n"
     "                for (int32_t e = A->row_ptr[k]; e < A->row_ptr[k + 1]; ++e) {\n"
     "                    float prod = (float)A->vals[e] * (float)v[A->col_idx[e]];\n"
     "                    s = s + prod;\n"
     "                }\n"
     "                y[k] = s;",
     "                double s = 0.0;\n"
     "                for (int32_t e = A->row_ptr[k]; e < A->row_ptr[k + 1]; ++e) {\n"
     "                    float prod = (float)A->vals[e] * (float)v[A->col_idx[e]];\n"
     "                    s = s + prod;\n"
     "                }\n"
     "                y[k] = (float)s;"),
    ("binary32 dense MV row sum accumulated in binary64 and rounded once",
     "                float s = 0.0f;\n"
     "                for (int64_t l = 0; l < m; ++l) {\n"
     "                    float prod = (float)col[l] * (float)v[l];\n"
     "                    s = s + prod;\n"
     "                }\n"
     "                y[k] = s;",
     "                double s = 0.0;\n"
     "                for (int64_t l = 0; l < m; ++l) {\n"
     "                    float prod = (float)col[l] * (float)v[l];\n"
     "                    s = s + prod;\n"
     "                }\n"
     "                y[k] = (float)s;"),
    ("binary32 CSR MV row summed from its last entry",
     "                for (int32_t e = A->row_ptr[k]; e < A->row_ptr[k + 1]; ++e) {\n"
     "                    float prod",
     "                for (int32_t e = A->row_ptr[k + 1] - 1; e >= A->row_ptr[k]; --e) {\n"
     "                    float prod"),
    ("binary32 projection update with one binary64 rounding",
     "            float zk = (float)z[k] - prod;",
     "            float zk = (float)(z[k] - (double)rf * q[k]);"),
    ("panel block step skips the last panel column",
     "for (int i = 0; i < b; ++i) axpy_st(z, st(r[i], c->prec), c->Q + (s + i) * c->ldq, m, c->prec);",
     "for (int i = 0; i + 1 < b; ++i) axpy_st(z, st(r[i], c->prec), c->Q + (s + i) * c->ldq, m, c->prec);"),
    ("two-level panels: a 4-panel block also acts beyond its own 8-panel",
     "if (e < E) panel_block(c, s, e, e, E);",
     "if (e < E) panel_block(c, s, e, e, lev > 0 ? c->n : E);"),
    ("blocked second pass leaves the last earlier column out",
     "                             0, s, c->Q, c->ldq, c->P, c->ldp, c->R + col * c->ldr, c->m, c->prec);",
     "                             0, s - 1, c->Q, c->ldq, c->P, c->ldp, c->R + col * c->ldr, c->m, c->prec);"),
    ("blocked second pass skips the last column of each outer panel",
     "            for (int64_t col = s; col < e; ++col)\n                reorth_range(",
     "            for (int64_t col = s; col + 1 < e; ++col)\n                reorth_range("),
    ("two-level panels: a finished 8-panel never acts on the later columns",
     "if (e < E) panel_block(c, s, e, e, E);",
     "if (e < E && lev > 0) panel_block(c, s, e, e, E);"),
]


@pytest.mark.parametrize("name,orig,planted", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, orig, planted):
    src = open(SRC).read()
    assert src.count(orig) >= 1, f"mutation anchor not found: {orig!r}"
    tmp = tempfile.mkdtemp(prefix="amgs_mut_")
    try:
        msrc = os.path.join(tmp, "mut.c")
        with open(msrc, "w") as f:
            f.write(src.replace(orig, planted, 1))
        lib = ref.load(ref.build(src=msrc, out=os.path.join(tmp, "libmut.so")))
        golden = read_golden("hand_example.txt")
        caught = []
        for pin in pins.ALL_PINS:
            try:
                fails = pin(lib, golden) if pin is pins.pin_hand_example else pin(lib)
            except Exception as e:  # a crash of the mutant also counts as caught
                fails = [repr(e)]
            if fails:
                caught.append(pin.__name__)
        assert caught, f"no pin catches mutant: {name}"
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
