/*
 * amgs_ref.c -- CPU oracle for A-orthonormalising modified Gram-Schmidt.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header
 * or helper with the GPU library.
 *
 * Problem (Section 1, eq. (1)): given Z (m x n, m >= n) and a symmetric
 * positive definite A (m x m), compute Z = QR with Q^T A Q = I_n and R upper
 * triangular with a positive diagonal.
 *
 * The three variants of Section 2 are implemented step by step:
 *   naive (Alg. 3 column / Alg. 4 row): r_ij = p_i^T z_j with p_i = A q_i,
 *         two matrix-vector products (MV) per column, 2n MV in total;
 *   HA    (Alg. 5 column / Alg. 7 row): p_j = x_j / r_jj (eq. (4)),
 *         one MV per column, n MV in total;
 *   HP    (Alg. 6 column / Alg. 8 row): X = A Z as one block product, then
 *         x_j^{(j-1)} = x_j^{(0)} - sum_{i<j} r_ij p_i (eq. (5)).
 *
 * Arithmetic conventions (the paper fixes none of these):
 *   - FP64 throughout in precision 0.  Compile with -ffp-contract=off so that
 *     every a - r*b is a rounded multiply followed by a rounded subtract.
 *   - dot products: rows are split into consecutive blocks of 1024; each block
 *     is summed left to right, then the block sums are added left to right.
 *     The result therefore does not depend on the number of OpenMP threads.
 *   - CSR MV: each row sums a_kl * v_l in stored (ascending column) order.
 *     Dense MV: y_k = sum_l A[l,k] v_l with l ascending (A is symmetric and
 *     column-major, so this walks column k).
 *   - division is a true division.
 *   - a column whose squared A-norm z_j^T x_j is not positive and finite is a
 *     breakdown: the routine stops and reports the 1-based column index.
 *
 * Precision 1 emulates the FP32-storage form: A, Z, Q, P, X hold binary32
 * values; MV, the projections r_ij = p_i^T z_j (binary32 accumulation) and
 * the updates z_j -= r_ij q_i, x_j -= r_ij p_i run in binary32; the squared
 * A-norm is accumulated in binary64 from the binary32 values, the square root
 * and the divisions q_j = z_j / r_jj, p_j = x_j / r_jj are binary64 and their
 * results are rounded to binary32.  R is binary64.
 *
 * Orientation 2 is the panel schedule of the GPU library (not in the paper;
 * a regrouping of the column algorithm's projections): columns are taken in
 * panels of 4; inside a panel the column algorithm runs on the panel's
 * columns only; after a panel [s, e) is finished, every later column c gets
 * the panel's effect as one block: W_i = p_i^T z_c (the same z_c for all i),
 * L_ik = p_i^T q_k (k < i, both inside the panel), r_ic = W_i -
 * sum_{k<i} L_ik r_kc (forward substitution, binary64), then z_c -= r_ic q_i
 * for i ascending (HP: also x_c -= r_ic p_i).  In exact arithmetic this is
 * the column algorithm, since z_c^{(i-1)} = z_c - sum_{k<i} r_kc q_k.  The
 * optional second pass below runs on column j at the same point as in the
 * column form (after its projections, before its MV).
 *
 * Orientation 4 is the same regrouping on two levels: panels of 8 columns,
 * each taken apart as two panels of 4 exactly as in orientation 2 but with
 * blocks acting only on the columns of the same 8-panel, and each finished
 * 8-panel acting on every later column as one block of 8 (W, L, r as above
 * with 8 columns).  A column therefore receives, in this order: the blocks
 * of every earlier 8-panel, the block of the earlier 4-panel of its own
 * 8-panel, then the column algorithm's projections inside its 4-panel.
 * With n <= 8 it is orientation 2.
 *
 * Orientation 5 is the same regrouping on three levels: panels of 16
 * columns, each taken apart as two panels of 8 exactly as in orientation 4
 * but with the 8-panel blocks acting only on the columns of the same
 * 16-panel, and each finished 16-panel acting on every later column as one
 * block of 16.  A column receives the blocks of every earlier 16-panel, the
 * block of the earlier 8-panel of its own 16-panel, the block of the earlier
 * 4-panel of its own 8-panel, then the projections inside its 4-panel.  With
 * n <= 16 it is orientation 4.
 *
 * Orientation 3 is classical Gram-Schmidt with the same three variants
 * (Section 2: the n-MV idea applied to CGS; Section 3, analysis of CGS):
 * column j takes all its coefficients from the unmodified column,
 * r_ij = p_i^T z_j^{(0)} for i < j, then z_j^{(j-1)} = z_j^{(0)} -
 * sum_{i<j} r_ij q_i, and for HP x_j^{(j-1)} = x_j^{(0)} - sum_{i<j} r_ij p_i;
 * naive and HA then form x_j = A z_j^{(j-1)}.  This classical step uses the
 * arithmetic of the second pass below (binary64 accumulation of the
 * coefficients and of each corrected entry, one rounding to storage), and
 * with reorth it is applied twice (CGS2).
 *
 * Optional reorthogonalisation (the paper names it in Section 2.1 without a
 * definition): after the MGS projections of column j, a classical second
 * pass s_i = p_i^T z_j for all i < j (binary64 accumulation), then
 * z_j <- z_j - sum_i s_i q_i (binary64, rounded once to storage), and
 * r_ij += s_i.  For HP the same s_i also correct x_j: x_j <- x_j -
 * sum_i s_i p_i (binary64, rounded once), applied after the first-pass
 * recurrence.
 *
 * reorth = 2, blocked second pass (orientation 4 only): when an outer panel
 * [S, E) starts, its columns have received every first-pass projection onto
 * the columns before S; each of them then gets the classical pass above
 * against all i < S at once (same arithmetic), and later, at its own step,
 * the pass against the earlier columns of its outer panel only, i in
 * [S, j).  The two parts together cover every i < j, as the per-column pass
 * does, with the earlier outer panels streamed once per outer panel instead
 * of once per column.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define REF_NAIVE 0
#define REF_HA 1
#define REF_HP 2
#define REF_COL 0
#define REF_ROW 1
#define REF_PANEL 2
#define REF_CGS 3
#define REF_PANEL2 4
#define REF_PANEL3 5
#define REF_FP64 0
#define REF_FP32 1
#define DOT_BLOCK 1024

typedef struct {
    int kind; /* 0 dense, 1 csr */
    int64_t m;
    const double *a; int64_t lda;                /* dense, column-major */
    const int32_t *row_ptr, *col_idx; const double *vals; /* csr */
} ref_op;

/* Round to the storage precision. */
static inline double st(double v, int prec) { return prec == REF_FP32 ? (double)(float)v : v; }

/* ---------------------------------------------------------------- dots */
/* r = a^T b accumulated in the storage precision (binary32 in precision 1). */
static double dot_st(const double *a, const double *b, int64_t m, int prec)
{
    int64_t nb = (m + DOT_BLOCK - 1) / DOT_BLOCK;
    double *part = (double *)malloc((size_t)(nb > 0 ? nb : 1) * sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t blk = 0; blk < nb; ++blk) {
        int64_t lo = blk * DOT_BLOCK, hi = lo + DOT_BLOCK < m ? lo + DOT_BLOCK : m;
        if (prec == REF_FP32) {
            float s = 0.0f;
            for (int64_t k = lo; k < hi; ++k) {
                float prod = (float)a[k] * (float)b[k];
                s = s + prod;
            }
            part[blk] = s;
        } else {
            double s = 0.0;
            for (int64_t k = lo; k < hi; ++k) {
                double prod = a[k] * b[k];
                s = s + prod;
            }
            part[blk] = s;
        }
    }
    double r;
    if (prec == REF_FP32) {
        float s = 0.0f;
        for (int64_t blk = 0; blk < nb; ++blk) s = s + (float)part[blk];
        r = s;
    } else {
        double s = 0.0;
        for (int64_t blk = 0; blk < nb; ++blk) s = s + part[blk];
        r = s;
    }
    free(part);
    return r;
}

/* a^T b accumulated in binary64 (used for the A-norm and the second pass). */
static double dot_hi(const double *a, const double *b, int64_t m)
{
    return dot_st(a, b, m, REF_FP64);
}

/* ---------------------------------------------------------------- axpy */
/* z <- z - r q  (eq. (9)), in the storage precision. */
static void axpy_st(double *z, double r, const double *q, int64_t m, int prec)
{
    if (prec == REF_FP32) {
        float rf = (float)r;
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < m; ++k) {
            float prod = rf * (float)q[k];
            float zk = (float)z[k] - prod;
            z[k] = zk;
        }
    } else {
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < m; ++k) {
            double prod = r * q[k];
            z[k] = z[k] - prod;
        }
    }
}

/* ---------------------------------------------------------------- MV */
/* y <- A v in the storage precision. */
static void mv_st(const ref_op *A, const double *v, double *y, int prec)
{
    int64_t m = A->m;
    if (A->kind == 1) {
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < m; ++k) {
            if (prec == REF_FP32) {
                float s = 0.0f;
                for (int32_t e = A->row_ptr[k]; e < A->row_ptr[k + 1]; ++e) {
                    float prod = (float)A->vals[e] * (float)v[A->col_idx[e]];
                    s = s + prod;
                }
                y[k] = s;
            } else {
                double s = 0.0;
                for (int32_t e = A->row_ptr[k]; e < A->row_ptr[k + 1]; ++e) {
                    double prod = A->vals[e] * v[A->col_idx[e]];
                    s = s + prod;
                }
                y[k] = s;
            }
        }
    } else {
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < m; ++k) {
            const double *col = A->a + k * A->lda;
            if (prec == REF_FP32) {
                float s = 0.0f;
                for (int64_t l = 0; l < m; ++l) {
                    float prod = (float)col[l] * (float)v[l];
                    s = s + prod;
                }
                y[k] = s;
            } else {
                double s = 0.0;
                for (int64_t l = 0; l < m; ++l) {
                    double prod = col[l] * v[l];
                    s = s + prod;
                }
                y[k] = s;
            }
        }
    }
}

/* y <- v / r  (eq. (10)): binary64 division, rounded to storage. */
static void scale(double *y, const double *v, double r, int64_t m, int prec)
{
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < m; ++k) y[k] = st(v[k] / r, prec);
}

/* ------------------------------------------------- second (reorth) pass */
/* s_i = p_i^T z for i < j (binary64), z <- z - sum_i s_i q_i, r_ij += s_i.
 * For HP, also x <- x - sum_i s_i p_i. */
static void reorth_range(double *z, double *x_or_null, int64_t i0, int64_t j, const double *Q,
                         int64_t ldq, const double *P, int64_t ldp, double *Rcol, int64_t m,
                         int prec)
{
    if (j <= i0) return;
    double *s = (double *)malloc((size_t)(j - i0) * sizeof(double));
    for (int64_t i = i0; i < j; ++i) s[i - i0] = dot_hi(P + i * ldp, z, m);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < m; ++k) {
        double zk = z[k];
        for (int64_t i = i0; i < j; ++i) {
            double prod = s[i - i0] * Q[i * ldq + k];
            zk = zk - prod;
        }
        z[k] = st(zk, prec);
        if (x_or_null) {
            double xk = x_or_null[k];
            for (int64_t i = i0; i < j; ++i) {
                double prod = s[i - i0] * P[i * ldp + k];
                xk = xk - prod;
            }
            x_or_null[k] = st(xk, prec);
        }
    }
    for (int64_t i = i0; i < j; ++i) Rcol[i] = Rcol[i] + s[i - i0];
    free(s);
}

/* The second pass of column j against every earlier column. */
static void reorth_pass(double *z, double *x_or_null, int64_t j, const double *Q, int64_t ldq,
                        const double *P, int64_t ldp, double *Rcol, int64_t m, int prec)
{
    reorth_range(z, x_or_null, 0, j, Q, ldq, P, ldp, Rcol, m, prec);
}

/* r_jj = sqrt(z^T x) with binary64 accumulation; returns 0 on breakdown. */
static int anorm(const double *z, const double *x, int64_t m, double *rjj)
{
    double rr = dot_hi(z, x, m);
    if (!(rr > 0.0) || !isfinite(rr)) return 0;
    *rjj = sqrt(rr);
    return 1;
}

/* ------------------------------------------------------------ driver */
/* Column-oriented: Alg. 3 (naive), Alg. 5 (HA), Alg. 6 (HP). */
static int qr_col(const ref_op *A, int64_t m, int64_t n, int64_t first, double *Q, int64_t ldq,
                  double *R, int64_t ldr, double *P, int64_t ldp, double *X, int variant,
                  int reorth, int prec, int64_t *mv_calls, int64_t *mv_cols)
{
    double *x = (double *)malloc((size_t)m * sizeof(double));
    if (variant == REF_HP) {            /* Alg. 6: X = A Z, one block MV */
        for (int64_t j = first; j < n; ++j) mv_st(A, Q + j * ldq, X + j * m, prec);
        *mv_calls += 1; *mv_cols += n - first;
    }
    int info = 0;
    /* columns before first are final (successive orthogonalisation) */
    for (int64_t j = first; j < n && !info; ++j) {
        double *z = Q + j * ldq;        /* holds z_j^{(i)}; overwritten by q_j */
        double *Rc = R + j * ldr;
        for (int64_t i = 0; i < j; ++i) {           /* projections */
            Rc[i] = dot_st(P + i * ldp, z, m, prec); /* r_ij = p_i^T z_j^{(i-1)} */
            axpy_st(z, Rc[i], Q + i * ldq, m, prec); /* z_j^{(i)} = z_j^{(i-1)} - r_ij q_i */
        }
        double *xr = NULL;
        if (variant == REF_HP) {
            /* x_j^{(j-1)} = x_j^{(0)} - sum_{i<j} r_ij p_i, i ascending */
            memcpy(x, X + j * m, (size_t)m * sizeof(double));
            for (int64_t i = 0; i < j; ++i) axpy_st(x, st(Rc[i], prec), P + i * ldp, m, prec);
            xr = x;
        }
        if (reorth) reorth_pass(z, xr, j, Q, ldq, P, ldp, Rc, m, prec);
        if (variant != REF_HP) {        /* boxed MV: x_j^{(j-1)} = A z_j^{(j-1)} */
            mv_st(A, z, x, prec);
            *mv_calls += 1; *mv_cols += 1;
        }
        double rjj;
        if (!anorm(z, x, m, &rjj)) { info = (int)(j + 1); break; }
        Rc[j] = rjj;
        scale(z, z, rjj, m, prec);                  /* q_j = z_j^{(j-1)} / r_jj */
        if (variant == REF_NAIVE) {                 /* boxed MV: p_j = A q_j */
            mv_st(A, z, P + j * ldp, prec);
            *mv_calls += 1; *mv_cols += 1;
        } else {
            scale(P + j * ldp, x, rjj, m, prec);    /* p_j = x_j^{(j-1)} / r_jj (eq. (4)) */
        }
    }
    free(x);
    return info;
}

/* Row-oriented: Alg. 4 (naive), Alg. 7 (HA), Alg. 8 (HP).  In HP(row) the
 * x-update printed in the paper is read as: at step i, for every j > i,
 * x_j^{(i)} = x_j^{(i-1)} - r_ij p_i (the row analogue of eq. (5)). */
static int qr_row(const ref_op *A, int64_t m, int64_t n, double *Q, int64_t ldq, double *R,
                  int64_t ldr, double *P, int64_t ldp, double *X, int variant, int reorth,
                  int prec, int64_t *mv_calls, int64_t *mv_cols)
{
    double *x = (double *)malloc((size_t)m * sizeof(double));
    if (variant == REF_HP) {
        for (int64_t j = 0; j < n; ++j) mv_st(A, Q + j * ldq, X + j * m, prec);
        *mv_calls += 1; *mv_cols += n;
    }
    int info = 0;
    for (int64_t i = 0; i < n && !info; ++i) {
        double *z = Q + i * ldq;
        double *xr = NULL;
        if (variant == REF_HP) xr = X + i * m;      /* already x_i^{(i-1)} */
        if (reorth) reorth_pass(z, xr, i, Q, ldq, P, ldp, R + i * ldr, m, prec);
        if (variant == REF_HP) {
            memcpy(x, X + i * m, (size_t)m * sizeof(double));
        } else {
            mv_st(A, z, x, prec);                   /* x_i^{(i-1)} = A z_i^{(i-1)} */
            *mv_calls += 1; *mv_cols += 1;
        }
        double rii;
        if (!anorm(z, x, m, &rii)) { info = (int)(i + 1); break; }
        R[i * ldr + i] = rii;
        scale(z, z, rii, m, prec);                  /* q_i */
        if (variant == REF_NAIVE) {
            mv_st(A, z, P + i * ldp, prec);         /* p_i = A q_i */
            *mv_calls += 1; *mv_cols += 1;
        } else {
            scale(P + i * ldp, x, rii, m, prec);    /* p_i = x_i^{(i-1)} / r_ii */
        }
        for (int64_t j = i + 1; j < n; ++j) {
            double rij = dot_st(P + i * ldp, Q + j * ldq, m, prec);
            R[j * ldr + i] = rij;
            axpy_st(Q + j * ldq, rij, Q + i * ldq, m, prec);
        }
        if (variant == REF_HP)
            for (int64_t j = i + 1; j < n; ++j)
                axpy_st(X + j * m, st(R[j * ldr + i], prec), P + i * ldp, m, prec);
    }
    free(x);
    return info;
}

/* Panel schedule (orientations 2 and 4): see the header comment. */
typedef struct {
    const ref_op *A;
    int64_t m, n;
    double *Q, *R, *P, *X, *x;
    int64_t ldq, ldr, ldp;
    int variant, reorth, prec;
    int64_t *mv_calls, *mv_cols;
    int nlev;
    const int *width;   /* panel widths, outermost first; each divides the one before */
    int64_t re_lo;      /* reorth == 2: the in-panel second pass starts at this column */
} panel_ctx;

/* The column algorithm on the columns [s, e) of a finished-below panel: each
 * column j gets its projections onto the panel's earlier columns i in [s, j),
 * then (HP) the same terms of eq. (5) on x_j, the optional second pass, its
 * MV (naive, HA), its A-norm and normalisation. */
static int panel_columns(const panel_ctx *c, int64_t s, int64_t e)
{
    const int64_t m = c->m;
    for (int64_t j = s; j < e; ++j) {
        double *z = c->Q + j * c->ldq;
        double *Rc = c->R + j * c->ldr;
        for (int64_t i = s; i < j; ++i) {
            Rc[i] = dot_st(c->P + i * c->ldp, z, m, c->prec);
            axpy_st(z, Rc[i], c->Q + i * c->ldq, m, c->prec);
        }
        double *xr = NULL;
        if (c->variant == REF_HP) {
            /* X[:, j] already holds the terms of the earlier panels */
            memcpy(c->x, c->X + j * m, (size_t)m * sizeof(double));
            for (int64_t i = s; i < j; ++i)
                axpy_st(c->x, st(Rc[i], c->prec), c->P + i * c->ldp, m, c->prec);
            xr = c->x;
        }
        /* the optional second pass, at the same point as in the column form;
         * in the blocked form only against the columns of its outer panel */
        if (c->reorth)
            reorth_range(z, xr, c->reorth == 2 ? c->re_lo : 0, j, c->Q, c->ldq, c->P, c->ldp, Rc,
                         m, c->prec);
        if (c->variant != REF_HP) {
            mv_st(c->A, z, c->x, c->prec);
            *c->mv_calls += 1; *c->mv_cols += 1;
        }
        double rjj;
        if (!anorm(z, c->x, m, &rjj)) return (int)(j + 1);
        Rc[j] = rjj;
        scale(z, z, rjj, m, c->prec);
        if (c->variant == REF_NAIVE) {
            mv_st(c->A, z, c->P + j * c->ldp, c->prec);
            *c->mv_calls += 1; *c->mv_cols += 1;
        } else {
            scale(c->P + j * c->ldp, c->x, rjj, m, c->prec);
        }
    }
    return 0;
}

/* The finished panel [s, e) acting on the columns [c0, c1) as one block:
 * W_i = p_i^T z_c, L_ik = p_i^T q_k (k < i, both in the panel), r_ic = W_i -
 * sum_{k<i} L_ik r_kc (binary64), z_c -= r_ic q_i for i ascending (HP also
 * x_c -= r_ic p_i). */
static void panel_block(const panel_ctx *c, int64_t s, int64_t e, int64_t c0, int64_t c1)
{
    const int64_t m = c->m;
    const int b = (int)(e - s);
    double *L = (double *)malloc((size_t)b * b * sizeof(double));
    double *W = (double *)malloc((size_t)b * sizeof(double));
    double *r = (double *)malloc((size_t)b * sizeof(double));
    for (int i = 0; i < b; ++i)
        for (int k = 0; k < i; ++k)
            L[i * b + k] = dot_st(c->P + (s + i) * c->ldp, c->Q + (s + k) * c->ldq, m, c->prec);
    for (int64_t col = c0; col < c1; ++col) {
        double *z = c->Q + col * c->ldq;
        for (int i = 0; i < b; ++i) W[i] = dot_st(c->P + (s + i) * c->ldp, z, m, c->prec);
        for (int i = 0; i < b; ++i) {
            double t = W[i];
            for (int k = 0; k < i; ++k) t = t - L[i * b + k] * r[k];
            r[i] = t;
            c->R[col * c->ldr + s + i] = t;
        }
        for (int i = 0; i < b; ++i) axpy_st(z, st(r[i], c->prec), c->Q + (s + i) * c->ldq, m, c->prec);
        if (c->variant == REF_HP)
            for (int i = 0; i < b; ++i)
                axpy_st(c->X + col * m, st(r[i], c->prec), c->P + (s + i) * c->ldp, m, c->prec);
    }
    free(L); free(W); free(r);
}

/* Columns [S, E) at level lev: panels of width[lev] in order; each is taken
 * apart at the next level (the column algorithm below the last one), and
 * once finished acts as one block on the remaining columns of [S, E). */
static int panel_range(panel_ctx *c, int64_t S, int64_t E, int lev)
{
    const int64_t B = c->width[lev];
    for (int64_t s = S; s < E; s += B) {
        const int64_t e = s + B < E ? s + B : E;
        if (c->reorth == 2 && lev == 0) {
            /* blocked second pass: every column of this outer panel against
             * all earlier columns at once (their first pass against those
             * is complete), then in-panel passes from s on */
            for (int64_t col = s; col < e; ++col)
                reorth_range(c->Q + col * c->ldq, c->variant == REF_HP ? c->X + col * c->m : NULL,
                             0, s, c->Q, c->ldq, c->P, c->ldp, c->R + col * c->ldr, c->m, c->prec);
            c->re_lo = s;
        }
        const int info = lev + 1 < c->nlev ? panel_range(c, s, e, lev + 1) : panel_columns(c, s, e);
        if (info) return info;
        if (e < E) panel_block(c, s, e, e, E);
    }
    return 0;
}

static int qr_panel(const ref_op *A, int64_t m, int64_t n, double *Q, int64_t ldq, double *R,
                    int64_t ldr, double *P, int64_t ldp, double *X, int variant, int reorth,
                    int prec, int nlev, const int *width, int64_t *mv_calls, int64_t *mv_cols)
{
    double *x = (double *)malloc((size_t)m * sizeof(double));
    if (variant == REF_HP) {
        for (int64_t j = 0; j < n; ++j) mv_st(A, Q + j * ldq, X + j * m, prec);
        *mv_calls += 1; *mv_cols += n;
    }
    panel_ctx c = {A, m, n, Q, R, P, X, x, ldq, ldr, ldp, variant, reorth, prec,
                   mv_calls, mv_cols, nlev, width, 0};
    const int info = panel_range(&c, 0, n, 0);
    free(x);
    return info;
}

/* Classical Gram-Schmidt, column form (orientation 3). */
static int qr_cgs(const ref_op *A, int64_t m, int64_t n, int64_t first, double *Q, int64_t ldq,
                  double *R, int64_t ldr, double *P, int64_t ldp, double *X, int variant,
                  int reorth, int prec, int64_t *mv_calls, int64_t *mv_cols)
{
    double *x = (double *)malloc((size_t)m * sizeof(double));
    if (variant == REF_HP) {
        for (int64_t j = first; j < n; ++j) mv_st(A, Q + j * ldq, X + j * m, prec);
        *mv_calls += 1; *mv_cols += n - first;
    }
    int info = 0;
    for (int64_t j = first; j < n && !info; ++j) {
        double *z = Q + j * ldq;        /* z_j^{(0)}, corrected in place */
        double *Rc = R + j * ldr;
        double *xr = NULL;
        if (variant == REF_HP) {
            memcpy(x, X + j * m, (size_t)m * sizeof(double));
            xr = x;
        }
        /* r_ij = p_i^T z_j^{(0)} for every i < j, then one correction */
        reorth_pass(z, xr, j, Q, ldq, P, ldp, Rc, m, prec);
        if (reorth) reorth_pass(z, xr, j, Q, ldq, P, ldp, Rc, m, prec);
        if (variant != REF_HP) {
            mv_st(A, z, x, prec);
            *mv_calls += 1; *mv_cols += 1;
        }
        double rjj;
        if (!anorm(z, x, m, &rjj)) { info = (int)(j + 1); break; }
        Rc[j] = rjj;
        scale(z, z, rjj, m, prec);
        if (variant == REF_NAIVE) {
            mv_st(A, z, P + j * ldp, prec);
            *mv_calls += 1; *mv_cols += 1;
        } else {
            scale(P + j * ldp, x, rjj, m, prec);
        }
    }
    free(x);
    return info;
}

static int run(const ref_op *A, int64_t n, int64_t first, const double *Z, int64_t ldz,
               double *Q, int64_t ldq, double *R, int64_t ldr, double *P, int64_t ldp,
               int variant, int orientation, int reorth, int prec, int64_t *stats)
{
    int64_t m = A->m;
    if (m < 0 || n < 0 || n > m || ldz < m || ldq < m || ldr < n) return -1;
    if (variant < 0 || variant > 2 || orientation < 0 || orientation > 5) return -1;
    if (prec < 0 || prec > 1) return -1;
    if (reorth < 0 || reorth > 2 || (reorth == 2 && orientation != REF_PANEL2)) return -1;
    /* successive orthogonalisation: columns before first are final in Q, P
     * and R (column and classical forms only) */
    if (first < 0 || first > n) return -1;
    if (first > 0 && (!P || (orientation != REF_COL && orientation != REF_CGS))) return -1;
    if (n == 0) { if (stats) stats[0] = stats[1] = 0; return 0; }
    if (!Z || !Q || !R) return -1;
    /* a0: working copy (Q holds z_j^{(i)}), R zeroed; inputs rounded to storage */
    for (int64_t j = first; j < n; ++j)
        for (int64_t k = 0; k < m; ++k) Q[j * ldq + k] = st(Z[j * ldz + k], prec);
    for (int64_t j = first; j < n; ++j) memset(R + j * ldr, 0, (size_t)n * sizeof(double));
    double *Pw = P;
    int64_t ldpw = ldp;
    if (!Pw) { Pw = (double *)calloc((size_t)m * n, sizeof(double)); ldpw = m; }
    double *X = NULL;
    if (variant == REF_HP) X = (double *)malloc((size_t)m * n * sizeof(double));
    int64_t calls = 0, cols = 0;
    static const int one_level[1] = {4}, two_level[2] = {8, 4}, three_level[3] = {16, 8, 4};
    int info = orientation == REF_COL
        ? qr_col(A, m, n, first, Q, ldq, R, ldr, Pw, ldpw, X, variant, reorth, prec, &calls, &cols)
        : orientation == REF_ROW
        ? qr_row(A, m, n, Q, ldq, R, ldr, Pw, ldpw, X, variant, reorth, prec, &calls, &cols)
        : orientation == REF_PANEL
        ? qr_panel(A, m, n, Q, ldq, R, ldr, Pw, ldpw, X, variant, reorth, prec, 1, one_level,
                   &calls, &cols)
        : orientation == REF_PANEL2
        ? qr_panel(A, m, n, Q, ldq, R, ldr, Pw, ldpw, X, variant, reorth, prec, 2, two_level,
                   &calls, &cols)
        : orientation == REF_PANEL3
        ? qr_panel(A, m, n, Q, ldq, R, ldr, Pw, ldpw, X, variant, reorth, prec, 3, three_level,
                   &calls, &cols)
        : qr_cgs(A, m, n, first, Q, ldq, R, ldr, Pw, ldpw, X, variant, reorth, prec, &calls, &cols);
    if (stats) { stats[0] = calls; stats[1] = cols; }
    free(X);
    if (!P) free(Pw);
    return info;
}

/* Round a matrix in place to storage precision (inputs of precision 1). */
static double *rounded_copy(const double *v, int64_t len, int prec)
{
    double *c = (double *)malloc((size_t)(len > 0 ? len : 1) * sizeof(double));
    for (int64_t k = 0; k < len; ++k) c[k] = st(v[k], prec);
    return c;
}

/* ---------------------------------------------------------- exports */
/* Dense symmetric A (column-major, lda >= m).  Returns 0 on success, j >= 1 if
 * column j broke down (columns before j are valid), -1 on a bad argument.
 * stats (nullable, 2 entries): number of MV calls (a block product counts
 * once) and number of MV columns.  first > 0: columns before first are final
 * in Q, P and R on entry (successive orthogonalisation; column and classical
 * forms). */
int amgs_ref_qr_dense(int64_t m, const double *a, int64_t lda, int64_t n, const double *Z,
                      int64_t ldz, double *Q, int64_t ldq, double *R, int64_t ldr, double *P,
                      int64_t ldp, int variant, int orientation, int reorth, int precision,
                      int64_t *stats, int64_t first)
{
    if (!a || lda < m) return -1;
    ref_op A = {0};
    A.kind = 0; A.m = m; A.lda = lda;
    double *ar = NULL;
    if (precision == REF_FP32) { ar = rounded_copy(a, lda * m, precision); A.a = ar; }
    else A.a = a;
    int info = run(&A, n, first, Z, ldz, Q, ldq, R, ldr, P, ldp, variant, orientation, reorth,
                   precision, stats);
    free(ar);
    return info;
}

/* CSR symmetric A (int32 indices, columns ascending within each row). */
int amgs_ref_qr_csr(int64_t m, int64_t nnz, const int32_t *row_ptr, const int32_t *col_idx,
                    const double *vals, int64_t n, const double *Z, int64_t ldz, double *Q,
                    int64_t ldq, double *R, int64_t ldr, double *P, int64_t ldp, int variant,
                    int orientation, int reorth, int precision, int64_t *stats, int64_t first)
{
    if (!row_ptr || (nnz > 0 && (!col_idx || !vals))) return -1;
    if (row_ptr[0] != 0 || row_ptr[m] != nnz) return -1;
    ref_op A = {0};
    A.kind = 1; A.m = m; A.row_ptr = row_ptr; A.col_idx = col_idx;
    double *vr = NULL;
    if (precision == REF_FP32) { vr = rounded_copy(vals, nnz, precision); A.vals = vr; }
    else A.vals = vals;
    int info = run(&A, n, first, Z, ldz, Q, ldq, R, ldr, P, ldp, variant, orientation, reorth,
                   precision, stats);
    free(vr);
    return info;
}

/* Plain matrix-vector product with the same conventions (for tests). */
int amgs_ref_mv_csr(int64_t m, const int32_t *row_ptr, const int32_t *col_idx,
                    const double *vals, const double *v, double *y, int precision)
{
    ref_op A = {0};
    A.kind = 1; A.m = m; A.row_ptr = row_ptr; A.col_idx = col_idx; A.vals = vals;
    mv_st(&A, v, y, precision);
    return 0;
}

int amgs_ref_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
