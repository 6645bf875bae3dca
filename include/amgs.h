/*
 * amgs.h -- C ABI of the MI355X library for A-orthonormalising modified
 * Gram-Schmidt (Imakura & Yamamoto, "Efficient implementations of the
 * modified Gram-Schmidt orthogonalization with a non-standard inner
 * product").
 *
 * Problem (Section 1, eq. (1)): given Z (m x n, m >= n) and a symmetric
 * positive definite A (m x m), compute
 *         Z = Q R,    Q^T A Q = I_n,
 * with R upper triangular and positive on the diagonal.  The A-inner product
 * is (x, y)_A = x^T A y (Section 1, notation).
 *
 * Variants (Section 2):
 *   AMGS_NAIVE  Alg. 3: r_ij = p_i^T z_j with p_i = A q_i; two
 *               matrix-vector products (MV) per column, 2n MV in total.
 *   AMGS_HA     Alg. 5: p_j = x_j / r_jj (eq. (4)); n MV in total.
 *   AMGS_HP     Alg. 6: X = A Z as one block product, then
 *               x_j = x_j^{(0)} - sum_{i<j} r_ij p_i (eq. (5)).
 * Every variant returns the numbers of the column-oriented algorithm
 * (Alg. 3/5/6); the library schedules the same per-column operations in
 * right-looking order (Section 2.1 notes that both orders compute the same
 * values).
 *
 * Precisions:
 *   AMGS_FP64   everything in binary64.
 *   AMGS_FP32   A, Z, Q, P (= AQ) and the HP block X are binary32; MV and the
 *               projections r_ij = p_i^T z_j, z_j -= r_ij q_i, x_j -= r_ij p_i
 *               run in binary32 with binary32 accumulation; the squared
 *               A-norm z_j^T x_j is accumulated in binary64, and the square
 *               root and the divisions q_j = z_j / r_jj, p_j = x_j / r_jj are
 *               binary64 rounded once to binary32.  R is binary64.
 *
 * Optional second pass (opts->reorth = 1; the paper mentions
 * reorthogonalisation in Section 2.1 without defining it): after the MGS
 * projections of column j, s_i = p_i^T z_j for all i < j (binary64
 * accumulation), z_j -= sum_i s_i q_i (binary64, rounded once), r_ij += s_i;
 * for HP also x_j -= sum_i s_i p_i.
 *
 * Conventions shared by all entry points:
 *   - Matrices are column-major with a leading dimension (ld >= rows).
 *   - Every matrix/vector pointer passed to amgs_qr_* is DEVICE memory owned
 *     by the caller; the library never allocates, frees or synchronises
 *     inside amgs_qr_*: all work is enqueued on `stream` (a hipStream_t;
 *     NULL = the null stream).  Scratch memory is the caller's `work`
 *     buffer of at least amgs_workspace_bytes(...) bytes.
 *   - Z may alias Q (in-place, ldz == ldq).  Otherwise Z is read only.
 *   - R is n x n binary64 in both precisions; its strictly lower triangle is
 *     set to zero.
 *   - `info` is a device int32: 0 on success, j >= 1 if column j (1-based)
 *     had a squared A-norm that was not positive and finite (Z rank
 *     deficient, A not positive definite, or cancellation); columns before
 *     j are valid, later ones are not.  It is written asynchronously.
 *   - Synchronous errors: AMGS_ERR_ARG for invalid sizes, leading
 *     dimensions, enum values or null pointers; AMGS_ERR_WORKSPACE when
 *     work_bytes is too small; AMGS_ERR_HIP when a launch fails.
 *   - n == 0 is a no-op returning AMGS_OK.
 *   - A CSR matrix must be valid: row_ptr[0] = 0, non-decreasing,
 *     row_ptr[m] = nnz, 0 <= col_idx < m.  amgs_csr_check() verifies this on
 *     the device; the solver itself does not re-check indices.
 *   - One handle may be used from one host thread at a time.
 */
#ifndef AMGS_H
#define AMGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { AMGS_NAIVE = 0, AMGS_HA = 1, AMGS_HP = 2 } amgs_variant_t;
typedef enum { AMGS_FP64 = 0, AMGS_FP32 = 1 } amgs_precision_t;
typedef enum {
    AMGS_OK = 0,
    AMGS_ERR_ARG = -1,
    AMGS_ERR_WORKSPACE = -2,
    AMGS_ERR_HIP = -3,
    AMGS_ERR_UNSUPPORTED = -4
} amgs_status_t;

typedef struct amgs_handle *amgs_handle_t;

/* Per-call options; passing NULL means all zero.
 *   reorth  1: second (reorthogonalisation) pass per column (see above),
 *           in either schedule: it runs on column j after the column's
 *           projections and before its MV.
 *           2: blocked second pass, two-level panel schedule only (panel =
 *           8; any other panel value, 16 included, AMGS_ERR_UNSUPPORTED).  When an eight-panel [S, S + 8)
 *           starts, its columns have all their first-pass projections onto
 *           the columns before S; each of them then gets the second pass
 *           against all i < S at once (s_ic = p_i^T z_c in binary64,
 *           z_c -= sum_{i<S} s_ic q_i in binary64 rounded once, r_ic += s_ic,
 *           HP also x_c -= sum_{i<S} s_ic p_i), and column j of the panel
 *           gets the per-column pass above against [S, j) only.  The earlier
 *           columns are streamed once per eight-panel instead of once per
 *           column.  Other values are AMGS_ERR_ARG.
 *   panel   0: the column algorithm's own order of operations (default).
 *           4: panel schedule.  Columns are taken in panels of four; inside
 *           a panel every step is the column algorithm's.  The effect of a
 *           finished panel I on a later column c is applied as one block:
 *           with W = P_I^T z_c (z_c before panel I) and
 *           L = strict_lower(P_I^T Q_I), the coefficients r_{I,c} solve
 *           (I + L) r_{I,c} = W by forward substitution, which in exact
 *           arithmetic are the modified Gram-Schmidt coefficients
 *           r_ic = p_i^T z_c^{(i-1)}; then z_c -= Q_I r_{I,c}.  For HP the
 *           terms of eq. (5) reach each x_c in ascending i, every 8 columns
 *           as a block and the rest in the column step.  Each later column
 *           is then read and written once per panel instead of once per
 *           column.  Rounding differs from the column order;
 *           A-orthogonality stays at the level of the column algorithm.
 *           8: two-level panel schedule.  Columns are taken in panels of
 *           eight, each taken apart as two panels of four exactly as above
 *           except that a four-column block acts only on the columns of its
 *           own eight-panel; a finished eight-panel then acts on every later
 *           column as one block of eight (W = P_I^T z_c, L, (I + L) r = W as
 *           above, with eight columns).  A column receives the blocks of
 *           the earlier eight-panels, then the block of the earlier
 *           four-panel of its own eight-panel, then the column steps of its
 *           four-panel.  Each later column is read and written once per
 *           eight columns; the block step runs on the matrix cores.
 *           16: three-level panel schedule, naive and HA only (HP:
 *           AMGS_ERR_UNSUPPORTED).  Columns are taken in panels of sixteen,
 *           each taken apart as two eight-panels exactly as above except
 *           that an eight-column block acts only on the columns of its own
 *           sixteen-panel; a finished sixteen-panel acts on every later
 *           column as one block of sixteen (W, L, (I + L) r = W as above,
 *           with sixteen columns).  A column receives the blocks of the
 *           earlier sixteen-panels, then that of the earlier eight-panel
 *           of its own sixteen-panel, then the four-panel steps.  Each
 *           later column is read and written once per sixteen columns.
 *           reorth = 1 is supported, reorth = 2 is not
 *           (AMGS_ERR_UNSUPPORTED).
 *           Not combined with cgs or first (AMGS_ERR_UNSUPPORTED); other
 *           values are AMGS_ERR_ARG.
 *   cgs     0: modified Gram-Schmidt (Algs. 3/5/6, default).
 *           1: classical Gram-Schmidt with the same variants (Section 2, the
 *           n-MV idea applied to CGS: CGS-naive, CGS-HA, CGS-HP, column
 *           form): all coefficients of column j come from the unmodified
 *           column, r_ij = p_i^T z_j^{(0)} for i < j, then
 *           z_j^{(j-1)} = z_j^{(0)} - sum_{i<j} r_ij q_i (HP also
 *           x_j = x_j^{(0)} - sum_{i<j} r_ij p_i), with binary64 accumulation
 *           of the coefficients and of each corrected entry, rounded once to
 *           storage.  With reorth = 1 the classical step is applied twice
 *           (the second pass above), i.e. CGS2.  Other values are
 *           AMGS_ERR_ARG.
 *   first   successive orthogonalisation (Section 2.1 notes that the column
 *           form suits it): columns 0..first-1 are already A-orthonormal and
 *           final -- Q[:, <first] holds q_1..q_first, P (which must then be
 *           passed, else AMGS_ERR_ARG) holds their p_i, and R[:first, :first]
 *           their R; none of these is read from Z or written.  Columns
 *           first..n-1 of Z are orthonormalised against them and against
 *           each other, each receiving its projections in ascending i as in
 *           the column algorithm, so the new columns equal those of one call
 *           on all n columns.  0 <= first <= n (else AMGS_ERR_ARG); with
 *           panel != 0, AMGS_ERR_UNSUPPORTED. */
typedef struct {
    int32_t reorth;
    int32_t panel;
    int32_t cgs;
    int32_t first;
} amgs_opts_t;

/* Counters of the most recent amgs_qr_* call on a handle. */
typedef struct {
    int64_t mv_calls;        /* MV launches: 2n naive, n HA, 1 block product HP */
    int64_t mv_columns;      /* columns multiplied by A */
    int64_t kernel_launches; /* all kernels enqueued */
    int64_t sweep_launches;  /* projection-sweep kernels enqueued */
    double  sweep_bytes;     /* algorithmic HBM bytes of all sweeps (see below) */
    double  mv_bytes;        /* algorithmic HBM bytes of all MV / block products */
    int64_t block_sweep_launches; /* panel schedule: sweeps after a panel's last column */
    double  block_sweep_bytes;    /* their algorithmic HBM bytes (part of sweep_bytes) */
} amgs_stats_t;

/* Handle bound to a device (HIP ordinal).  Returns AMGS_ERR_ARG for a bad
 * ordinal or NULL out-pointer.  The handle holds device properties, launch
 * geometry and counters; destroying it frees nothing the caller owns. */
amgs_status_t amgs_create(amgs_handle_t *h, int device);
amgs_status_t amgs_destroy(amgs_handle_t h);

/* Bytes of device workspace needed by amgs_qr_csr (is_dense = 0) or
 * amgs_qr_dense (is_dense = 1) for these sizes; P_given = 1 if the caller
 * passes its own P (= AQ) buffer.  Returns 0 for invalid arguments.  The
 * workspace holds reduction partials, the HP block X, P when not given and,
 * for CSR with the naive and HA variants, a padded copy of up to 8 entries
 * per row of A that the column MV reads.  That copy comes last and takes
 * 8 m (4 + element size) + 4 ceil(m / 512) bytes, each of the three parts
 * rounded up to a multiple of 256.  A workspace that lacks exactly that room
 * is still accepted: the column MV then reads the CSR arrays directly
 * (slower for rows of at most 8 entries, the same results bit for bit).
 * The contents need not be preserved between calls. */
size_t amgs_workspace_bytes(amgs_handle_t h, int64_t m, int64_t n, int32_t is_dense,
                            amgs_variant_t v, amgs_precision_t p, int32_t P_given,
                            const amgs_opts_t *o);

/* Z = QR, Q^T A Q = I for CSR A (Alg. 3 / 5 / 6, eq. (1)).
 *   row_ptr[m+1], col_idx[nnz]: int32; vals[nnz]: binary64 (AMGS_FP64) or
 *   binary32 (AMGS_FP32), matching `p`.  Z, Q, P: element type of `p`.
 *   m <= 2^31 - 1 and nnz <= 2^31 - 1025 (int32 indices with headroom for
 *   the kernels' entry stepping), else AMGS_ERR_ARG.
 *   P (nullable, ld ldp): receives the auxiliary vectors p_j = A q_j
 *   (Section 2.1); when NULL the workspace holds them. */
amgs_status_t amgs_qr_csr(amgs_handle_t h, int64_t m, int64_t nnz, const int32_t *row_ptr,
                          const int32_t *col_idx, const void *vals, int64_t n,
                          const void *Z, int64_t ldz, void *Q, int64_t ldq, double *R,
                          int64_t ldr, void *P, int64_t ldp, amgs_variant_t v,
                          amgs_precision_t p, const amgs_opts_t *o, void *work,
                          size_t work_bytes, int32_t *info, void *stream);

/* Size of the per-GPU static scratch array of amgs_qr_csr_static: 64 MiB. */
#define AMGS_STATIC_SCRATCH_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation, arguments and results as amgs_qr_csr, without the work /
 * work_bytes pair.  The workspace is a static device array of
 * AMGS_STATIC_SCRATCH_BYTES bytes that the library holds on every GPU it
 * runs on until the process ends (its address is looked up once per device
 * by amgs_create).  The call allocates and frees nothing and never
 * synchronises; the caller still passes every input and output buffer.
 *   - Size limit: AMGS_ERR_WORKSPACE, before any launch, when the
 *     workspace these sizes need without the padded copy of A (see
 *     amgs_workspace_bytes) exceeds AMGS_STATIC_SCRATCH_BYTES.  When the
 *     array also holds the padded copy the column MV reads it, else CSR
 *     directly; results equal amgs_qr_csr's bit for bit either way.
 *   - Sharing: every call on one GPU uses that GPU's one array, which keeps
 *     the previous call's contents (nothing in it needs to start at zero).
 *     Calls that overlap on one GPU -- on two streams, from two host
 *     threads, or two graphs replayed concurrently -- race on it; order
 *     them on one stream or with events.
 *   - AMGS_ERR_UNSUPPORTED for a device ordinal of 64 or more (no scratch
 *     address kept for it). */
amgs_status_t amgs_qr_csr_static(amgs_handle_t h, int64_t m, int64_t nnz,
                                 const int32_t *row_ptr, const int32_t *col_idx,
                                 const void *vals, int64_t n, const void *Z, int64_t ldz, void *Q,
                                 int64_t ldq, double *R, int64_t ldr, void *P, int64_t ldp,
                                 amgs_variant_t v, amgs_precision_t p, const amgs_opts_t *o,
                                 int32_t *info, void *stream);

/* Same for a dense symmetric A (column-major, lda >= m); the block product
 * X = A Z of HP (Alg. 6) runs on the matrix cores. */
amgs_status_t amgs_qr_dense(amgs_handle_t h, int64_t m, const void *A, int64_t lda, int64_t n,
                            const void *Z, int64_t ldz, void *Q, int64_t ldq, double *R,
                            int64_t ldr, void *P, int64_t ldp, amgs_variant_t v,
                            amgs_precision_t p, const amgs_opts_t *o, void *work,
                            size_t work_bytes, int32_t *info, void *stream);

/* Device-side CSR validation: writes 0 to *flag if the structure is valid,
 * 1 otherwise (flag is device int32). */
amgs_status_t amgs_csr_check(amgs_handle_t h, int64_t m, int64_t nnz, const int32_t *row_ptr,
                             const int32_t *col_idx, int32_t *flag, void *stream);

/* ---------------------------------------------------------------------
 * Batched form: many independent problems (each its own CSR A_k, Z_k) in
 * one persistent launch replayed from a HIP graph.  Each instance is the
 * single-problem computation above (Alg. 5 or 6) on one workgroup.
 * ------------------------------------------------------------------- */
typedef struct {
    int64_t m, n, nnz;          /* instance sizes (m >= n >= 1) */
    const int32_t *row_ptr;     /* device, m+1 */
    const int32_t *col_idx;     /* device, nnz */
    const void *vals;           /* device, nnz, element type of the precision */
    const void *Z; int64_t ldz; /* device, read only (may alias Q) */
    void *Q; int64_t ldq;       /* device, output */
    double *R; int64_t ldr;     /* device, output n x n */
} amgs_batch_desc_t;

typedef struct amgs_batch_plan *amgs_batch_plan_t;

/* Build a plan for `batch` instances with sizes m_host[k], n_host[k] (host
 * arrays): largest-first work order, per-size-class kernel tiles chosen by
 * the autotuner (autotune = 1 times the candidates on the device with
 * synthetic data of the same shapes; 0 uses the built-in table).  The plan
 * owns its small device tables.  Returns AMGS_ERR_ARG on invalid sizes. */
amgs_status_t amgs_batch_plan_create(amgs_handle_t h, int32_t batch, const int64_t *m_host,
                                     const int64_t *n_host, amgs_variant_t v,
                                     amgs_precision_t p, const amgs_opts_t *o,
                                     int32_t autotune, amgs_batch_plan_t *plan);
amgs_status_t amgs_batch_plan_destroy(amgs_batch_plan_t plan);
/* Device workspace bytes the plan needs (P and X blocks of every instance). */
size_t amgs_batch_workspace_bytes(amgs_batch_plan_t plan);

/* Run every instance of the plan: desc is a DEVICE array of `batch`
 * descriptors in the order the sizes were given; info is a DEVICE int32
 * array of `batch` entries (per-instance breakdown index, 0 = success).
 * desc[k].m and desc[k].n must be the sizes the plan was created with: the
 * plan's workspace offsets are laid out for them, and the descriptors are
 * device memory, which the call does not read back to check.
 * The first call for a given (desc, work, info) captures the launch into a
 * HIP graph; later calls replay it on the stream they pass.  Every pass of a
 * plan uses the plan's one work-queue counter, so a pass waits (on the
 * device) for the previous pass of the same plan to end, whatever stream
 * either was enqueued on; a call made while `stream` is being captured
 * leaves that ordering to the caller's graph.  One plan may be used from one
 * host thread at a time. */
amgs_status_t amgs_qr_batched(amgs_batch_plan_t plan, const amgs_batch_desc_t *desc,
                              void *work, size_t work_bytes, int32_t *info, void *stream);

/* Tile chosen for each size class (written to out[0..nclass-1] as packed
 * integers; returns the number of classes). */
int32_t amgs_batch_plan_tiles(amgs_batch_plan_t plan, int32_t *out, int32_t cap);

/* ---------------------------------------------------------------------
 * Introspection
 * ------------------------------------------------------------------- */
amgs_status_t amgs_get_stats(amgs_handle_t h, amgs_stats_t *out);
const char *amgs_status_string(amgs_status_t s);

/* Kernel timing with HIP events recorded on the call's stream around each
 * launch of a kernel category (0 = projection sweep, 1 = MV / column
 * kernels, 2 = block product X = AZ, 3 = the panel schedule's block sweep
 * after a panel's last column, which also counts in category 0).
 * amgs_profile_enable(h, 1) starts recording for subsequent calls;
 * amgs_profile_read() synchronises on the recorded events and returns the
 * summed milliseconds and launch count of a category since the last reset
 * (AMGS_ERR_ARG for a category outside 0..3). */
amgs_status_t amgs_profile_enable(amgs_handle_t h, int32_t on);
amgs_status_t amgs_profile_read(amgs_handle_t h, int32_t category, double *total_ms,
                                int64_t *launches);
amgs_status_t amgs_profile_reset(amgs_handle_t h);

#ifdef __cplusplus
}
#endif
#endif /* AMGS_H */
