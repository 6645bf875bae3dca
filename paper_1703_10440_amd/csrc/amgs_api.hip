// amgs_api.hip -- host side of the C ABI declared in include/amgs.h:
// argument checks, workspace layout, and the per-column launch schedule of
// the single-problem solver.
#include <hip/hip_runtime.h>

#include <mutex>
#include <new>
#include <vector>

#include "../../include/amgs.h"
#include "amgs_internal.h"
#include "amgs_batched.h"
#include "amgs_handle.h"

// Scratch of amgs_qr_csr_static: a file-scope device array, one copy per
// GPU at that GPU's own address, held by the loaded code object until the
// process ends.  On the host the name is only a stand-in for the symbol, not
// a device address, so host code never hands it to a kernel or a copy:
// amgs_create looks up each device's address once, with that device
// current, and every later use goes through the pointer kept for it.
__device__ __align__(256) char scratch[AMGS_STATIC_SCRATCH_BYTES];

namespace {

using namespace amgs;

constexpr int SCRATCH_MAX_DEV = 64;
std::mutex g_scratch_mu;
void *g_scratch[SCRATCH_MAX_DEV];   // device address of `scratch` per ordinal

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev)
    {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard()
    {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

hipEvent_t take_event(amgs_handle *h)
{
    if (!h->pool.empty()) {
        hipEvent_t e = h->pool.back();
        h->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Records an event pair around one launch when profiling is on.
struct ProfScope {
    amgs_handle *h;
    int cat;
    hipStream_t s;
    hipEvent_t a = nullptr, b = nullptr;
    ProfScope(amgs_handle *h_, int cat_, hipStream_t s_) : h(h_), cat(cat_), s(s_)
    {
        if (!h->profiling || cat < 0) return;
        a = take_event(h);
        b = take_event(h);
        if (a && b) (void)hipEventRecord(a, s);
    }
    ~ProfScope()
    {
        if (!h->profiling || cat < 0 || !a || !b) return;
        (void)hipEventRecord(b, s);
        h->recs.push_back({cat, a, b, -1});
    }
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct Layout {
    size_t part, s_part, rr_part, S, zt, xv, X, P, wpart, lpart, lpart8, wred, rb_part, rb_s,
        ell_col, ell_val, tile_long, ell_d16, ell_wide;
    size_t base;    // bytes without the padded copy of A
    size_t total;   // bytes with it (the size the query reports)
};

// Row chunks of the panel-schedule sweeps (256 threads of panel_rows rows).
int64_t panel_chunks(int64_t m, size_t w)
{
    const int64_t rows = 256 * (int64_t)panel_rows_for(w == 8);
    const int64_t g = (m + rows - 1) / rows;
    return g < 1 ? 1 : g;
}

Layout layout(int64_t m, int64_t n, const Geo &g, int variant, size_t w, int P_given, int reorth,
              int panel, int is_dense)
{
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align256(bytes);
        return o;
    };
    // MV kernels never use more than MAX_G_MV workgroups, whatever the CSR
    // lane count, so the size does not depend on nnz
    int64_t g_rr = g.g_rows1 > MAX_G_MV ? g.g_rows1 : MAX_G_MV;
    const int64_t g_p = panel ? panel_chunks(m, w) : 0;
    L.part = take((size_t)n * (panel ? g_p : g.g_rows) * 8);
    L.s_part = reorth ? take((size_t)n * g.g_rows2 * 8) : off;
    L.rr_part = take((size_t)g_rr * 8);
    L.S = reorth ? take((size_t)n * 8) : off;
    L.zt = (variant != VAR_HP || reorth) ? take((size_t)m * w) : off;
    L.xv = variant != VAR_HP ? take((size_t)m * w) : off;
    L.X = variant == VAR_HP ? take((size_t)m * n * w) : off;
    L.P = P_given ? off : take((size_t)m * n * w);
    // two levels (panel 8) or three (panel 16): block sweeps of width 8, and
    // of 16 for three levels
    const bool two = panel == PANEL_B1 || panel == PANEL_B2;
    const size_t pb = panel == PANEL_B2 ? PANEL_B2 : two ? PANEL_B1 : PANEL_B;
    // the outer block sweep may use more row chunks than the panel sweeps
    // (its partials are stored in XCD order: the chunk count rounded up to
    // a multiple of 8 entries each)
    const int64_t g_b = two ? (bsweep_chunks(m, w) + 7) / 8 * 8 : 0;
    const int64_t g_w = g_b > g_p ? g_b : g_p;
    L.wpart = panel ? take((size_t)n * pb * g_w * 8) : off;
    L.lpart = panel ? take((size_t)PANEL_B * PANEL_B * g_p * 8) : off;
    L.lpart8 = two ? take((size_t)pb * pb * g_b * 8) : off;
    L.wred = two ? take((size_t)(n * pb + pb * pb) * 8 * 8) : off;
    // blocked second pass: coefficient partials and coefficients of an outer panel
    const bool rb = two && reorth == 2;
    L.rb_part = rb ? take((size_t)n * PANEL_B1 * g_b * 8) : off;
    L.rb_s = rb ? take((size_t)n * PANEL_B1 * 8) : off;
    L.base = off;
    // padded copy of a CSR A for the column MV (naive and HA), last, so that
    // a smaller workspace can leave it out; the size does not depend on nnz,
    // which only decides whether the copy is used
    const bool ell = !is_dense && variant != VAR_HP;
    L.ell_col = ell ? take((size_t)ELL_K * m * 4) : off;
    L.ell_val = ell ? take((size_t)ELL_K * m * w) : off;
    L.tile_long = ell ? take((size_t)((m + MV_TILE - 1) / MV_TILE) * 4) : off;
    L.ell_d16 = ell ? take((size_t)ELL_K * m * 2) : off;
    L.ell_wide = ell ? take(4) : off;
    L.total = off;
    return L;
}

bool valid_enums(amgs_variant_t v, amgs_precision_t p)
{
    return (v == AMGS_NAIVE || v == AMGS_HA || v == AMGS_HP) && (p == AMGS_FP64 || p == AMGS_FP32);
}

// Algorithmic HBM bytes of one sweep at step j (see the design notes): each
// later column is read and written once (read only at j = 0), plus the
// vectors q_{j-1}, z_j, x_j (or p_j) read and q_j, p_j written.
double sweep_bytes(int64_t m, int64_t n, int64_t j, size_t w, int variant)
{
    const double ncols = (double)(n - j - 1);
    const double per_col = (j > 0 ? 2.0 : 1.0) * (double)m * (double)w;
    double vec = 2.0 + (j > 0 ? 1.0 : 0.0) + (variant == VAR_NAIVE ? 0.0 : 1.0) + 1.0;
    return ncols * per_col + vec * (double)m * (double)w;
}

template <typename T>
amgs_status_t run_panel(amgs_handle *h, Ctx &c, int variant, int reorth);

template <typename T>
amgs_status_t run_cgs(amgs_handle *h, Ctx &c, int variant, int reorth);

template <typename T>
amgs_status_t run_single(amgs_handle *h, Ctx &c, int variant, int reorth)
{
    if (c.panel) return run_panel<T>(h, c, variant, reorth);
    if (c.cgs) return run_cgs<T>(h, c, variant, reorth);
    const size_t w = sizeof(T);
    amgs_stats_t &st = h->stats;
    st = amgs_stats_t{};
    launch_init<T>(c, c.Z != c.Q ? c.n - c.first : 0);
    st.kernel_launches++;
    if (c.ell_k) {
        launch_csr_to_ell<T>(c);
        st.kernel_launches++;
    }
    const double mvA = c.is_dense ? (double)c.m * (double)c.m * w
                                  : (double)c.nnz * (w + 4) + 4.0 * (double)(c.m + 1);
    if (variant == VAR_HP) {
        ProfScope ps(h, 2, c.stream);
        if (c.is_dense) launch_dense_gemm<T>(c);
        else launch_csr_spmm<T>(c);
        st.kernel_launches++;
        st.mv_calls += 1;
        st.mv_columns += c.n - c.first;
        st.mv_bytes += mvA + 2.0 * (double)c.m * (c.n - c.first) * w;
    }
    // successive orthogonalisation: the final columns j < first project the
    // new columns in the same right-looking order (no column kernel, so the
    // finished row r_{j-1, first..} is published by a small kernel)
    for (int64_t j = 0; j < c.first; ++j) {
        if (j > 0) {
            launch_publish<T>(c, j - 1);
            st.kernel_launches++;
        }
        launch_sweep<T>(c, j, variant, 0);
        st.kernel_launches++;
        st.sweep_launches++;
        if (variant == VAR_HP && launch_hp_xblock<T>(c, j, j + 1)) st.kernel_launches++;
    }
    for (int64_t j = c.first; j < c.n; ++j) {
        int64_t n_rr;
        {
            ProfScope ps(h, variant == VAR_HP ? 1 : -1, c.stream);
            if (variant == VAR_HP) {
                if (reorth && j > 0) {
                    launch_col_hp<T>(c, j, true);
                    launch_reorth_fin(c, j);
                    launch_reorth_b<T>(c, j, true);
                    st.kernel_launches += 3;
                    n_rr = c.geo.g_rows1;   // A-norm partials of k_reorth_b
                } else {
                    launch_col_hp<T>(c, j, false);
                    st.kernel_launches += 1;
                    n_rr = c.geo.g_rows2;
                }
            } else {
                // with profiling on, the column MV (category 1) is timed with
                // events bound to its dispatch
                hipEvent_t m0 = nullptr, m1 = nullptr;
                if (h->profiling) {
                    m0 = take_event(h);
                    m1 = take_event(h);
                }
                if (reorth && j > 0) {
                    launch_reorth_a<T>(c, j);
                    launch_reorth_fin(c, j);
                    launch_reorth_b<T>(c, j, false);
                    c.ev_start = m0;
                    c.ev_stop = m1;
                    launch_mv<T>(c, j, SRC_VEC);
                    st.kernel_launches += 4;
                } else {
                    c.ev_start = m0;
                    c.ev_stop = m1;
                    launch_mv<T>(c, j, SRC_UPD);
                    st.kernel_launches += 1;
                }
                c.ev_start = c.ev_stop = nullptr;
                if (m0 && m1) h->recs.push_back({1, m0, m1, -1});
                st.mv_calls += 1;
                st.mv_columns += 1;
                // A once; z_j and q_{j-1} read (z_j only at j = 0, or the
                // corrected column after the second pass), x_j and z_j written
                // (x_j only after the second pass)
                const double vecs = (reorth && j > 0) ? 2.0 : (j > 0 ? 4.0 : 3.0);
                st.mv_bytes += mvA + vecs * (double)c.m * w;
                if (variant == VAR_NAIVE) {
                    launch_mv<T>(c, j, SRC_DIV);
                    st.kernel_launches += 1;
                    st.mv_calls += 1;
                    st.mv_columns += 1;
                    st.mv_bytes += mvA + 2.0 * (double)c.m * w;
                }
                n_rr = c.n_rr_mv;
            }
        }
        if (h->profiling) {
            // events bound to the sweep's own dispatch: exact kernel time
            hipEvent_t e0 = take_event(h), e1 = take_event(h);
            c.ev_start = e0;
            c.ev_stop = e1;
            launch_sweep<T>(c, j, variant, n_rr);
            c.ev_start = c.ev_stop = nullptr;
            if (e0 && e1) h->recs.push_back({0, e0, e1, -1});
        } else {
            launch_sweep<T>(c, j, variant, n_rr);
        }
        st.kernel_launches++;
        if (variant == VAR_HP) {
            ProfScope ps(h, 1, c.stream);
            if (launch_hp_xblock<T>(c, j, j + 1)) st.kernel_launches++;
        }
        st.sweep_launches++;
        st.sweep_bytes += sweep_bytes(c.m, c.n, j, w, variant);
    }
    if (hipGetLastError() != hipSuccess) return AMGS_ERR_HIP;
    return AMGS_OK;
}

// Algorithmic HBM bytes of one panel-schedule sweep: each later column is
// read, and written back when a pending update applies (for HP with its x
// column); plus z_j and x_j read, q_j and p_j written (naive: p_j read), the
// pending q_k (HP: and p_k) and the dot vectors p_d, d < j, read.
double psweep_bytes(int64_t m, size_t w, int64_t ncols, int64_t kw, int64_t bd, int variant)
{
    const double col = (double)m * (double)w;
    double per_col = kw > 0 ? 2.0 : 1.0;
    double vec = (variant == VAR_NAIVE ? 3.0 : 4.0) + (double)kw + (double)(bd - 1);
    return (double)ncols * per_col * col + vec * col;
}

// Panel schedule (opts->panel).  One level (panel = 4): the column
// algorithm inside each panel of PANEL_B columns; after a panel's last column
// one sweep applies the previous panel to every later column and forms the
// dots with this panel's p vectors, and k_pfin turns them into the
// coefficients r_{I,c}.  Two levels (panel = 8): outer panels of PANEL_B1
// columns, each taken apart as inner panels of PANEL_B exactly as above but
// with the inner blocks acting only on the columns of the same outer panel;
// after an outer panel's last column, k_bsweep applies the previous outer
// panel to every later column and forms the dots with this outer panel's p
// vectors, and k_wred + k_pfin2 solve for the coefficients.  A column thus
// receives the blocks of the earlier outer panels, then the block of the
// earlier inner panel of its own outer panel, then the column steps of its
// inner panel (the order of the two-level panel reading of the method).
// Three levels (panel = 16, naive and HA): sixteen-panels taken apart as two
// eight-panels exactly as above, the eight-column block acting only inside
// its sixteen-panel (a dots-only k_bsweep over the other eight columns);
// after a sixteen-panel, k_bsweep of width 16 over every later column; and
// before one, an update-only k_bsweep applies the previous sixteen-panel to
// its own columns, so the column kernels never hold a pending block wider
// than eight.
template <typename T>
amgs_status_t run_panel(amgs_handle *h, Ctx &c, int variant, int reorth)
{
    const size_t w = sizeof(T);
    amgs_stats_t &st = h->stats;
    st = amgs_stats_t{};
    // two levels: the later columns' first read is in the block sweep after
    // the second eight-panel, which takes them from Z (from_z below), so only
    // the first two eight-panels are copied; three levels: the second
    // sixteen-panel's columns are first read by the update-only sweep before
    // it, and the later ones by the sweep after it, both from Z, so only the
    // first sixteen-panel is copied
    {
        const int64_t keep = c.panel == PANEL_B2 ? PANEL_B2 : c.panel == PANEL_B1 ? 2 * PANEL_B1 : c.n;
        launch_init<T>(c, c.Z == c.Q ? 0 : c.n > keep ? keep : c.n);
    }
    st.kernel_launches++;
    if (c.ell_k) {
        launch_csr_to_ell<T>(c);
        st.kernel_launches++;
    }
    const double mvA = c.is_dense ? (double)c.m * (double)c.m * w
                                  : (double)c.nnz * (w + 4) + 4.0 * (double)(c.m + 1);
    if (variant == VAR_HP) {
        ProfScope ps(h, 2, c.stream);
        if (c.is_dense) launch_dense_gemm<T>(c);
        else launch_csr_spmm<T>(c);
        st.kernel_launches++;
        st.mv_calls += 1;
        st.mv_columns += c.n;
        st.mv_bytes += mvA + 2.0 * (double)c.m * c.n * w;
    }
    static_assert(HP_XB % PANEL_B == 0 && HP_XB % PANEL_B1 == 0,
                  "x-block passes fall on (outer) panel boundaries");
    // three levels: 16-panels taken apart as 8-panels, each as two 4-panels
    const bool three = c.panel == PANEL_B2;
    const bool two = c.panel == PANEL_B1 || three;
    const int64_t B = PANEL_B;
    const int64_t B1 = two ? PANEL_B1 : PANEL_B;   // 8-panel width (= B for one level)
    const int64_t B2 = PANEL_B2;
    // launch with HIP events bound to the dispatch when profiling (category
    // 0, and 3 for the block sweep after an outer panel)
    auto profiled = [&](bool block, auto &&launch) {
        if (h->profiling) {
            hipEvent_t e0 = take_event(h), e1 = take_event(h);
            c.ev_start = e0;
            c.ev_stop = e1;
            launch();
            c.ev_start = c.ev_stop = nullptr;
            if (e0 && e1) h->recs.push_back({0, e0, e1, block ? 3 : -1});
        } else {
            launch();
        }
    };
    // blocked second pass (reorth = 2, two levels only): each outer panel's
    // columns first get the previous outer panel's block, then the second
    // pass against every earlier column at once; the per-column pass then
    // covers only the earlier columns of the outer panel
    const bool blk = two && c.reorth_blk;
    for (int64_t S = 0; S < c.n; S += B1) {
        const int64_t E = S + B1 < c.n ? S + B1 : c.n;
        const int64_t bp0 = S > 0 ? S - B1 : S;   // the previous outer panel [bp0, S)
        // three levels: the 16-panel [S16, E16) of this 8-panel; before its
        // first 8-panel, the previous 16-panel's block is applied to its
        // columns (a 16-wide block is too wide for the column-step kernels)
        const int64_t S16 = three ? S / B2 * B2 : S;
        const int64_t E16 = three ? (S16 + B2 < c.n ? S16 + B2 : c.n) : E;
        if (three && S == S16 && S16 > 0) {
            profiled(false, [&] {
                launch_bsweep<T>(c, S16 - B2, S16, S16, S16, S16, E16, S16 < 2 * B2, PANEL_B2);
            });
            st.kernel_launches++;
            st.sweep_launches++;
            st.sweep_bytes += ((double)(E16 - S16) * 2.0 + (double)B2) * (double)c.m * w;
        }
        if (blk && S > 0) {
            profiled(false, [&] { launch_bsweep<T>(c, bp0, S, S, S, S, E); });
            launch_rb<T>(c, S, E, variant);
            st.kernel_launches += 4;
            st.sweep_launches++;
            st.sweep_bytes += (double)(E - S) * 2.0 * (double)c.m * w + (double)(S - bp0) * (double)c.m * w;
        }
        c.re_lo = blk ? S : 0;
        // the outer block still pending for this panel's columns (three
        // levels: the first 8-panel of its 16-panel has none left, the
        // second has the first)
        const int64_t ob0 = (blk || (three && S == S16)) ? S : bp0;
        for (int64_t s = S; s < E; s += B) {
            const int64_t e = s + B < E ? s + B : E;
            // the block still pending for this panel's columns: the previous
            // outer panel for the first inner panel, else the previous inner one
            const int64_t pk0 = s == S ? ob0 : s - B, pk1 = s;
            for (int64_t j = s; j < e; ++j) {
                // (with the blocked pass, and with three levels at the start
                // of a 16-panel, the first column of an outer panel has no
                // pending term either: it takes the same block-step path)
                const bool first_blk = j == s && (pk1 > pk0 || (j == S && S > 0 && ob0 == S));
                int64_t n_rr = 0;
                // column kernels publish r_{j-1,c} only inside the panel
                c.n_pub = e;
                {
                    ProfScope ps(h, variant == VAR_HP ? 1 : -1, c.stream);
                    // the optional second pass runs on column j after its
                    // projections, before its MV, as in the column schedule
                    const bool ro = reorth && j > c.re_lo;
                    if (first_blk) {
                        // HP: the x terms of the pending block unless an
                        // x-block pass at s has applied them
                        launch_pcol_blk<T>(c, variant, j, pk0, pk1, s % HP_XB == 0 ? s : pk0);
                        st.kernel_launches++;
                        n_rr = pcol_blk_partials(c);
                        if (ro) {
                            // the block-corrected z_j is in zt (naive, HA) or in
                            // Q (HP), with no single pending term left
                            c.no_pend = 1;
                            c.z_in_zt = variant == VAR_HP ? 0 : 1;
                            launch_reorth_a<T>(c, j);
                            c.no_pend = 0;
                            c.z_in_zt = 0;
                            launch_reorth_fin(c, j);
                            launch_reorth_b<T>(c, j, variant == VAR_HP);
                            st.kernel_launches += 3;
                            n_rr = c.geo.g_rows1;   // A-norm partials of k_reorth_b (HP)
                        }
                    } else if (variant == VAR_HP) {
                        // the recurrence terms since the last x-block pass
                        if (ro) {
                            launch_col_hp<T>(c, j, true);
                            launch_reorth_fin(c, j);
                            launch_reorth_b<T>(c, j, true);
                            st.kernel_launches += 3;
                            n_rr = c.geo.g_rows1;
                        } else {
                            launch_col_hp<T>(c, j, false);
                            st.kernel_launches++;
                            n_rr = c.geo.g_rows2;
                        }
                    } else if (ro) {
                        launch_reorth_a<T>(c, j);
                        launch_reorth_fin(c, j);
                        launch_reorth_b<T>(c, j, false);
                        st.kernel_launches += 3;
                    }
                    if (variant != VAR_HP) {
                        hipEvent_t m0 = nullptr, m1 = nullptr;
                        if (h->profiling) {
                            m0 = take_event(h);
                            m1 = take_event(h);
                        }
                        c.ev_start = m0;
                        c.ev_stop = m1;
                        launch_mv<T>(c, j, (first_blk || ro) ? SRC_VEC : SRC_UPD);
                        c.ev_start = c.ev_stop = nullptr;
                        if (m0 && m1) h->recs.push_back({1, m0, m1, -1});
                        st.kernel_launches++;
                        st.mv_calls += 1;
                        st.mv_columns += 1;
                        st.mv_bytes += mvA + ((first_blk || ro) ? 2.0 : (j > 0 ? 4.0 : 3.0)) * (double)c.m * w;
                        if (variant == VAR_NAIVE) {
                            launch_mv<T>(c, j, SRC_DIV);
                            st.kernel_launches++;
                            st.mv_calls += 1;
                            st.mv_columns += 1;
                            st.mv_bytes += mvA + 2.0 * (double)c.m * w;
                        }
                        n_rr = c.n_rr_mv;
                    }
                }
                c.n_pub = c.n;
                // the sweep of step j: inside a panel (also the last column
                // of the matrix); after an inner panel of an outer one (the
                // block of the inner panel for the rest of the outer panel);
                // after an outer panel (one level: the block sweep itself;
                // two levels: normalisation and the L row only, k_bsweep follows)
                const bool inner_end = j == e - 1 && e < E;
                const bool outer_end = j == e - 1 && e == E && E < c.n;
                int64_t k0, k1, d0, c0, c1;
                if (inner_end) {
                    k0 = pk0; k1 = pk1; d0 = s; c0 = e; c1 = E;
                } else if (outer_end && two) {
                    k0 = k1 = j; d0 = j; c0 = c1 = E;
                } else if (outer_end) {
                    k0 = bp0; k1 = S; d0 = s; c0 = E; c1 = c.n;
                } else {
                    k0 = j == s ? pk0 : j - 1;
                    k1 = j == s ? pk1 : j;
                    d0 = j; c0 = j + 1; c1 = e;
                }
                const bool block1 = outer_end && !two;
                profiled(block1, [&] { launch_psweep<T>(c, variant, j, k0, k1, d0, s, c0, c1, n_rr); });
                st.kernel_launches++;
                st.sweep_launches++;
                const double pb = psweep_bytes(c.m, w, c1 > c0 ? c1 - c0 : 0, k1 - k0, j - d0 + 1, variant);
                st.sweep_bytes += pb;
                if (block1) {
                    st.block_sweep_launches++;
                    st.block_sweep_bytes += pb;
                }
                if (inner_end) {
                    launch_pfin<T>(c, s, e, E);
                    st.kernel_launches++;
                }
                if (outer_end && three) {
                    if (E < E16) {
                        // the first 8-panel of a 16-panel: its block's dots
                        // for the other 8-panel only
                        profiled(false, [&] { launch_bsweep<T>(c, S, S, S, E, E, E16, false, PANEL_B1); });
                        launch_pfin2<T>(c, S, E, E, E16, PANEL_B1);
                        st.kernel_launches += 3;
                        st.sweep_launches++;
                        st.sweep_bytes += ((double)(E16 - E) + (double)(E - S)) * (double)c.m * w;
                    } else {
                        // a finished 16-panel: the previous 16-panel's block
                        // on every later column and this one's dots; the
                        // columns from E16 on are read from Z until they are
                        // first written (the first two 16-panels)
                        const int64_t k0b = S16 > 0 ? S16 - B2 : S16;
                        profiled(true, [&] {
                            launch_bsweep<T>(c, k0b, S16, S16, E16, E16, c.n, S16 < 2 * B2, PANEL_B2);
                        });
                        const double col = (double)c.m * (double)w;
                        const double bb = (double)(c.n - E16) * (S16 > k0b ? 2.0 : 1.0) * col
                                          + (double)((S16 - k0b) + (E16 - S16)) * col;
                        st.kernel_launches++;
                        st.sweep_launches++;
                        st.sweep_bytes += bb;
                        st.block_sweep_launches++;
                        st.block_sweep_bytes += bb;
                        launch_pfin2<T>(c, S16, E16, E16, c.n, PANEL_B2);
                        st.kernel_launches += 2;
                    }
                } else if (outer_end) {
                    if (two) {
                        // [E, n) lacks the block [bp0, S) also with blk; after the
                        // first two eight-panels the columns from E on have never
                        // been written and are read from Z
                        profiled(true, [&] { launch_bsweep<T>(c, bp0, S, S, E, E, c.n, S < 2 * B1); });
                        const double col = (double)c.m * (double)w;
                        const double bb = (double)(c.n - E) * (S > bp0 ? 2.0 : 1.0) * col
                                          + (double)((S - bp0) + (E - S)) * col;
                        st.kernel_launches++;
                        st.sweep_launches++;
                        st.sweep_bytes += bb;
                        st.block_sweep_launches++;
                        st.block_sweep_bytes += bb;
                        launch_pfin2<T>(c, S, E, E, c.n);
                        st.kernel_launches += 2;
                    } else {
                        launch_pfin<T>(c, s, e, c.n);
                        st.kernel_launches++;
                    }
                    // HP: once r_{i,c} of the last HP_XB columns are final,
                    // their recurrence terms go to every x column from E on
                    if (variant == VAR_HP && launch_hp_xblock<T>(c, E, E)) st.kernel_launches++;
                }
            }
        }
    }
    c.re_lo = 0;
    if (hipGetLastError() != hipSuccess) return AMGS_ERR_HIP;
    return AMGS_OK;
}

// Classical Gram-Schmidt (opts->cgs): per column j, the coefficients
// r_ij = p_i^T z_j^{(0)} of all i < j from the unmodified column (one pass
// over P_{<j}), z_j -= sum_i r_ij q_i (HP: x_j -= sum_i r_ij p_i), optionally
// a second such pass, then the column MV (naive / HA) and the normalisation.
template <typename T>
amgs_status_t run_cgs(amgs_handle *h, Ctx &c, int variant, int reorth)
{
    const size_t w = sizeof(T);
    amgs_stats_t &st = h->stats;
    st = amgs_stats_t{};
    launch_init<T>(c, c.Z != c.Q ? c.n - c.first : 0);
    st.kernel_launches++;
    if (c.ell_k) {
        launch_csr_to_ell<T>(c);
        st.kernel_launches++;
    }
    const double mvA = c.is_dense ? (double)c.m * (double)c.m * w
                                  : (double)c.nnz * (w + 4) + 4.0 * (double)(c.m + 1);
    if (variant == VAR_HP) {
        ProfScope ps(h, 2, c.stream);
        if (c.is_dense) launch_dense_gemm<T>(c);
        else launch_csr_spmm<T>(c);
        st.kernel_launches++;
        st.mv_calls += 1;
        st.mv_columns += c.n - c.first;
        st.mv_bytes += mvA + 2.0 * (double)c.m * (c.n - c.first) * w;
    }
    const int passes = reorth ? 2 : 1;
    for (int64_t j = c.first; j < c.n; ++j) {
        int64_t n_rr;
        if (j > 0) {
            // classical passes: zt = z_j, then zt (HA) or Q[:, j] (HP) corrected
            for (int pass = 0; pass < passes; ++pass) {
                c.z_in_zt = (pass > 0 && variant != VAR_HP) ? 1 : 0;
                launch_reorth_a<T>(c, j);
                c.z_in_zt = 0;
                launch_reorth_fin(c, j);
                launch_reorth_b<T>(c, j, variant == VAR_HP);
                st.kernel_launches += 3;
            }
        }
        if (variant == VAR_HP) {
            if (j == 0) {
                c.x_from = 0;
                launch_col_hp<T>(c, 0, false);
                c.x_from = -1;
                st.kernel_launches++;
                n_rr = c.geo.g_rows2;
            } else {
                n_rr = c.geo.g_rows1;   // A-norm partials of k_reorth_b
            }
        } else {
            // j = 0: the MV copies z_0 to zt; later columns read zt
            launch_mv<T>(c, j, j > 0 ? SRC_VEC : SRC_UPD);
            st.kernel_launches++;
            st.mv_calls += 1;
            st.mv_columns += 1;
            st.mv_bytes += mvA + (j > 0 ? 2.0 : 3.0) * (double)c.m * w;
            if (variant == VAR_NAIVE) {
                launch_mv<T>(c, j, SRC_DIV);
                st.kernel_launches++;
                st.mv_calls += 1;
                st.mv_columns += 1;
                st.mv_bytes += mvA + 2.0 * (double)c.m * w;
            }
            n_rr = c.n_rr_mv;
        }
        // normalise column j only (no later columns, no dots)
        launch_psweep<T>(c, variant, j, j, j, j, j, j + 1, j + 1, n_rr);
        st.kernel_launches++;
        st.sweep_launches++;
    }
    if (hipGetLastError() != hipSuccess) return AMGS_ERR_HIP;
    return AMGS_OK;
}

amgs_status_t qr_common(amgs_handle *h, Ctx &c, amgs_variant_t v, amgs_precision_t p,
                        const amgs_opts_t *o, void *work, size_t work_bytes, int P_given)
{
    const int reorth_mode = o ? o->reorth : 0;
    const int reorth = reorth_mode != 0;
    const int panel = o ? o->panel : 0;
    if (reorth_mode < 0 || reorth_mode > 2) return AMGS_ERR_ARG;
    if (reorth_mode == 2 && panel != PANEL_B1) return AMGS_ERR_UNSUPPORTED;
    const int cgs = o ? o->cgs : 0;
    const int64_t first = o ? o->first : 0;
    if (panel != 0 && panel != PANEL_B && panel != PANEL_B1 && panel != PANEL_B2) return AMGS_ERR_ARG;
    if (panel == PANEL_B2 && v == AMGS_HP) return AMGS_ERR_UNSUPPORTED;
    if (cgs != 0 && cgs != 1) return AMGS_ERR_ARG;
    if (first < 0 || first > c.n) return AMGS_ERR_ARG;
    if (first > 0 && !P_given) return AMGS_ERR_ARG;   // p_i of the final columns are needed
    if (panel && (cgs || first)) return AMGS_ERR_UNSUPPORTED;
    if (first == c.n) return AMGS_OK;
    const size_t w = p == AMGS_FP64 ? 8 : 4;
    c.geo = make_geo(c.m, c.nnz, c.is_dense);
    Layout L = layout(c.m, c.n, c.geo, (int)v, w, P_given, cgs ? 1 : reorth_mode, panel,
                      c.is_dense);
    if (!work || work_bytes < L.base) return AMGS_ERR_WORKSPACE;
    char *base = (char *)work;
    c.sp.part = base + L.part;
    c.sp.g = c.geo.g_rows;
    c.panel = panel;
    c.cgs = cgs;
    c.first = first;
    c.z_in_zt = 0;
    c.x_from = -1;
    c.n_pub = c.n;
    // the panel-sweep kernel also normalises the columns of the classical form
    c.g_p = panel_chunks(c.m, w);
    if (panel) {
        c.sp.g = c.g_p;
        c.wpart = base + L.wpart;
        c.lpart = base + L.lpart;
        c.lpart8 = base + L.lpart8;
        c.wred = base + L.wred;
        c.g_b = bsweep_chunks(c.m, w);
        c.reorth_blk = reorth_mode == 2;
        c.rb_part = base + L.rb_part;
        c.rb_s = (double *)(base + L.rb_s);
    }
    c.s_part = (double *)(base + L.s_part);
    c.rr_part = (double *)(base + L.rr_part);
    c.S = (double *)(base + L.S);
    c.zt = base + L.zt;
    c.xv = base + L.xv;
    c.X = v == AMGS_HP ? (void *)(base + L.X) : nullptr;
    if (!P_given) {
        c.P = base + L.P;
        c.ldp = c.m;
    }
    c.n_rr_mv = c.is_dense ? c.geo.g_dense : c.geo.g_csr;
    c.ell_k = 0;
    if (!c.is_dense && v != AMGS_HP && c.geo.lanes == 0 && work_bytes >= L.total) {
        // K = the mean row length rounded up (at most ELL_K here); longer
        // rows keep their remaining entries in the CSR arrays
        int64_t k = (c.nnz + c.m - 1) / c.m;
        c.ell_k = (int32_t)(k < 1 ? 1 : k > ELL_K ? ELL_K : k);
        c.ell_col = (int32_t *)(base + L.ell_col);
        c.ell_val = base + L.ell_val;
        c.tile_long = (int32_t *)(base + L.tile_long);
        c.ell_d16 = (int16_t *)(base + L.ell_d16);
        c.ell_wide = (int32_t *)(base + L.ell_wide);
    }
    DeviceGuard dg(h->device);
    return p == AMGS_FP64 ? run_single<double>(h, c, (int)v, reorth)
                          : run_single<float>(h, c, (int)v, reorth);
}

bool common_args_ok(amgs_handle_t h, int64_t m, int64_t n, const void *Z, int64_t ldz,
                    const void *Q, int64_t ldq, const double *R, int64_t ldr, const void *P,
                    int64_t ldp, amgs_variant_t v, amgs_precision_t p, const int32_t *info)
{
    if (!h || m < 0 || n < 0 || n > m || !valid_enums(v, p)) return false;
    if (n == 0) return true;
    if (!Z || !Q || !R || !info) return false;
    if (ldz < m || ldq < m || ldr < n) return false;
    if (P && ldp < m) return false;
    if (Z == Q && ldz != ldq) return false;
    if (m > (int64_t)0x7fffffff) return false; // int32 row indices in CSR
    return true;
}

} // namespace

namespace amgs {
Geo make_geo(int64_t m, int64_t nnz, int is_dense)
{
    Geo g{};
    // about 256 row chunks of 256*U rows (U <= 8): more rows per thread
    // keep more loads in flight in the streaming kernels
    const int64_t cap = 256 * 256;
    g.U = m <= cap ? 1 : m <= 2 * cap ? 2 : m <= 4 * cap ? 4 : 8;
    g.g_rows = (m + 256 * g.U - 1) / (256 * g.U);
    if (g.g_rows < 1) g.g_rows = 1;
    // the column and second-pass kernels hold several vectors per row in
    // registers, so they keep at most 4 rows per thread
    g.U2 = g.U < 4 ? g.U : 4;
    g.g_rows2 = (m + 256 * g.U2 - 1) / (256 * g.U2);
    if (g.g_rows2 < 1) g.g_rows2 = 1;
    g.g_rows1 = (m + 255) / 256;
    if (g.g_rows1 < 1) g.g_rows1 = 1;
    const double avg = m > 0 ? (double)nnz / (double)m : 0.0;
    g.lanes = avg <= 7.5 ? 0 : avg <= 12 ? 1 : avg <= 24 ? 2 : avg <= 48 ? 4 : avg <= 96 ? 8
            : avg <= 192 ? 16 : avg <= 384 ? 32 : 64;
    const int64_t rows_per_wg = g.lanes == 0 ? MV_TILE : 512 / g.lanes;
    g.g_csr = (m + rows_per_wg - 1) / rows_per_wg;
    if (g.g_csr > MAX_G_MV) g.g_csr = MAX_G_MV;
    if (g.g_csr < 1) g.g_csr = 1;
    g.g_dense = (m + DENSE_CB - 1) / DENSE_CB;
    if (g.g_dense > MAX_G_MV) g.g_dense = MAX_G_MV;
    if (g.g_dense < 1) g.g_dense = 1;
    (void)is_dense;
    return g;
}
} // namespace amgs

extern "C" {

amgs_status_t amgs_create(amgs_handle_t *out, int device)
{
    if (!out) return AMGS_ERR_ARG;
    *out = nullptr;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return AMGS_ERR_ARG;
    amgs_handle *h = new (std::nothrow) amgs_handle();
    if (!h) return AMGS_ERR_HIP;
    h->device = device;
    h->num_cu = 0;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) h->num_cu = prop.multiProcessorCount;
    h->scratch = nullptr;
    if (device < SCRATCH_MAX_DEV) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (!g_scratch[device]) {
            DeviceGuard dg(device);
            void *ptr = nullptr;
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
                (void)hipGetLastError();
                delete h;
                return AMGS_ERR_HIP;
            }
            g_scratch[device] = ptr;
        }
        h->scratch = g_scratch[device];
    }
    h->stats = amgs_stats_t{};
    h->profiling = 0;
    for (int i = 0; i < AMGS_PROF_NCAT; ++i) {
        h->prof_ms[i] = 0.0;
        h->prof_n[i] = 0;
    }
    *out = h;
    return AMGS_OK;
}

amgs_status_t amgs_destroy(amgs_handle_t h)
{
    if (!h) return AMGS_ERR_ARG;
    for (auto &r : h->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : h->pool) (void)hipEventDestroy(e);
    delete h;
    return AMGS_OK;
}

size_t amgs_workspace_bytes(amgs_handle_t h, int64_t m, int64_t n, int32_t is_dense,
                            amgs_variant_t v, amgs_precision_t p, int32_t P_given,
                            const amgs_opts_t *o)
{
    if (!h || m < 0 || n < 0 || n > m || !valid_enums(v, p)) return 0;
    if (n == 0) return 0;
    // nnz only selects the CSR lane count, which does not change any size
    Geo g = make_geo(m, is_dense ? 0 : m, is_dense);
    const int panel = o ? o->panel : 0;
    const int cgs = o ? o->cgs : 0;
    if (panel != 0 && panel != PANEL_B && panel != PANEL_B1 && panel != PANEL_B2) return 0;
    if (panel == PANEL_B2 && v == AMGS_HP) return 0;
    if (cgs != 0 && cgs != 1) return 0;
    const int reorth_mode = o ? o->reorth : 0;
    if (reorth_mode < 0 || reorth_mode > 2) return 0;
    if (reorth_mode == 2 && panel != PANEL_B1) return 0;
    Layout L = layout(m, n, g, (int)v, p == AMGS_FP64 ? 8 : 4, P_given,
                      cgs ? 1 : reorth_mode, panel, is_dense);
    return L.total;
}

amgs_status_t amgs_qr_csr(amgs_handle_t h, int64_t m, int64_t nnz, const int32_t *row_ptr,
                          const int32_t *col_idx, const void *vals, int64_t n, const void *Z,
                          int64_t ldz, void *Q, int64_t ldq, double *R, int64_t ldr, void *P,
                          int64_t ldp, amgs_variant_t v, amgs_precision_t p,
                          const amgs_opts_t *o, void *work, size_t work_bytes, int32_t *info,
                          void *stream)
{
    if (!common_args_ok(h, m, n, Z, ldz, Q, ldq, R, ldr, P, ldp, v, p, info)) return AMGS_ERR_ARG;
    // entry positions are int32 in the kernels, which step up to 512 past a
    // row's end before testing it: keep that headroom below 2^31
    if (nnz < 0 || nnz > (int64_t)0x7fffffff - 1024) return AMGS_ERR_ARG;
    if (n == 0) return AMGS_OK;
    if (!row_ptr || (nnz > 0 && (!col_idx || !vals))) return AMGS_ERR_ARG;
    Ctx c{};
    c.m = m; c.n = n; c.is_dense = 0;
    c.row_ptr = row_ptr; c.col_idx = col_idx; c.vals = vals; c.nnz = nnz;
    c.Z = Z; c.ldz = ldz; c.Q = Q; c.ldq = ldq; c.R = R; c.ldr = ldr;
    c.P = P; c.ldp = ldp; c.info = info; c.stream = (hipStream_t)stream;
    return qr_common(h, c, v, p, o, work, work_bytes, P != nullptr);
}

amgs_status_t amgs_qr_csr_static(amgs_handle_t h, int64_t m, int64_t nnz,
                                 const int32_t *row_ptr, const int32_t *col_idx,
                                 const void *vals, int64_t n, const void *Z, int64_t ldz, void *Q,
                                 int64_t ldq, double *R, int64_t ldr, void *P, int64_t ldp,
                                 amgs_variant_t v, amgs_precision_t p, const amgs_opts_t *o,
                                 int32_t *info, void *stream)
{
    // the same kernels as amgs_qr_csr, with this device's scratch array as
    // the workspace; a problem needing more than the array holds is
    // rejected by the workspace check (AMGS_ERR_WORKSPACE) before any launch
    if (!h) return AMGS_ERR_ARG;
    if (!h->scratch) return AMGS_ERR_UNSUPPORTED;
    return amgs_qr_csr(h, m, nnz, row_ptr, col_idx, vals, n, Z, ldz, Q, ldq, R, ldr, P, ldp, v,
                       p, o, h->scratch, AMGS_STATIC_SCRATCH_BYTES, info, stream);
}

amgs_status_t amgs_qr_dense(amgs_handle_t h, int64_t m, const void *A, int64_t lda, int64_t n,
                            const void *Z, int64_t ldz, void *Q, int64_t ldq, double *R,
                            int64_t ldr, void *P, int64_t ldp, amgs_variant_t v,
                            amgs_precision_t p, const amgs_opts_t *o, void *work,
                            size_t work_bytes, int32_t *info, void *stream)
{
    if (!common_args_ok(h, m, n, Z, ldz, Q, ldq, R, ldr, P, ldp, v, p, info)) return AMGS_ERR_ARG;
    if (n == 0) return AMGS_OK;
    if (!A || lda < m) return AMGS_ERR_ARG;
    Ctx c{};
    c.m = m; c.n = n; c.is_dense = 1; c.A = A; c.lda = lda; c.nnz = m * m;
    c.Z = Z; c.ldz = ldz; c.Q = Q; c.ldq = ldq; c.R = R; c.ldr = ldr;
    c.P = P; c.ldp = ldp; c.info = info; c.stream = (hipStream_t)stream;
    return qr_common(h, c, v, p, o, work, work_bytes, P != nullptr);
}

amgs_status_t amgs_csr_check(amgs_handle_t h, int64_t m, int64_t nnz, const int32_t *row_ptr,
                             const int32_t *col_idx, int32_t *flag, void *stream)
{
    if (!h || m < 0 || nnz < 0 || !row_ptr || !flag || (nnz > 0 && !col_idx)) return AMGS_ERR_ARG;
    DeviceGuard dg(h->device);
    launch_csr_check(m, nnz, row_ptr, col_idx, flag, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? AMGS_OK : AMGS_ERR_HIP;
}

amgs_status_t amgs_get_stats(amgs_handle_t h, amgs_stats_t *out)
{
    if (!h || !out) return AMGS_ERR_ARG;
    *out = h->stats;
    return AMGS_OK;
}

const char *amgs_status_string(amgs_status_t s)
{
    switch (s) {
    case AMGS_OK: return "ok";
    case AMGS_ERR_ARG: return "invalid argument";
    case AMGS_ERR_WORKSPACE: return "workspace too small";
    case AMGS_ERR_HIP: return "HIP launch or runtime error";
    case AMGS_ERR_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

amgs_status_t amgs_profile_enable(amgs_handle_t h, int32_t on)
{
    if (!h) return AMGS_ERR_ARG;
    h->profiling = on ? 1 : 0;
    return AMGS_OK;
}

amgs_status_t amgs_profile_read(amgs_handle_t h, int32_t category, double *total_ms,
                                int64_t *launches)
{
    if (!h || category < 0 || category >= AMGS_PROF_NCAT) return AMGS_ERR_ARG;
    DeviceGuard dg(h->device);
    for (auto &r : h->recs) {
        if (hipEventSynchronize(r.b) != hipSuccess) return AMGS_ERR_HIP;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return AMGS_ERR_HIP;
        h->prof_ms[r.cat] += ms;
        h->prof_n[r.cat] += 1;
        if (r.cat2 >= 0) {
            h->prof_ms[r.cat2] += ms;
            h->prof_n[r.cat2] += 1;
        }
        h->pool.push_back(r.a);
        h->pool.push_back(r.b);
    }
    h->recs.clear();
    if (total_ms) *total_ms = h->prof_ms[category];
    if (launches) *launches = h->prof_n[category];
    return AMGS_OK;
}

amgs_status_t amgs_profile_reset(amgs_handle_t h)
{
    if (!h) return AMGS_ERR_ARG;
    double ms;
    int64_t n;
    amgs_status_t s = amgs_profile_read(h, 0, &ms, &n);
    for (int i = 0; i < AMGS_PROF_NCAT; ++i) {
        h->prof_ms[i] = 0.0;
        h->prof_n[i] = 0;
    }
    return s;
}

} // extern "C"
