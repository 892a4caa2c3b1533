// hk_api.cpp -- the C ABI of libhk (include/hk.h): argument checking,
// context and device memory, and the stream-ordered launch sequence of each
// call.  Every numerical step runs in the HIP kernels of this directory.
#include "../../include/hk.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <limits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "hk_internal.h"

using namespace hk;

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    hipError_t ensure(size_t bytes)
    {
        if (bytes <= cap) return hipSuccess;
        release();
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            p = nullptr;
            return e;
        }
        cap = bytes;
        return hipSuccess;
    }
};

// What the launches need to know of a line list besides its values: which
// optional fields it has, and bounds that size the tile ranges.
struct ListInfo {
    bool has_self = false, has_delta = false, has_A = false;
    double max_abs_delta = 0.0;
    // bounds of the width parameters, for the reach of Lorentz-width cutoffs
    double max_gamma_air = 0.0, max_gamma_self = 0.0, max_A21 = 0.0, min_n_air = 0.0, max_n_air = 0.0;
    double nu_max = 0.0;  // largest line centre (bounds the Doppler core widths)
};

// Device buffers of one work plan (work_plan.hip) and its partial sums.
struct PlanBufs {
    DevBuf ref, seg, first, slot, bsum, total, partial;
    void release()
    {
        for (DevBuf* b : {&ref, &seg, &first, &slot, &bsum, &total, &partial}) b->release();
    }
};

// The device state of one opacity pass over one line list: per-line records,
// tile ranges, the work plans of the wing and the series kernels, the series
// grid and the binary32 sums.  A context holds two: hk_opacity_stream
// alternates them between chunks, so that one chunk is prepared while the
// kernels of the one before it still run.
struct Lane {
    DevBuf wing, widx, core, ranges, ranges_core;
    PlanBufs wplan, cplan;
    DevBuf kc;
    DevBuf w32, c32, f32sum, f32comp, f32scale, f32partial;
    // per-workgroup counts of the points the network evaluated in a
    // HK_F32_SURROGATE series launch
    DevBuf sg_used;
    void release()
    {
        for (DevBuf* b : {&wing, &widx, &core, &ranges, &ranges_core, &kc, &w32, &c32, &f32sum, &f32comp,
                          &f32scale, &f32partial, &sg_used})
            b->release();
        wplan.release();
        cplan.release();
    }
};

struct hk_ctx {
    int device = 0;
    hipStream_t own = nullptr;     // created with the context
    hipStream_t stream = nullptr;  // where work is enqueued (may be the null stream)
    int64_t lds_bytes = kSortLdsBytes;  // LDS a sort workgroup may use
    int64_t lds_max = 65536;            // the device's LDS per workgroup (the radix sorts)
    void* noalloc_scratch = nullptr;    // this device's hk_kdist_noalloc array
    std::string err;
    // line list, ascending (nu, index)
    int64_t n_lines = 0;
    bool lines_loaded = false;
    ListInfo li;
    double last_P = 0.0;  // pressure of the state being computed
    hk_species species{296.0, 0.0};
    DevBuf lines;  // 8 arrays of n doubles
    // streamed lists: the second device line buffer, pinned host staging
    // (two buffers of pin_cap doubles) and the events of their copies, and
    // the per-chunk evaluation counters of the last hk_opacity_stream call
    DevBuf lines_alt;
    double* pin[2] = {nullptr, nullptr};
    size_t pin_cap = 0;
    hipEvent_t ev_copied[2] = {nullptr, nullptr};
    DevBuf st_counts;
    int32_t last_stream_chunks = 0;  // > 0: hk_stats reports that call
    int64_t stream_lines = 0;
    // the state of an opacity pass (ln), and the second one that a stream
    // of chunks alternates with
    Lane ln, ln_alt;
    // the series on a second stream, concurrent with the wing: the stream
    // and the fork / join events
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // streamed chunks: the wing's own stream, and per chunk parity the
    // events of the fork and of the series' and the wing's ends; ev_kappa
    // marks the last update of kappa (a binary64 wing adds to it)
    hipStream_t wing_s = nullptr;
    hipEvent_t ev_cfork[2] = {nullptr, nullptr}, ev_ccore[2] = {nullptr, nullptr},
               ev_cwing[2] = {nullptr, nullptr}, ev_kappa = nullptr;
    DevBuf partial;  // evaluation counters of hk_stats
    DevBuf kscratch;
    bool have_run = false;
    int f64_points_per_lane = 4;  // tile shape of the binary64 opacity kernel (4 or 8)
    int f32_points_per_lane = 4;  // tile shape of the binary32 opacity kernel
    int wing_edge_paths = 1;      // 0: window-edge runs take the general path (same bits)
    int tables_overlap = 0;       // 1: tables run the series beside the wing on the second stream
    // batched tables: per-state records, ranges and sums of one batch, the
    // per-state evaluation counters of the last call, and the tile shapes
    // chosen by timing, per (precision, lines, points, cutoff/dnu)
    DevBuf tb_idx, tb_wing, tb_core, tb_w32, tb_c32, tb_ranges, tb_ranges_c, tb_out, tb_comp, tb_scale, tb_kappa,
        tb_counts, tb_series, tb_prep;
    int64_t tables_batch = 0;  // states per launch; 0 = as many as fit in tables_mem
    int64_t tables_mem = (int64_t)32 << 30;
    int tables_autotune = 1;
    int32_t last_tables_states = 0;  // > 0: hk_stats reports that hk_tables call
    int tables_ppl_used = 0;          // tile shape of the last hk_tables call
    struct Tuned {
        int precision;
        int64_t n_lines, n_points, cut_steps;
        int ppl;
    };
    std::vector<Tuned> tuned;
    // learned surrogate: binary32 parameters, Adam moments, the bfloat16
    // compute copy, training partials, certification errors and mask
    DevBuf sg_theta, sg_m, sg_v, sg_copy, sg_part, sg_ploss, sg_err, sg_mask;
    bool sg_loaded = false, sg_certified = false;
    // the running total of the points the network evaluated (element 0),
    // over the passes of one hk_opacity / hk_opacity_stream call
    DevBuf sg_used_total;
    double sg_budget = 0.0;  // of the current certification
    // resampling: QR factors of the Chebyshev design matrix for the bin
    // sizes of the last call (main and ragged last bin), and the quadrature
    DevBuf rs_Q, rs_R, rs_Ql, rs_Rl, rs_quad;
    int64_t rs_m = -1, rs_ml = -1;
    int rs_nc = 0;
    bool rs_quad_ready = false;
    int64_t sg_step = 0;  // Adam steps taken
    int64_t sg_cursor = 0;  // next training sample
    // stage timing: events recorded around each timed launch, resolved
    // lazily (pending pairs) so timing adds no host synchronisation
    bool timing = false;
    hk_timing tsum{};
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> pending;
    std::vector<hipEvent_t> free_events;
};

namespace {

thread_local std::string t_err;

int fail(hk_ctx* ctx, int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_err = buf;
    if (ctx) ctx->err = buf;
    return code;
}

int hip_fail(hk_ctx* ctx, hipError_t e, const char* what)
{
    return fail(ctx, e == hipErrorOutOfMemory ? HK_ENOMEM : HK_EDEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

#define HK_HIP(ctx, call, what)                         \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
    } while (0)

bool isfin(double v) { return std::isfinite(v); }

int check_ctx(hk_ctx* ctx)
{
    if (!ctx) return fail(nullptr, HK_EINVAL, "context is NULL");
    return HK_OK;
}

int check_state(hk_ctx* ctx, const hk_state* st)
{
    if (!st) return fail(ctx, HK_EINVAL, "state is NULL");
    if (!isfin(st->T) || !(st->T > 0.0)) return fail(ctx, HK_EINVAL, "T must be finite and > 0 (got %g)", st->T);
    if (!isfin(st->P) || !(st->P >= 0.0)) return fail(ctx, HK_EINVAL, "P must be finite and >= 0 (got %g)", st->P);
    if (!isfin(st->P_self) || !(st->P_self >= 0.0) || !(st->P_self <= st->P))
        return fail(ctx, HK_EINVAL, "P_self must satisfy 0 <= P_self <= P (got %g, P = %g)", st->P_self, st->P);
    if (!isfin(st->q_ratio) || !(st->q_ratio > 0.0))
        return fail(ctx, HK_EINVAL, "q_ratio must be finite and > 0 (got %g)", st->q_ratio);
    if (!isfin(st->abundance) || !(st->abundance >= 0.0))
        return fail(ctx, HK_EINVAL, "abundance must be finite and >= 0 (got %g)", st->abundance);
    return HK_OK;
}

int check_grid(hk_ctx* ctx, const hk_grid* g)
{
    if (!g) return fail(ctx, HK_EINVAL, "grid is NULL");
    if (!isfin(g->nu_min)) return fail(ctx, HK_EINVAL, "nu_min must be finite");
    if (!isfin(g->dnu) || !(g->dnu > 0.0)) return fail(ctx, HK_EINVAL, "dnu must be finite and > 0 (got %g)", g->dnu);
    if (g->n_points < 0 || g->n_points > HK_MAX_POINTS)
        return fail(ctx, HK_EINVAL, "n_points must be in [0, %lld] (got %lld)", (long long)HK_MAX_POINTS,
                    (long long)g->n_points);
    if (!isfin(g->cutoff) || !(g->cutoff >= 0.0))
        return fail(ctx, HK_EINVAL, "cutoff must be finite and >= 0 (got %g)", g->cutoff);
    if (!isfin(g->cutoff_lorentz) || !(g->cutoff_lorentz >= 0.0))
        return fail(ctx, HK_EINVAL, "cutoff_lorentz must be finite and >= 0 (got %g)", g->cutoff_lorentz);
    double last = g->nu_min + (double)(g->n_points > 0 ? g->n_points - 1 : 0) * g->dnu;
    if (!isfin(last)) return fail(ctx, HK_EINVAL, "grid end is not finite");
    return HK_OK;
}

int check_bins(hk_ctx* ctx, const hk_bins* b, GValues* gv)
{
    if (!b) return fail(ctx, HK_EINVAL, "bins is NULL");
    if (b->points_per_bin < 1) return fail(ctx, HK_EINVAL, "points_per_bin must be >= 1");
    if (b->n_g < 1 || b->n_g > HK_MAX_G) return fail(ctx, HK_EINVAL, "n_g must be in [1, %d]", HK_MAX_G);
    if (!b->g) return fail(ctx, HK_EINVAL, "g is NULL");
    if (b->rule != HK_RULE_STEP && b->rule != HK_RULE_LINEAR)
        return fail(ctx, HK_EINVAL, "rule %d is neither HK_RULE_STEP nor HK_RULE_LINEAR", b->rule);
    gv->n = b->n_g;
    gv->rule = b->rule;
    for (int q = 0; q < b->n_g; ++q) {
        if (!isfin(b->g[q]) || !(b->g[q] > 0.0) || !(b->g[q] < 1.0))
            return fail(ctx, HK_EINVAL, "g[%d] = %g is not in (0, 1)", q, b->g[q]);
        gv->g[q] = b->g[q];
    }
    for (int q = b->n_g; q < 64; ++q) gv->g[q] = 0.5;
    return HK_OK;
}

hipEvent_t take_event(hk_ctx* ctx)
{
    if (!ctx->free_events.empty()) {
        hipEvent_t e = ctx->free_events.back();
        ctx->free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets one stage's launches with events when timing is on.
struct StageTimer {
    hk_ctx* ctx;
    int stage;
    hipStream_t strm;
    hipEvent_t a = nullptr, b = nullptr;
    StageTimer(hk_ctx* c, int s) : StageTimer(c, s, c->stream) {}
    StageTimer(hk_ctx* c, int s, hipStream_t st) : ctx(c), stage(s), strm(st)
    {
        if (!ctx->timing) return;
        a = take_event(ctx);
        b = take_event(ctx);
        if (a && b) (void)hipEventRecord(a, strm);
    }
    void stop()
    {
        if (!a || !b) return;
        (void)hipEventRecord(b, strm);
        ctx->pending.push_back({stage, {a, b}});
        a = b = nullptr;
    }
    ~StageTimer()
    {
        if (a) ctx->free_events.push_back(a);
        if (b) ctx->free_events.push_back(b);
    }
};

double* lines_field(hk_ctx* ctx, int k) { return static_cast<double*>(ctx->lines.p) + (size_t)k * ctx->n_lines; }

LinesDev lines_dev(hk_ctx* ctx)
{
    LinesDev L;
    L.nu = lines_field(ctx, 0);
    L.S_ref = lines_field(ctx, 1);
    L.E_lower = lines_field(ctx, 2);
    L.gamma_air = lines_field(ctx, 3);
    L.n_air = lines_field(ctx, 4);
    L.gamma_self = ctx->li.has_self ? lines_field(ctx, 5) : L.gamma_air;
    L.delta = ctx->li.has_delta ? lines_field(ctx, 6) : nullptr;
    L.A21 = ctx->li.has_A ? lines_field(ctx, 7) : nullptr;
    L.n = ctx->n_lines;
    return L;
}

// Per-state constants of the line preparation (eq. 18-21 of §2.3, the
// Doppler factor sqrt(2 k T / m) / c, the natural width factor 1/(4 pi c)).
PrepParams prep_params(const hk_ctx* ctx, const hk_state* st, const hk_grid* grid)
{
    PrepParams pp;
    pp.T = st->T;
    pp.T_ref = ctx->species.T_ref;
    pp.P = st->P;
    pp.P_self = st->P_self;
    pp.q_ratio = st->q_ratio * st->abundance;  // S scales with the species' weight
    pp.dop = std::sqrt(2.0 * kKB * st->T / (ctx->species.mass_amu * kAMU)) / kC;
    pp.nat = 1.0 / (4.0 * kPi * kC);
    pp.tscale = st->T / ctx->species.T_ref;
    pp.nu_min = grid->nu_min;
    pp.dnu = grid->dnu;
    pp.cutoff = grid->cutoff;
    pp.cutoff_lorentz = grid->cutoff_lorentz;
    pp.n_points = (int32_t)grid->n_points;
    return pp;
}

// A line can reach a grid tile only if its unshifted centre lies within the
// cutoff plus the largest pressure shift (+ two grid steps of slack for the
// rounding of the window bounds).  Its series region a^2+u^2 < 100 lies
// within 10 alpha of the centre, and alpha = nu * dop is largest for the
// largest nu.
// The largest cutoff of any line: the absolute cutoff, or cutoff_lorentz
// times an upper bound of Gamma_L (eq. 20 with each parameter at its
// extreme over the loaded lines; (T/T_ref)^-n is monotone in n).
double max_cutoff(const ListInfo& li, double T_ref, const hk_state* st, const hk_grid* grid)
{
    if (!(grid->cutoff_lorentz > 0.0)) return grid->cutoff;
    const double ts = st->T / T_ref;
    const double f = std::max(std::pow(ts, -li.min_n_air), std::pow(ts, -li.max_n_air));
    const double gl = li.max_A21 / (4.0 * kPi * kC) +
                      f * (li.max_gamma_air * (st->P - st->P_self) + li.max_gamma_self * st->P_self);
    return grid->cutoff_lorentz * gl * (1.0 + 1e-9);
}
double max_cutoff(const hk_ctx* ctx, const hk_state* st, const hk_grid* grid)
{
    return max_cutoff(ctx->li, ctx->species.T_ref, st, grid);
}
double wing_reach(const hk_ctx* ctx, const hk_state* st, const hk_grid* grid)
{
    return max_cutoff(ctx, st, grid) + ctx->li.max_abs_delta * st->P + 2.0 * grid->dnu;
}
double core_reach(const hk_ctx* ctx, const hk_state* st, const hk_grid* grid, const PrepParams& pp)
{
    return std::min(10.0 * pp.dop * ctx->li.nu_max, max_cutoff(ctx, st, grid)) + ctx->li.max_abs_delta * st->P +
           2.0 * grid->dnu;
}

// Runs fn(i0, i1, t) over [0, n) split into contiguous ranges, on up to 8
// host threads when the range is large (the host side of loading a list).
template <typename F>
void host_ranges(int64_t n, int n_max_threads, F fn)
{
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int t = n < ((int64_t)1 << 16) ? 1 : (int)std::min<unsigned>((unsigned)n_max_threads, hw);
    if (t <= 1) {
        fn((int64_t)0, n, 0);
        return;
    }
    std::vector<std::thread> th;
    th.reserve((size_t)t);
    for (int k = 0; k < t; ++k) th.emplace_back(fn, n * k / t, n * (k + 1) / t, k);
    for (auto& x : th) x.join();
}

int check_species(hk_ctx* ctx, const hk_species* sp)
{
    if (!sp) return fail(ctx, HK_EINVAL, "species must not be NULL");
    if (!isfin(sp->T_ref) || !(sp->T_ref > 0.0)) return fail(ctx, HK_EINVAL, "T_ref must be finite and > 0");
    if (!isfin(sp->mass_amu) || !(sp->mass_amu > 0.0)) return fail(ctx, HK_EINVAL, "mass_amu must be finite and > 0");
    return HK_OK;
}

// Whether line i of L breaks a value rule of hk_load_lines.
bool line_bad(const hk_lines* L, int64_t i)
{
    return !isfin(L->nu[i]) || !(L->nu[i] > 0.0) || !isfin(L->S_ref[i]) || !(L->S_ref[i] >= 0.0) ||
           !isfin(L->E_lower[i]) || !isfin(L->gamma_air[i]) || !(L->gamma_air[i] >= 0.0) || !isfin(L->n_air[i]) ||
           (L->gamma_self && (!isfin(L->gamma_self[i]) || !(L->gamma_self[i] >= 0.0))) ||
           (L->delta && !isfin(L->delta[i])) || (L->A21 && (!isfin(L->A21[i]) || !(L->A21[i] >= 0.0)));
}

// The shape rules of a line list: a count in range, the required fields there.
bool lines_shape_ok(const hk_lines* L)
{
    return L && L->n >= 0 && L->n <= (int64_t)INT32_MAX &&
           (L->n == 0 || (L->nu && L->S_ref && L->E_lower && L->gamma_air && L->n_air));
}

// The rules of a line list (hk_load_lines), with the error of the first
// offending line, in input order; chunk >= 0 names the chunk of a streamed
// list in the message.  Used to report: scan_lists tests the rules in the
// same pass that gathers the bounds.
int check_lines(hk_ctx* ctx, const hk_lines* L, int64_t chunk)
{
    char pre[40] = "";
    if (chunk >= 0) snprintf(pre, sizeof pre, "chunk %lld: ", (long long)chunk);
    if (!L) return fail(ctx, HK_EINVAL, "%slines must not be NULL", pre);
    if (L->n < 0 || L->n > (int64_t)INT32_MAX)
        return fail(ctx, HK_EINVAL, "%sline count %lld out of range", pre, (long long)L->n);
    const int64_t n = L->n;
    if (n > 0 && (!L->nu || !L->S_ref || !L->E_lower || !L->gamma_air || !L->n_air))
        return fail(ctx, HK_EINVAL, "%snu, S_ref, E_lower, gamma_air and n_air are required", pre);
    std::vector<int64_t> first(8, n);
    host_ranges(n, 8, [&](int64_t i0, int64_t i1, int t) {
        for (int64_t i = i0; i < i1; ++i)
            if (line_bad(L, i)) {
                first[(size_t)t] = i;
                return;
            }
    });
    const int64_t i = *std::min_element(first.begin(), first.end());
    if (i == n) return HK_OK;
    const long long li = (long long)i;
    if (!isfin(L->nu[i]) || !(L->nu[i] > 0.0))
        return fail(ctx, HK_EINVAL, "%snu[%lld] = %g must be finite and > 0", pre, li, L->nu[i]);
    if (!isfin(L->S_ref[i]) || !(L->S_ref[i] >= 0.0))
        return fail(ctx, HK_EINVAL, "%sS_ref[%lld] = %g must be finite and >= 0", pre, li, L->S_ref[i]);
    if (!isfin(L->E_lower[i])) return fail(ctx, HK_EINVAL, "%sE_lower[%lld] is not finite", pre, li);
    if (!isfin(L->gamma_air[i]) || !(L->gamma_air[i] >= 0.0))
        return fail(ctx, HK_EINVAL, "%sgamma_air[%lld] must be finite and >= 0", pre, li);
    if (!isfin(L->n_air[i])) return fail(ctx, HK_EINVAL, "%sn_air[%lld] is not finite", pre, li);
    if (L->gamma_self && (!isfin(L->gamma_self[i]) || !(L->gamma_self[i] >= 0.0)))
        return fail(ctx, HK_EINVAL, "%sgamma_self[%lld] must be finite and >= 0", pre, li);
    if (L->delta && !isfin(L->delta[i])) return fail(ctx, HK_EINVAL, "%sdelta[%lld] is not finite", pre, li);
    return fail(ctx, HK_EINVAL, "%sA21[%lld] must be finite and >= 0", pre, li);
}

// One list's result of scan_lists: whether a line breaks a value rule; if
// none does, the list's flags and bounds and whether nu is non-decreasing.
struct ListScan {
    bool bad = false, sorted = true;
    ListInfo info;
};

// One pass over the values of lists L[0 .. k) (each of valid shape), by one
// team of up to 8 host threads that each take the same share of every list:
// the value rules, the bounds and the order test read each value once.
std::vector<ListScan> scan_lists(const hk_lines* L, int64_t k)
{
    struct Part {
        bool any = false, bad = false, sorted = true;
        ListInfo b;
    };
    int64_t total = 0;
    for (int64_t c = 0; c < k; ++c) total += L[c].n;
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const int T = total < ((int64_t)1 << 16) ? 1 : (int)std::min(8u, hw);
    std::vector<Part> part((size_t)(k * T));
    // column by column (each value is still read once), in loops without
    // branches that the compiler vectorises: a comparison with NaN is false
    constexpr double kMax = std::numeric_limits<double>::max();
    auto nonneg = [](const double* v, int64_t i0, int64_t i1, double& mx) {
        int ok = 1;
        double m = mx;
        for (int64_t i = i0; i < i1; ++i) {
            ok &= (v[i] >= 0.0) & (v[i] <= kMax);
            m = v[i] > m ? v[i] : m;
        }
        mx = m;
        return ok;
    };
    auto work = [&](int t) {
        for (int64_t c = 0; c < k; ++c) {
            const hk_lines* l = &L[c];
            const int64_t i0 = l->n * t / T, i1 = l->n * (t + 1) / T;
            if (i0 >= i1) continue;
            Part& p = part[(size_t)(c * T + t)];
            ListInfo& b = p.b;
            p.any = true;
            int ok = 1, up = 1;
            double nu_max = 0.0;
            for (int64_t i = i0; i < i1; ++i) {
                ok &= (l->nu[i] > 0.0) & (l->nu[i] <= kMax);
                nu_max = l->nu[i] > nu_max ? l->nu[i] : nu_max;
            }
            for (int64_t i = std::max<int64_t>(i0, 1); i < i1; ++i) up &= !(l->nu[i] < l->nu[i - 1]);
            double s_max = 0.0;
            ok &= nonneg(l->S_ref, i0, i1, s_max);
            for (int64_t i = i0; i < i1; ++i) ok &= std::fabs(l->E_lower[i]) <= kMax;
            ok &= nonneg(l->gamma_air, i0, i1, b.max_gamma_air);
            double n_lo = l->n_air[i0], n_hi = l->n_air[i0];
            for (int64_t i = i0; i < i1; ++i) {
                ok &= std::fabs(l->n_air[i]) <= kMax;
                n_lo = l->n_air[i] < n_lo ? l->n_air[i] : n_lo;
                n_hi = l->n_air[i] > n_hi ? l->n_air[i] : n_hi;
            }
            if (l->gamma_self)
                ok &= nonneg(l->gamma_self, i0, i1, b.max_gamma_self);
            else
                b.max_gamma_self = b.max_gamma_air;
            if (l->delta) {
                double d = 0.0;
                for (int64_t i = i0; i < i1; ++i) {
                    const double a = std::fabs(l->delta[i]);
                    ok &= a <= kMax;
                    d = a > d ? a : d;
                }
                b.max_abs_delta = d;
            }
            if (l->A21) ok &= nonneg(l->A21, i0, i1, b.max_A21);
            b.nu_max = nu_max;
            b.min_n_air = n_lo;
            b.max_n_air = n_hi;
            p.bad = !ok;
            p.sorted = up;
        }
    };
    if (T == 1) {
        work(0);
    } else {
        std::vector<std::thread> th;
        th.reserve((size_t)T);
        for (int t = 0; t < T; ++t) th.emplace_back(work, t);
        for (auto& x : th) x.join();
    }
    std::vector<ListScan> out((size_t)k);
    for (int64_t c = 0; c < k; ++c) {
        ListScan& r = out[(size_t)c];
        ListInfo& li = r.info;
        li.has_self = L[c].gamma_self != nullptr;
        li.has_delta = L[c].delta != nullptr;
        li.has_A = L[c].A21 != nullptr;
        bool first = true;
        for (int t = 0; t < T; ++t) {
            const Part& p = part[(size_t)(c * T + t)];
            if (!p.any) continue;
            r.bad = r.bad || p.bad;
            r.sorted = r.sorted && p.sorted;
            const ListInfo& b = p.b;
            li.max_abs_delta = std::max(li.max_abs_delta, b.max_abs_delta);
            li.max_gamma_air = std::max(li.max_gamma_air, b.max_gamma_air);
            li.max_gamma_self = std::max(li.max_gamma_self, b.max_gamma_self);
            li.max_A21 = std::max(li.max_A21, b.max_A21);
            li.min_n_air = first ? b.min_n_air : std::min(li.min_n_air, b.min_n_air);
            li.max_n_air = first ? b.max_n_air : std::max(li.max_n_air, b.max_n_air);
            li.nu_max = std::max(li.nu_max, b.nu_max);
            first = false;
        }
    }
    return out;
}

// The indices of an unordered list sorted by (nu, index) -- the order a
// stable sort by nu gives -- on up to 8 host threads: each sorts a
// contiguous part of (nu, index) pairs, then the parts are merged pairwise.
std::vector<int64_t> line_order(const double* nu, int64_t n)
{
    struct Key {
        double nu;
        int64_t i;
    };
    const auto less = [](const Key& x, const Key& y) { return x.nu < y.nu || (x.nu == y.nu && x.i < y.i); };
    std::vector<Key> a((size_t)n), b((size_t)n);
    host_ranges(n, 8, [&](int64_t i0, int64_t i1, int) {
        for (int64_t i = i0; i < i1; ++i) a[(size_t)i] = Key{nu[i], i};
    });
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    int parts = 1;
    while (parts * 2 <= (int)std::min(8u, hw) && n >= ((int64_t)1 << 16)) parts *= 2;
    std::vector<int64_t> bound((size_t)parts + 1);
    for (int k = 0; k <= parts; ++k) bound[(size_t)k] = n * k / parts;
    auto on_threads = [](int count, auto fn) {
        std::vector<std::thread> th;
        for (int k = 0; k < count; ++k) th.emplace_back(fn, k);
        for (auto& x : th) x.join();
    };
    on_threads(parts, [&](int k) { std::sort(a.begin() + bound[(size_t)k], a.begin() + bound[(size_t)k + 1], less); });
    for (int w = 1; w < parts; w *= 2) {
        on_threads(parts / (2 * w), [&](int m) {
            const size_t lo = (size_t)bound[(size_t)(2 * w * m)], mid = (size_t)bound[(size_t)(2 * w * m + w)];
            const size_t hi = (size_t)bound[(size_t)(2 * w * m + 2 * w)];
            std::merge(a.begin() + lo, a.begin() + mid, a.begin() + mid, a.begin() + hi, b.begin() + lo, less);
        });
        a.swap(b);
    }
    std::vector<int64_t> perm((size_t)n);
    host_ranges(n, 8, [&](int64_t i0, int64_t i1, int) {
        for (int64_t i = i0; i < i1; ++i) perm[(size_t)i] = a[(size_t)i].i;
    });
    return perm;
}

// Writes a validated list as field arrays of n values (dst[k n + i], k = 0
// .. 7: nu, S_ref, E_lower, gamma_air, n_air, gamma_self, delta, A21) in
// ascending (nu, input index) order; absent optional fields are not written
// (the launches use gamma_air for gamma_self and read no delta or A21).  A
// list already in non-decreasing nu (sorted, as scan_lists found) is copied
// as it is (a stable sort would not move it).
void order_lines(const hk_lines* L, bool sorted, double* dst)
{
    const int64_t n = L->n;
    if (n == 0) return;
    const double* src[8] = {L->nu, L->S_ref, L->E_lower, L->gamma_air, L->n_air, L->gamma_self, L->delta, L->A21};
    if (sorted) {  // one thread: the copy runs at memory speed (as fast as eight threads made per piece)
        for (int k = 0; k < 8; ++k)
            if (src[k]) std::memcpy(dst + (size_t)k * n, src[k], (size_t)n * sizeof(double));
        return;
    }
    const std::vector<int64_t> perm = line_order(L->nu, n);
    host_ranges(n, 8, [&](int64_t i0, int64_t i1, int) {
        for (int k = 0; k < 8; ++k) {
            double* d = dst + (size_t)k * n;
            if (src[k])
                for (int64_t i = i0; i < i1; ++i) d[i] = src[k][perm[(size_t)i]];
        }
    });
}

// Runs (first field, field count) of the fields order_lines writes, for the
// copies to the device (none for an empty list).
std::vector<std::pair<size_t, size_t>> present_fields(const hk_lines* L)
{
    std::vector<std::pair<size_t, size_t>> f;
    if (L->n == 0) return f;
    f.push_back({0, 5});
    if (L->gamma_self) f.push_back({5, 1});
    if (L->delta) f.push_back({6, 1});
    if (L->A21) f.push_back({7, 1});
    return f;
}

}  // namespace

namespace {

constexpr int32_t kCountBlocks = 256;  // partial sums per evaluation count

// Partial sums sized by their bound up to this many bytes; beyond it (grids
// above ~2e7 points) the plan is read back instead.
constexpr int64_t kPlanBoundBytes = (int64_t)1 << 30;

// The work plan of n_states states (work_plan.hip): reference tile ranges
// for reach[s], segment lengths, then the items of the tiles whose ranges
// (2 n_tiles per state) are given, into pb.  exact, or a bound above
// kPlanBoundBytes: read the totals back (one host synchronisation) for
// *items and the partial sums; else their bounds.
int make_plan(hk_ctx* ctx, PlanBufs& pb, const int64_t* ranges, int64_t n_tiles, int32_t n_states,
              const double* reach, int32_t tp, int64_t min_seg, const hk_grid* grid, bool exact, WorkPlan* wp,
              hipStream_t strm, const double* reach_dev = nullptr)
{
    const int64_t n = ctx->n_lines;
    const int32_t np = (int32_t)grid->n_points;
    const int64_t n_ref = ((int64_t)np + kRefTilePoints - 1) / kRefTilePoints;
    const int64_t P = n_tiles * n_states;
    HK_HIP(ctx, pb.ref.ensure((size_t)std::max<int64_t>(n_ref * n_states, 1) * 2 * sizeof(int64_t)),
           "allocating the work plan");
    HK_HIP(ctx, pb.seg.ensure((size_t)std::max(n_states, 1) * sizeof(int64_t)), "allocating the work plan");
    HK_HIP(ctx, pb.first.ensure((size_t)std::max<int64_t>(P, 1) * sizeof(int64_t)), "allocating the work plan");
    HK_HIP(ctx, pb.slot.ensure((size_t)std::max<int64_t>(P, 1) * sizeof(int64_t)), "allocating the work plan");
    HK_HIP(ctx, pb.bsum.ensure((size_t)plan_scratch_count(P) * sizeof(int64_t)), "allocating the work plan");
    HK_HIP(ctx, pb.total.ensure(2 * sizeof(int64_t)), "allocating the work plan");
    int64_t* ref = static_cast<int64_t*>(pb.ref.p);
    int64_t* seg = static_cast<int64_t*>(pb.seg.p);
    int64_t* first = static_cast<int64_t*>(pb.first.p);
    int64_t* slot = static_cast<int64_t*>(pb.slot.p);
    int64_t* total = static_cast<int64_t*>(pb.total.p);
    const double* nu = lines_field(ctx, 0);
    if (reach_dev)  // reach_dev: the same reaches on the device, every state in one launch
        HK_HIP(ctx, launch_tile_ranges(nu, n, n_ref, kRefTilePoints, grid->nu_min, grid->dnu, np, 0.0, ref, strm,
                                       reach_dev, n_states),
               "tile_ranges");
    else
        for (int32_t s = 0; s < n_states; ++s)
            HK_HIP(ctx, launch_tile_ranges(nu, n, n_ref, kRefTilePoints, grid->nu_min, grid->dnu, np, reach[s],
                                           ref + (int64_t)s * 2 * n_ref, strm),
                   "tile_ranges");
    HK_HIP(ctx, launch_seg_length(ref, n_ref, n_states, np, n, min_seg, seg, strm), "seg_length");
    HK_HIP(ctx, launch_work_plan(ranges, n_tiles, n_states, seg, first, slot, static_cast<int64_t*>(pb.bsum.p), total,
                                 strm),
           "work_plan");
    int64_t items = plan_items_bound(P, n_states);
    int64_t points = n_states * plan_partial_points_bound(np, tp);
    if (exact || points * 8 > kPlanBoundBytes) {
        int64_t h[2] = {0, 0};
        HK_HIP(ctx, hipMemcpyAsync(h, total, sizeof h, hipMemcpyDeviceToHost, strm), "reading the work plan");
        HK_HIP(ctx, hipStreamSynchronize(strm), "hipStreamSynchronize");
        items = h[0];
        points = h[1] * tp;
    }
    HK_HIP(ctx, pb.partial.ensure((size_t)std::max<int64_t>(points, 1) * 8), "allocating partial sums");
    *wp = WorkPlan{seg, first, slot, total, P, items};
    return HK_OK;
}

// The wing stage of n_states states whose records lie n_lines apart: the
// plan, then the wing items and the reduction of cut tiles.  ranges: tile
// ranges for tiles of `ppl` points per lane; reach[s]: state s's wing reach;
// out: kappa (binary64) or the Kahan sums (binary32, with comp), n_points
// per state.
int wing_stage(hk_ctx* ctx, int precision, int ppl, const void* recs, const WingIdx* idx, const int64_t* ranges,
               int64_t n_tiles, int32_t n_states, const double* reach, const hk_grid* grid, void* out, float* comp,
               int accumulate, bool exact)
{
    const bool f64 = precision == HK_F64;
    const int32_t tp = f64 ? opacity_f64_tile_points(ppl) : opacity_f32_tile_points(ppl);
    WorkPlan wp;
    // binary32: segments of whole 256-line compensation blocks
    if (int rc = make_plan(ctx, ctx->ln.wplan, ranges, n_tiles, n_states, reach, tp, f64 ? 64 : 256, grid, exact, &wp,
                           ctx->stream))
        return rc;
    const int64_t n = ctx->n_lines;
    const int32_t np = (int32_t)grid->n_points;
    if (f64)
        HK_HIP(ctx, launch_wing_f64(ppl, static_cast<const WingRec*>(recs), idx, ranges, n, n_tiles, n_states, wp,
                                    grid->nu_min, grid->dnu, np, static_cast<double*>(out),
                                    static_cast<double*>(ctx->ln.wplan.partial.p), accumulate, ctx->wing_edge_paths, ctx->stream),
               "wing_f64");
    else
        HK_HIP(ctx, launch_wing_f32(ppl, static_cast<const WingRec32*>(recs), idx, ranges, n, n_tiles, n_states, wp,
                                    np, static_cast<float*>(out), comp,
                                    static_cast<float2*>(ctx->ln.wplan.partial.p), ctx->wing_edge_paths, ctx->stream),
               "wing_f32");
    return HK_OK;
}

// The side stream (the series beside the wing) and its fork / join
// events, made on first use.
int ensure_side(hk_ctx* ctx)
{
    if (ctx->side) return HK_OK;
    HK_HIP(ctx, hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking), "hipStreamCreate");
    HK_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming), "hipEventCreate");
    HK_HIP(ctx, hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming), "hipEventCreate");
    return HK_OK;
}

// Clears the running count of surrogate evaluations (stream-ordered, by a
// fill kernel), at the start of each hk_opacity / hk_opacity_stream call.
int reset_surrogate_count(hk_ctx* ctx)
{
    HK_HIP(ctx, ctx->sg_used_total.ensure(sizeof(int64_t)), "allocating surrogate counters");
    HK_HIP(ctx, launch_zero(ctx->sg_used_total.p, sizeof(int64_t), ctx->stream), "zero");
    return HK_OK;
}

// Times the batched wing kernel at 2, 4 and 8 points per lane on the first
// states of a batch (one untimed launch, then one timed launch each) and
// returns the fastest shape.  The shapes give identical results, so the
// choice affects time only.
int autotune_wing(hk_ctx* ctx, int precision, const hk_state* states, int32_t n_try, const hk_grid* grid,
                  int* best_out)
{
    const int64_t n = ctx->n_lines;
    const int32_t np = (int32_t)grid->n_points;
    const double* nu = lines_field(ctx, 0);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HK_HIP(ctx, hipEventCreate(&e0), "hipEventCreate");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(ctx, HK_EDEVICE, "hipEventCreate failed");
    }
    int best = 0;
    float best_ms = 0.0f;
    hipError_t err = hipSuccess;
    std::vector<double> reach((size_t)n_try);
    for (int32_t s = 0; s < n_try; ++s) reach[(size_t)s] = wing_reach(ctx, &states[s], grid);
    for (int cand : {2, 4, 8}) {
        if (precision == HK_F64 && cand == 2) continue;  // binary64 groups points by four
        const int32_t tp = precision == HK_F64 ? opacity_f64_tile_points(cand) : opacity_f32_tile_points(cand);
        const int64_t n_tiles = ((int64_t)np + tp - 1) / tp;
        err = ctx->tb_ranges.ensure((size_t)std::max<int64_t>(n_tiles * n_try, 1) * 2 * sizeof(int64_t));
        if (err != hipSuccess) break;
        int64_t* ranges = static_cast<int64_t*>(ctx->tb_ranges.p);
        for (int32_t s = 0; s < n_try && err == hipSuccess; ++s)
            err = launch_tile_ranges(nu, n, n_tiles, tp, grid->nu_min, grid->dnu, np,
                                     wing_reach(ctx, &states[s], grid), ranges + (int64_t)s * 2 * n_tiles,
                                     ctx->stream);
        float ms = 0.0f;
        for (int rep = 0; rep < 2 && err == hipSuccess; ++rep) {
            if (rep == 1) err = hipEventRecord(e0, ctx->stream);
            if (err != hipSuccess) break;
            const void* recs = precision == HK_F64 ? ctx->tb_wing.p : ctx->tb_w32.p;
            if (int rc = wing_stage(ctx, precision, cand, recs, static_cast<WingIdx*>(ctx->tb_idx.p), ranges, n_tiles,
                                    n_try, reach.data(), grid, ctx->tb_out.p, static_cast<float*>(ctx->tb_comp.p), 0,
                                    false)) {
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return rc;
            }
            if (rep == 1) {
                err = hipEventRecord(e1, ctx->stream);
                if (err == hipSuccess) err = hipEventSynchronize(e1);
                if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
            }
        }
        if (err != hipSuccess) break;
        if (best == 0 || ms < best_ms) {
            best = cand;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return hip_fail(ctx, err, "autotuning the opacity tiles");
    *best_out = best;
    return HK_OK;
}

}  // namespace

namespace {

// Thin QR of the m x nc Chebyshev design matrix A[i][c] = T_c(t_i),
// t_i = 2 (i + 1/2)/m - 1, by Householder reflections (Golub & Van Loan,
// Alg. 5.2.1): Q row-major [m][nc], R row-major [nc][nc] upper triangular.
void chebyshev_qr(int64_t m, int nc, std::vector<double>& Q, std::vector<double>& R)
{
    std::vector<double> A((size_t)m * nc);
    for (int64_t i = 0; i < m; ++i) {
        const double t = 2.0 * ((double)i + 0.5) / (double)m - 1.0;
        double tm = 1.0, tc = t;
        A[(size_t)i * nc] = 1.0;
        if (nc > 1) A[(size_t)i * nc + 1] = t;
        for (int c = 2; c < nc; ++c) {
            const double tn = 2.0 * t * tc - tm;
            tm = tc;
            tc = tn;
            A[(size_t)i * nc + c] = tn;
        }
    }
    std::vector<std::vector<double>> V(nc);  // reflector k acts on rows k..m-1
    for (int k = 0; k < nc; ++k) {
        double nrm = 0.0;
        for (int64_t i = k; i < m; ++i) nrm += A[(size_t)i * nc + k] * A[(size_t)i * nc + k];
        nrm = std::sqrt(nrm);
        std::vector<double> v((size_t)(m - k));
        for (int64_t i = k; i < m; ++i) v[(size_t)(i - k)] = A[(size_t)i * nc + k];
        const double alpha = v[0] >= 0.0 ? -nrm : nrm;
        v[0] -= alpha;
        double vn = 0.0;
        for (double x : v) vn += x * x;
        if (vn > 0.0) {
            for (int c = k; c < nc; ++c) {
                double dot = 0.0;
                for (int64_t i = k; i < m; ++i) dot += v[(size_t)(i - k)] * A[(size_t)i * nc + c];
                const double f = 2.0 * dot / vn;
                for (int64_t i = k; i < m; ++i) A[(size_t)i * nc + c] -= f * v[(size_t)(i - k)];
            }
        }
        V[k] = std::move(v);
    }
    R.assign((size_t)nc * nc, 0.0);
    for (int r = 0; r < nc; ++r)
        for (int c = r; c < nc; ++c) R[(size_t)r * nc + c] = A[(size_t)r * nc + c];
    // Q = H_0 ... H_{nc-1} applied to the first nc columns of the identity
    Q.assign((size_t)m * nc, 0.0);
    for (int c = 0; c < nc; ++c) Q[(size_t)c * nc + c] = 1.0;
    for (int k = nc - 1; k >= 0; --k) {
        const std::vector<double>& v = V[k];
        double vn = 0.0;
        for (double x : v) vn += x * x;
        if (vn == 0.0) continue;
        for (int c = 0; c < nc; ++c) {
            double dot = 0.0;
            for (int64_t i = k; i < m; ++i) dot += v[(size_t)(i - k)] * Q[(size_t)i * nc + c];
            const double f = 2.0 * dot / vn;
            for (int64_t i = k; i < m; ++i) Q[(size_t)i * nc + c] -= f * v[(size_t)(i - k)];
        }
    }
}

int upload_qr(hk_ctx* ctx, int64_t m, int nc, DevBuf& dQ, DevBuf& dR)
{
    std::vector<double> Q, R;
    chebyshev_qr(m, nc, Q, R);
    HK_HIP(ctx, dQ.ensure(Q.size() * sizeof(double)), "allocating QR factors");
    HK_HIP(ctx, dR.ensure(R.size() * sizeof(double)), "allocating QR factors");
    HK_HIP(ctx, hipMemcpy(dQ.p, Q.data(), Q.size() * sizeof(double), hipMemcpyHostToDevice), "copying QR factors");
    HK_HIP(ctx, hipMemcpy(dR.p, R.data(), R.size() * sizeof(double), hipMemcpyHostToDevice), "copying QR factors");
    return HK_OK;
}

}  // namespace

void hk::set_thread_error(const char* msg) { t_err = msg; }

extern "C" {

int hk_version(void) { return 100; }

const char* hk_last_error(const hk_ctx* ctx)
{
    if (ctx) return ctx->err.c_str();
    return t_err.c_str();
}

int hk_create(int device, hk_ctx** out)
{
    if (!out) return fail(nullptr, HK_EINVAL, "out is NULL");
    if (surrogate_n_params() != HK_SURR_N_PARAMS || surrogate_cells() != HK_SURR_CELLS_X * HK_SURR_CELLS_Y)
        return fail(nullptr, HK_EUNSUPPORTED, "surrogate layout differs from hk.h");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0)
        return fail(nullptr, HK_EDEVICE, "no HIP device available (%s)", hipGetErrorString(e));
    if (device < 0 || device >= n) return fail(nullptr, HK_EINVAL, "device %d out of range [0, %d)", device, n);
    hk_ctx* ctx = new (std::nothrow) hk_ctx();
    if (!ctx) return fail(nullptr, HK_ENOMEM, "out of host memory");
    ctx->device = device;
    e = hipSetDevice(device);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->own, hipStreamNonBlocking);
    if (e != hipSuccess) {
        int rc = hip_fail(nullptr, e, "hk_create");
        delete ctx;
        return rc;
    }
    ctx->stream = ctx->own;
    // the no-allocation sort array of this device: its address, taken once
    // per context with the device current
    e = noalloc_scratch_address(&ctx->noalloc_scratch);
    if (e != hipSuccess) {
        int rc = hip_fail(nullptr, e, "hk_create: address of the fixed sort scratch");
        (void)hipStreamDestroy(ctx->own);
        delete ctx;
        return rc;
    }
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0) {
        ctx->lds_bytes = std::min<int64_t>(lds, kSortLdsBytes);
        ctx->lds_max = lds;
    }
    *out = ctx;
    return HK_OK;
}

int hk_destroy(hk_ctx* ctx)
{
    if (!ctx) return HK_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    for (hipStream_t x : {ctx->side, ctx->wing_s})
        if (x) (void)hipStreamSynchronize(x);
    ctx->lines.release();
    ctx->lines_alt.release();
    ctx->st_counts.release();
    for (int x = 0; x < 2; ++x)
        if (ctx->pin[x]) (void)hipHostFree(ctx->pin[x]);
    ctx->ln.release();
    ctx->ln_alt.release();
    for (hipEvent_t e : {ctx->ev_copied[0], ctx->ev_copied[1], ctx->ev_cfork[0], ctx->ev_cfork[1], ctx->ev_ccore[0],
                         ctx->ev_ccore[1], ctx->ev_cwing[0], ctx->ev_cwing[1], ctx->ev_kappa, ctx->ev_fork,
                         ctx->ev_join})
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t x : {ctx->side, ctx->wing_s})
        if (x) (void)hipStreamDestroy(x);
    ctx->partial.release();
    ctx->kscratch.release();
    for (DevBuf* b : {&ctx->tb_idx, &ctx->tb_wing, &ctx->tb_core, &ctx->tb_w32, &ctx->tb_c32, &ctx->tb_ranges,
                      &ctx->tb_ranges_c, &ctx->tb_out, &ctx->tb_comp, &ctx->tb_scale, &ctx->tb_kappa,
                      &ctx->tb_counts, &ctx->tb_series, &ctx->tb_prep})
        b->release();
    for (DevBuf* b : {&ctx->sg_theta, &ctx->sg_m, &ctx->sg_v, &ctx->sg_copy, &ctx->sg_part, &ctx->sg_ploss,
                      &ctx->sg_err, &ctx->sg_mask, &ctx->sg_used_total, &ctx->rs_Q, &ctx->rs_R, &ctx->rs_Ql, &ctx->rs_Rl,
                      &ctx->rs_quad})
        b->release();
    for (auto& p : ctx->pending) {
        (void)hipEventDestroy(p.second.first);
        (void)hipEventDestroy(p.second.second);
    }
    for (hipEvent_t e : ctx->free_events) (void)hipEventDestroy(e);
    if (ctx->own) (void)hipStreamDestroy(ctx->own);
    delete ctx;
    return HK_OK;
}

int hk_set_stream(hk_ctx* ctx, void* hip_stream)
{
    if (int rc = check_ctx(ctx)) return rc;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return HK_OK;
}

int hk_sync(hk_ctx* ctx)
{
    if (int rc = check_ctx(ctx)) return rc;
    HK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    HK_HIP(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    return HK_OK;
}

}  // extern "C"

namespace {

// The message of line i of a list that breaks a rule of hk_load_lines
// (values in L at index i; `shown` is the index the message names).
int bad_line(hk_ctx* ctx, const hk_lines* L, int64_t i, int64_t shown)
{
    const long long li = (long long)shown;
    if (!isfin(L->nu[i]) || !(L->nu[i] > 0.0))
        return fail(ctx, HK_EINVAL, "nu[%lld] = %g must be finite and > 0", li, L->nu[i]);
    if (!isfin(L->S_ref[i]) || !(L->S_ref[i] >= 0.0))
        return fail(ctx, HK_EINVAL, "S_ref[%lld] = %g must be finite and >= 0", li, L->S_ref[i]);
    if (!isfin(L->E_lower[i])) return fail(ctx, HK_EINVAL, "E_lower[%lld] is not finite", li);
    if (!isfin(L->gamma_air[i]) || !(L->gamma_air[i] >= 0.0))
        return fail(ctx, HK_EINVAL, "gamma_air[%lld] must be finite and >= 0", li);
    if (!isfin(L->n_air[i])) return fail(ctx, HK_EINVAL, "n_air[%lld] is not finite", li);
    if (L->gamma_self && (!isfin(L->gamma_self[i]) || !(L->gamma_self[i] >= 0.0)))
        return fail(ctx, HK_EINVAL, "gamma_self[%lld] must be finite and >= 0", li);
    if (L->delta && !isfin(L->delta[i])) return fail(ctx, HK_EINVAL, "delta[%lld] is not finite", li);
    return fail(ctx, HK_EINVAL, "A21[%lld] must be finite and >= 0", li);
}

// The check of a list in device memory (the rules of check_lines) and its
// bounds (as scan_lists finds them), by a kernel; one synchronisation.
// *sorted: nu is already non-decreasing.
int check_lines_device(hk_ctx* ctx, const hk_lines* L, ListInfo* li, bool* sorted)
{
    const int64_t n = L->n;
    *li = ListInfo();
    li->has_self = L->gamma_self != nullptr;
    li->has_delta = L->delta != nullptr;
    li->has_A = L->A21 != nullptr;
    *sorted = true;
    if (n == 0) return HK_OK;
    LinesDev D;
    D.nu = L->nu;
    D.S_ref = L->S_ref;
    D.E_lower = L->E_lower;
    D.gamma_air = L->gamma_air;
    D.n_air = L->n_air;
    D.gamma_self = L->gamma_self;
    D.delta = L->delta;
    D.A21 = L->A21;
    D.n = n;
    const int32_t nb = check_lines_blocks(n);
    DevBuf part;
    std::vector<CheckPart> h((size_t)nb);
    hipError_t e = part.ensure((size_t)nb * sizeof(CheckPart));
    if (e == hipSuccess) e = launch_check_lines(D, part.p, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h.data(), part.p, h.size() * sizeof(CheckPart), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    part.release();
    if (e != hipSuccess) return hip_fail(ctx, e, "checking the line list on the device");
    CheckPart c = h[0];
    for (const CheckPart& b : h) {
        c.first_bad = std::min(c.first_bad, b.first_bad);
        c.first_unordered = std::min(c.first_unordered, b.first_unordered);
        c.max_abs_delta = std::max(c.max_abs_delta, b.max_abs_delta);
        c.max_gamma_air = std::max(c.max_gamma_air, b.max_gamma_air);
        c.max_gamma_self = std::max(c.max_gamma_self, b.max_gamma_self);
        c.max_A21 = std::max(c.max_A21, b.max_A21);
        c.min_n_air = std::min(c.min_n_air, b.min_n_air);
        c.max_n_air = std::max(c.max_n_air, b.max_n_air);
        c.nu_max = std::max(c.nu_max, b.nu_max);
    }
    if (c.first_bad < n) {  // read that line back for the message
        const int64_t i = c.first_bad;
        double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        const double* src[8] = {L->nu, L->S_ref, L->E_lower, L->gamma_air, L->n_air, L->gamma_self, L->delta, L->A21};
        for (int k = 0; k < 8; ++k)
            if (src[k]) HK_HIP(ctx, hipMemcpy(&v[k], src[k] + i, sizeof(double), hipMemcpyDeviceToHost), "reading a line");
        hk_lines one{1, &v[0], &v[1], &v[2], &v[3], &v[4], L->gamma_self ? &v[5] : nullptr,
                     L->delta ? &v[6] : nullptr, L->A21 ? &v[7] : nullptr};
        return bad_line(ctx, &one, 0, i);
    }
    li->max_abs_delta = c.max_abs_delta;
    li->max_gamma_air = c.max_gamma_air;
    li->max_gamma_self = c.max_gamma_self;
    li->max_A21 = c.max_A21;
    li->min_n_air = c.min_n_air;
    li->max_n_air = c.max_n_air;
    li->nu_max = c.nu_max;
    *sorted = c.first_unordered >= n;
    return HK_OK;
}

}  // namespace

extern "C" {

int hk_load_lines(hk_ctx* ctx, const hk_lines* L, const hk_species* sp, int lines_on_device)
{
    if (!L || !sp) return fail(ctx, HK_EINVAL, "lines and species must not be NULL");
    if (L->n < 0 || L->n > (int64_t)INT32_MAX) return fail(ctx, HK_EINVAL, "line count %lld out of range", (long long)L->n);
    if (int rc = check_species(ctx, sp)) return rc;
    ListScan scan;
    if (!lines_on_device) {
        if (!lines_shape_ok(L)) return check_lines(ctx, L, -1);
        scan = scan_lists(L, 1)[0];
        if (scan.bad) return check_lines(ctx, L, -1);
    }
    if (int rc = check_ctx(ctx)) return rc;
    const int64_t n = L->n;
    if (lines_on_device && n > 0 && (!L->nu || !L->S_ref || !L->E_lower || !L->gamma_air || !L->n_air))
        return fail(ctx, HK_EINVAL, "nu, S_ref, E_lower, gamma_air and n_air are required");
    HK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    ListInfo li;
    bool sorted = true;
    if (lines_on_device) {
        if (int rc = check_lines_device(ctx, L, &li, &sorted)) return rc;
    } else {
        li = scan.info;
        sorted = scan.sorted;
    }
    HK_HIP(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    ctx->n_lines = n;
    ctx->lines_loaded = false;
    ctx->have_run = false;
    ctx->last_stream_chunks = 0;
    const size_t cap = (size_t)8 * (size_t)(n > 0 ? n : 1);
    HK_HIP(ctx, ctx->lines.ensure(cap * sizeof(double)), "allocating the line list");
    const double* src[8] = {L->nu, L->S_ref, L->E_lower, L->gamma_air, L->n_air, L->gamma_self, L->delta, L->A21};
    double* dst = static_cast<double*>(ctx->lines.p);
    const hipMemcpyKind kind = lines_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    const auto fields = present_fields(L);
    if (sorted) {
        for (const auto& f : fields)
            for (size_t k = f.first; k < f.first + f.second; ++k)
                HK_HIP(ctx, hipMemcpyAsync(dst + k * n, src[k], (size_t)n * sizeof(double), kind, ctx->stream),
                       "copying the line list");
    } else {
        // ordered on the device: a host list is first copied as it is
        DevBuf staging, scratch;
        hipError_t e = hipSuccess;
        const double* dsrc[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
        if (lines_on_device) {
            for (int k = 0; k < 8; ++k) dsrc[k] = src[k];
        } else {
            e = staging.ensure(cap * sizeof(double));
            for (const auto& f : fields)
                for (size_t k = f.first; k < f.first + f.second && e == hipSuccess; ++k) {
                    double* d = static_cast<double*>(staging.p) + k * n;
                    e = hipMemcpyAsync(d, src[k], (size_t)n * sizeof(double), hipMemcpyHostToDevice, ctx->stream);
                    dsrc[k] = d;
                }
        }
        const uint32_t* perm = nullptr;
        if (e == hipSuccess) e = scratch.ensure(line_sort_scratch_bytes(n));
        if (e == hipSuccess) e = launch_line_order(dsrc[0], n, scratch.p, &perm, ctx->stream);
        for (const auto& f : fields)
            for (size_t k = f.first; k < f.first + f.second && e == hipSuccess; ++k)
                e = launch_gather(dsrc[k], perm, n, dst + k * n, ctx->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        staging.release();
        scratch.release();
        if (e != hipSuccess) return hip_fail(ctx, e, "ordering the line list");
    }
    HK_HIP(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    ctx->li = li;
    ctx->species = *sp;
    ctx->lines_loaded = true;
    return HK_OK;
}

// One opacity pass between its launch and its finish: the streams of its
// preparation and finish and of its series, the fork event after which the
// wing may run and the series' end, and what the wing launch and the finish
// take.  Its
// pointers are those of the lane it was launched with.
struct Flight {
    int precision = HK_F64;
    hipStream_t s = nullptr, cs = nullptr;  // preparation and finish; the series
    hipEvent_t fork = nullptr, core_done = nullptr;
    double* kappa = nullptr;
    int accumulate = 0;
    int32_t np = 0;
    int64_t n = 0;
    // the wing
    int ppl = 0;
    const void* recs = nullptr;  // WingRec (binary64) or WingRec32
    const WingIdx* widx = nullptr;
    const int64_t* ranges = nullptr;
    int64_t n_tiles = 0;
    WorkPlan wwp{};
    void* wpartial = nullptr;
    double nu_min = 0.0, dnu = 0.0;
    // the finish: the series grid, the binary32 sums and scale
    void* series = nullptr;
    float *fs = nullptr, *fc = nullptr;
    int32_t* scale = nullptr;
    // HK_F32_SURROGATE: the series launch's per-workgroup counts
    const int64_t* sg_used = nullptr;
    int64_t used_n = 0;
};

// Binary32 profiles with compensated binary32 sums, after the binary64 line
// preparation: scale, binary32 records, tile ranges and both plans on f->s,
// then the series on f->cs; the wing and kappa = (sum + comp) 2^-s in
// binary64 are left to flight_wing and flight_finish.
static int launch_f32_pass(hk_ctx* ctx, const hk_grid* grid, double reach, double reach_core, WingRec* wing,
                           WingIdx* widx, CoreRec* core, const int64_t* ranges_c, int64_t n_tiles_c, bool surrogate,
                           Flight* f)
{
    const hipStream_t s = f->s;
    const int64_t n = ctx->n_lines;
    const int32_t np = (int32_t)grid->n_points;
    const size_t nb = (size_t)std::max<int64_t>(n, 1);
    const int32_t nblk = 256;
    HK_HIP(ctx, ctx->ln.w32.ensure(nb * sizeof(WingRec32)), "allocating binary32 records");
    HK_HIP(ctx, ctx->ln.c32.ensure(nb * sizeof(CoreRec32)), "allocating binary32 records");
    HK_HIP(ctx, ctx->ln.f32sum.ensure((size_t)std::max(np, 1) * sizeof(float)), "allocating binary32 sums");
    HK_HIP(ctx, ctx->ln.f32comp.ensure((size_t)std::max(np, 1) * sizeof(float)), "allocating binary32 sums");
    HK_HIP(ctx, ctx->ln.f32scale.ensure(sizeof(int32_t)), "allocating the scale");
    HK_HIP(ctx, ctx->ln.f32partial.ensure((size_t)nblk * sizeof(double)), "allocating the scale");
    WingRec32* w32 = static_cast<WingRec32*>(ctx->ln.w32.p);
    CoreRec32* c32 = static_cast<CoreRec32*>(ctx->ln.c32.p);
    int32_t* scale = static_cast<int32_t*>(ctx->ln.f32scale.p);
    const int ppl = ctx->f32_points_per_lane;
    const int32_t tp = opacity_f32_tile_points(ppl);
    const int64_t n_tiles = ((int64_t)np + tp - 1) / tp;
    HK_HIP(ctx, ctx->ln.ranges.ensure((size_t)std::max<int64_t>(n_tiles, 1) * 2 * sizeof(int64_t)),
           "allocating tile ranges");
    int64_t* ranges = static_cast<int64_t*>(ctx->ln.ranges.p);
    {
        StageTimer tm(ctx, HK_STAGE_LINE_PREP, s);
        if (n > 0) {
            HK_HIP(ctx, launch_f32_scale(wing, core, n, static_cast<double*>(ctx->ln.f32partial.p), nblk, scale, s),
                   "f32_scale");
            HK_HIP(ctx, launch_line_prep_f32(wing, widx, core, n, grid->nu_min, grid->dnu, scale, w32, c32, s),
                   "line_prep_f32");
        } else {
            HK_HIP(ctx, launch_zero(scale, sizeof(int32_t), s), "zero");
        }
        HK_HIP(ctx, launch_tile_ranges(static_cast<double*>(ctx->lines.p), n, n_tiles, tp, grid->nu_min,
                                       grid->dnu, np, reach, ranges, s),
               "tile_ranges");
        tm.stop();
    }
    // as in binary64: both plans, then the series on its stream into its own
    // grid while the wing runs; the finish adds it
    HK_HIP(ctx, ctx->ln.kc.ensure((size_t)std::max(np, 1) * sizeof(double)), "allocating the series grid");
    WorkPlan wwp, cwp;
    {
        StageTimer tm(ctx, HK_STAGE_LINE_PREP, s);
        // segments of whole 256-line compensation blocks for the wing
        if (int rc = make_plan(ctx, ctx->ln.wplan, ranges, n_tiles, 1, &reach, tp, 256, grid, false, &wwp, s))
            return rc;
        if (int rc = make_plan(ctx, ctx->ln.cplan, ranges_c, n_tiles_c, 1, &reach_core, core_f32_tile_points(), 64,
                               grid, false, &cwp, s))
            return rc;
        tm.stop();
    }
    HK_HIP(ctx, hipEventRecord(f->fork, s), "hipEventRecord");
    HK_HIP(ctx, hipStreamWaitEvent(f->cs, f->fork, 0), "hipStreamWaitEvent");
    const int64_t used_n = surrogate ? plan_blocks(cwp.launch_items) : 0;
    {
        StageTimer tm(ctx, HK_STAGE_CORE, f->cs);
        if (surrogate)
            HK_HIP(ctx, ctx->ln.sg_used.ensure((size_t)std::max<int64_t>(used_n, 1) * sizeof(int64_t)),
                   "allocating surrogate counters");
        HK_HIP(ctx, launch_core_f32(widx, c32, ranges_c, n, n_tiles_c, 1, cwp, np, static_cast<float*>(ctx->ln.kc.p),
                                    static_cast<float*>(ctx->ln.cplan.partial.p), surrogate ? ctx->sg_copy.p : nullptr,
                                    surrogate ? static_cast<const uint8_t*>(ctx->sg_mask.p) : nullptr,
                                    surrogate ? static_cast<int64_t*>(ctx->ln.sg_used.p) : nullptr, used_n,
                                    f->cs),
               "core_f32");
        tm.stop();
    }
    HK_HIP(ctx, hipEventRecord(f->core_done, f->cs), "hipEventRecord");
    f->ppl = ppl;
    f->recs = w32;
    f->ranges = ranges;
    f->n_tiles = n_tiles;
    f->wwp = wwp;
    f->wpartial = ctx->ln.wplan.partial.p;
    f->series = ctx->ln.kc.p;
    f->fs = static_cast<float*>(ctx->ln.f32sum.p);
    f->fc = static_cast<float*>(ctx->ln.f32comp.p);
    f->scale = scale;
    if (surrogate && n_tiles_c > 0) {
        f->sg_used = static_cast<const int64_t*>(ctx->ln.sg_used.p);
        f->used_n = used_n;
    }
    return HK_OK;
}

// The argument rules of hk_opacity and hk_opacity_stream (no device).
static int check_opacity_args(hk_ctx* ctx, const hk_state* st, const hk_grid* grid, int precision, void* kappa)
{
    if (int rc = check_state(ctx, st)) return rc;
    if (int rc = check_grid(ctx, grid)) return rc;
    if (precision != HK_F64 && precision != HK_F32_KAHAN && precision != HK_F32_SURROGATE)
        return fail(ctx, HK_EINVAL, "unknown precision %d", precision);
    if (precision != HK_F64 && !(grid->cutoff_lorentz > 0.0) && !(grid->cutoff / grid->dnu < 8388608.0))
        return fail(ctx, HK_EINVAL, "binary32 profiles need cutoff/dnu < 2^23 (got %g)", grid->cutoff / grid->dnu);
    if (grid->n_points > 0 && !kappa) return fail(ctx, HK_EINVAL, "kappa is NULL");
    return HK_OK;
}

// Launches one state over the loaded list, with ctx->ln's buffers: line
// preparation, tile ranges and both work plans on s, then (event fork) the
// series on stream cs (event core_done at its end).  The wing (flight_wing)
// and the finish (flight_finish) follow.
static int opacity_launch(hk_ctx* ctx, const hk_state* st, const hk_grid* grid, int precision, double* kappa,
                          int accumulate, hipStream_t s, hipStream_t cs, hipEvent_t fork, hipEvent_t core_done,
                          Flight* f)
{
    const int64_t n = ctx->n_lines;
    const int32_t np = (int32_t)grid->n_points;
    *f = Flight{};
    f->precision = precision;
    f->s = s;
    f->cs = cs;
    f->fork = fork;
    f->core_done = core_done;
    f->kappa = kappa;
    f->accumulate = accumulate;
    f->np = np;
    f->n = n;
    f->nu_min = grid->nu_min;
    f->dnu = grid->dnu;

    const PrepParams pp = prep_params(ctx, st, grid);
    ctx->last_P = st->P;

    const size_t nb = (size_t)std::max<int64_t>(n, 1);
    HK_HIP(ctx, ctx->ln.wing.ensure(nb * sizeof(WingRec)), "allocating line records");
    HK_HIP(ctx, ctx->ln.widx.ensure(nb * sizeof(WingIdx)), "allocating line records");
    HK_HIP(ctx, ctx->ln.core.ensure(nb * sizeof(CoreRec)), "allocating line records");
    const int ppl = ctx->f64_points_per_lane;
    const int32_t tp = opacity_f64_tile_points(ppl);
    const int64_t n_tiles = ((int64_t)np + tp - 1) / tp;
    const int32_t tpc = precision == HK_F64 ? core_f64_tile_points() : core_f32_tile_points();
    const int64_t n_tiles_c = ((int64_t)np + tpc - 1) / tpc;
    HK_HIP(ctx, ctx->ln.ranges.ensure((size_t)std::max<int64_t>(n_tiles, 1) * 2 * sizeof(int64_t)),
           "allocating tile ranges");
    HK_HIP(ctx, ctx->ln.ranges_core.ensure((size_t)std::max<int64_t>(n_tiles_c, 1) * 2 * sizeof(int64_t)),
           "allocating tile ranges");

    const LinesDev L = lines_dev(ctx);
    WingRec* wing = static_cast<WingRec*>(ctx->ln.wing.p);
    WingIdx* widx = static_cast<WingIdx*>(ctx->ln.widx.p);
    CoreRec* core = static_cast<CoreRec*>(ctx->ln.core.p);
    int64_t* ranges = static_cast<int64_t*>(ctx->ln.ranges.p);
    const double reach = wing_reach(ctx, st, grid);
    const double reach_core = core_reach(ctx, st, grid, pp);
    int64_t* ranges_c = static_cast<int64_t*>(ctx->ln.ranges_core.p);
    f->widx = widx;

    {
        StageTimer tm(ctx, HK_STAGE_LINE_PREP, s);
        HK_HIP(ctx, launch_line_prep_f64(L, pp, wing, widx, core, s), "line_prep_f64");
        if (precision == HK_F64)  // binary32 wing tiles have their own ranges
            HK_HIP(ctx, launch_tile_ranges(L.nu, n, n_tiles, tp, grid->nu_min, grid->dnu, np, reach, ranges, s),
                   "tile_ranges");
        HK_HIP(ctx, launch_tile_ranges(L.nu, n, n_tiles_c, tpc, grid->nu_min, grid->dnu, np, reach_core,
                                       ranges_c, s),
               "tile_ranges");
        tm.stop();
    }
    if (precision != HK_F64)
        return launch_f32_pass(ctx, grid, reach, reach_core, wing, widx, core, ranges_c, n_tiles_c,
                               precision == HK_F32_SURROGATE, f);
    // The series runs on a second stream, concurrent with the wing (each
    // leaves the VALU idle ~20% of the time, which the other fills), into a
    // grid of its own; the finish adds it to the wing's: kappa_j = wing_j +
    // series_j, the same single addition as adding in place.  Both work plans
    // are made first, on s, so that only the two big kernels run side by
    // side (small kernels queued behind a running one wait for CUs).
    HK_HIP(ctx, ctx->ln.kc.ensure((size_t)std::max(np, 1) * sizeof(double)), "allocating the series grid");
    WorkPlan wwp, cwp;
    {
        StageTimer tm(ctx, HK_STAGE_LINE_PREP, s);
        if (int rc = make_plan(ctx, ctx->ln.wplan, ranges, n_tiles, 1, &reach, tp, 64, grid, false, &wwp, s))
            return rc;
        if (int rc = make_plan(ctx, ctx->ln.cplan, ranges_c, n_tiles_c, 1, &reach_core, tpc, 64, grid, false, &cwp,
                               s))
            return rc;
        tm.stop();
    }
    HK_HIP(ctx, hipEventRecord(fork, s), "hipEventRecord");
    HK_HIP(ctx, hipStreamWaitEvent(f->cs, fork, 0), "hipStreamWaitEvent");
    {
        StageTimer tm(ctx, HK_STAGE_CORE, f->cs);
        HK_HIP(ctx, launch_core_f64(wing, widx, core, ranges_c, n, n_tiles_c, 1, cwp, grid->nu_min, grid->dnu, np,
                                    static_cast<double*>(ctx->ln.kc.p), static_cast<double*>(ctx->ln.cplan.partial.p),
                                    f->cs),
               "core_f64");
        tm.stop();
    }
    HK_HIP(ctx, hipEventRecord(core_done, f->cs), "hipEventRecord");
    f->ppl = ppl;
    f->recs = wing;
    f->ranges = ranges;
    f->n_tiles = n_tiles;
    f->wwp = wwp;
    f->wpartial = ctx->ln.wplan.partial.p;
    f->series = ctx->ln.kc.p;
    return HK_OK;
}

// The wing of a launched pass, on w: f->s's own stream, or another one
// (which then waits for the fork, and for kappa_ready when not null: a
// binary64 wing adds to kappa; wing_done is recorded at its end).
static int flight_wing(hk_ctx* ctx, const Flight& f, hipStream_t w, hipEvent_t kappa_ready, hipEvent_t wing_done)
{
    if (w != f.s) HK_HIP(ctx, hipStreamWaitEvent(w, f.fork, 0), "hipStreamWaitEvent");
    if (kappa_ready) HK_HIP(ctx, hipStreamWaitEvent(w, kappa_ready, 0), "hipStreamWaitEvent");
    StageTimer tm(ctx, HK_STAGE_OPACITY, w);
    if (f.precision == HK_F64)
        HK_HIP(ctx, launch_wing_f64(f.ppl, static_cast<const WingRec*>(f.recs), f.widx, f.ranges, f.n, f.n_tiles, 1,
                                    f.wwp, f.nu_min, f.dnu, f.np, f.kappa, static_cast<double*>(f.wpartial),
                                    f.accumulate ? 1 : 0, ctx->wing_edge_paths, w),
               "wing_f64");
    else
        HK_HIP(ctx, launch_wing_f32(f.ppl, static_cast<const WingRec32*>(f.recs), f.widx, f.ranges, f.n, f.n_tiles,
                                    1, f.wwp, f.np, f.fs, f.fc, static_cast<float2*>(f.wpartial),
                                    ctx->wing_edge_paths, w),
               "wing_f32");
    tm.stop();
    if (w != f.s) HK_HIP(ctx, hipEventRecord(wing_done, w), "hipEventRecord");
    return HK_OK;
}

// The finish of a pass on f.s, after the series (and the wing, when it ran
// on another stream: wing_done): the surrogate's count added to the running
// total, then kappa from the binary32 sums, or the series grid added to it.
static int flight_finish(hk_ctx* ctx, const Flight& f, hipEvent_t wing_done)
{
    if (wing_done) HK_HIP(ctx, hipStreamWaitEvent(f.s, wing_done, 0), "hipStreamWaitEvent");
    HK_HIP(ctx, hipStreamWaitEvent(f.s, f.core_done, 0), "hipStreamWaitEvent");
    if (f.sg_used)
        HK_HIP(ctx, launch_sum_counts(f.sg_used, f.used_n, static_cast<int64_t*>(ctx->sg_used_total.p), 1, f.s),
               "sum_counts");
    if (f.precision == HK_F64)
        HK_HIP(ctx, launch_add_f64(f.kappa, static_cast<const double*>(f.series), f.np, f.s), "add_f64");
    else
        HK_HIP(ctx, launch_f32_finish(f.fs, f.fc, static_cast<const float*>(f.series), f.scale, f.np, f.kappa,
                                      f.accumulate, f.s),
               "f32_finish");
    ctx->have_run = true;
    return HK_OK;
}

// One state over the loaded list on ctx's stream: the launch, the wing on
// the same stream, the finish.
static int opacity_run(hk_ctx* ctx, const hk_state* st, const hk_grid* grid, int precision, double* kappa,
                       int accumulate)
{
    if (int rc = ensure_side(ctx)) return rc;  // makes ev_fork and ev_join
    Flight f;
    if (int rc = opacity_launch(ctx, st, grid, precision, kappa, accumulate, ctx->stream, ctx->side, ctx->ev_fork,
                                ctx->ev_join, &f))
        return rc;
    if (int rc = flight_wing(ctx, f, ctx->stream, nullptr, nullptr)) return rc;
    return flight_finish(ctx, f, nullptr);
}

int hk_opacity(hk_ctx* ctx, const hk_state* st, const hk_grid* grid, int precision, void* kappa,
               void* comp, int accumulate)
{
    // arguments first, the context last: the checks run without a device
    if (int rc = check_opacity_args(ctx, st, grid, precision, kappa)) return rc;
    if (comp) return fail(ctx, HK_EINVAL, "comp must be NULL (kappa holds the result in binary64)");
    if (int rc = check_ctx(ctx)) return rc;
    if (!ctx->lines_loaded) return fail(ctx, HK_ENOTREADY, "no line list loaded (call hk_load_lines first)");
    if (precision == HK_F32_SURROGATE && !ctx->sg_certified)
        return fail(ctx, HK_ENOTREADY, "HK_F32_SURROGATE needs a certified surrogate (hk_surrogate_certify)");
    if (precision != HK_F64 && !(max_cutoff(ctx, st, grid) / grid->dnu < 8388608.0))
        return fail(ctx, HK_EINVAL, "binary32 profiles need (largest cutoff)/dnu < 2^23 (got %g)",
                    max_cutoff(ctx, st, grid) / grid->dnu);
    HK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    ctx->last_tables_states = 0;
    ctx->last_stream_chunks = 0;
    if (int rc = reset_surrogate_count(ctx)) return rc;
    return opacity_run(ctx, st, grid, precision, static_cast<double*>(kappa), accumulate);
}

// Sizes every per-line buffer of opacity_run for lists of up to n lines, so
// that a stream of chunks never reallocates (and so never synchronises) in
// its loop.
static int reserve_line_buffers(hk_ctx* ctx, int64_t n, int precision)
{
    const size_t nb = (size_t)std::max<int64_t>(n, 1);
    for (Lane* l : {&ctx->ln, &ctx->ln_alt}) {
        HK_HIP(ctx, l->wing.ensure(nb * sizeof(WingRec)), "allocating line records");
        HK_HIP(ctx, l->widx.ensure(nb * sizeof(WingIdx)), "allocating line records");
        HK_HIP(ctx, l->core.ensure(nb * sizeof(CoreRec)), "allocating line records");
        if (precision != HK_F64) {
            HK_HIP(ctx, l->w32.ensure(nb * sizeof(WingRec32)), "allocating binary32 records");
            HK_HIP(ctx, l->c32.ensure(nb * sizeof(CoreRec32)), "allocating binary32 records");
        }
    }
    HK_HIP(ctx, ctx->lines.ensure((size_t)8 * nb * sizeof(double)), "allocating the line list");
    HK_HIP(ctx, ctx->lines_alt.ensure((size_t)8 * nb * sizeof(double)), "allocating the line list");
    return HK_OK;
}

static int stream_resources(hk_ctx* ctx, size_t pin_doubles)
{
    if (int rc = ensure_side(ctx)) return rc;
    if (!ctx->wing_s) HK_HIP(ctx, hipStreamCreateWithFlags(&ctx->wing_s, hipStreamNonBlocking), "hipStreamCreate");
    for (hipEvent_t* e : {&ctx->ev_copied[0], &ctx->ev_copied[1], &ctx->ev_cfork[0], &ctx->ev_cfork[1],
                          &ctx->ev_ccore[0], &ctx->ev_ccore[1], &ctx->ev_cwing[0], &ctx->ev_cwing[1], &ctx->ev_kappa})
        if (!*e) HK_HIP(ctx, hipEventCreateWithFlags(e, hipEventDisableTiming), "hipEventCreate");
    if (pin_doubles > ctx->pin_cap) {
        for (int x = 0; x < 2; ++x) {
            if (ctx->pin[x]) (void)hipHostFree(ctx->pin[x]);
            ctx->pin[x] = nullptr;
        }
        ctx->pin_cap = 0;
        for (int x = 0; x < 2; ++x)
            HK_HIP(ctx, hipHostMalloc((void**)&ctx->pin[x], pin_doubles * sizeof(double), hipHostMallocDefault),
                   "allocating pinned staging");
        ctx->pin_cap = pin_doubles;
    }
    return HK_OK;
}

int hk_opacity_stream(hk_ctx* ctx, const hk_lines* chunks, int32_t n_chunks, const hk_species* sp,
                      const hk_state* st, const hk_grid* grid, int precision, double* kappa, int accumulate)
{
    if (int rc = check_opacity_args(ctx, st, grid, precision, kappa)) return rc;
    if (n_chunks < 0 || n_chunks > HK_MAX_CHUNKS)
        return fail(ctx, HK_EINVAL, "n_chunks = %d out of [0, %d]", n_chunks, HK_MAX_CHUNKS);
    if (n_chunks > 0 && !chunks) return fail(ctx, HK_EINVAL, "chunks is NULL");
    if (int rc = check_species(ctx, sp)) return rc;
    // every chunk is checked before any work is enqueued: the shapes, then
    // one pass over the values of the chunks before the first misshapen one;
    // errors are reported in chunk order
    int32_t n_shaped = 0;
    while (n_shaped < n_chunks && lines_shape_ok(&chunks[n_shaped])) ++n_shaped;
    const std::vector<ListScan> scan = scan_lists(chunks, n_shaped);
    std::vector<ListInfo> info((size_t)n_chunks);
    int64_t n_max = 0, n_total = 0;
    for (int32_t c = 0; c < n_chunks; ++c) {
        if (c == n_shaped || scan[(size_t)c].bad) return check_lines(ctx, &chunks[c], c);
        info[(size_t)c] = scan[(size_t)c].info;
        if (precision != HK_F64 && !(max_cutoff(info[(size_t)c], sp->T_ref, st, grid) / grid->dnu < 8388608.0))
            return fail(ctx, HK_EINVAL, "chunk %d: binary32 profiles need (largest cutoff)/dnu < 2^23 (got %g)", c,
                        max_cutoff(info[(size_t)c], sp->T_ref, st, grid) / grid->dnu);
        n_max = std::max(n_max, chunks[c].n);
        n_total += chunks[c].n;
    }
    if (int rc = check_ctx(ctx)) return rc;
    if (precision == HK_F32_SURROGATE && !ctx->sg_certified)
        return fail(ctx, HK_ENOTREADY, "HK_F32_SURROGATE needs a certified surrogate (hk_surrogate_certify)");
    HK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    const int64_t np = grid->n_points;
    if (n_chunks == 0) {  // the opacity of no lines
        if (!accumulate && np > 0)
            HK_HIP(ctx, launch_zero(kappa, (size_t)np * sizeof(double), ctx->stream), "zero");
        return HK_OK;
    }
    // the loaded list is replaced: from here on it is the chunk being computed
    ctx->lines_loaded = false;
    ctx->have_run = false;
    ctx->last_tables_states = 0;
    ctx->last_stream_chunks = 0;
    HK_HIP(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    if (int rc = reserve_line_buffers(ctx, n_max, precision)) return rc;
    if (int rc = stream_resources(ctx, (size_t)8 * (size_t)std::max<int64_t>(n_max, 1))) return rc;
    if (int rc = reset_surrogate_count(ctx)) return rc;
    HK_HIP(ctx, ctx->st_counts.ensure((size_t)kCountBlocks * 3 * (size_t)n_chunks * sizeof(int64_t)),
           "allocating counters");
    ctx->species = *sp;
    // Chunk c is copied and prepared on ctx's stream S with lane c & 1 (device
    // line buffer, records, plans and sums); its series and its wing run on
    // the two other streams (which trade roles from chunk to chunk); its
    // finish (the update of kappa) is enqueued on S after the preparation of
    // chunk c+1, so that chunk c+1 is copied and prepared, and its kernels
    // start, while the kernels of chunk c still run.  The finishes, on S, keep kappa's
    // updates in chunk order (a binary64 wing, which adds to kappa, waits
    // for the previous finish), so the result is that of the chunks one at
    // a time; S waits for both streams in each finish, so the call ends on
    // it.  Lane c & 1 is free again when the finish of chunk c-2, enqueued
    // on S before the copy of chunk c, has run.
    Flight prev;
    auto finish = [&](int32_t c, const Flight& f) -> int {
        if (int rc = flight_finish(ctx, f, ctx->ev_cwing[c & 1])) return rc;
        HK_HIP(ctx, launch_eval_counts(f.widx, f.n,
                                       static_cast<int64_t*>(ctx->st_counts.p) + (size_t)kCountBlocks * 3 * c,
                                       kCountBlocks, ctx->stream),
               "eval_counts");
        return HK_OK;
    };
    auto one_chunk = [&](int32_t c) -> int {
        const int x = c & 1;
        const int64_t n = chunks[c].n;
        // staging x last held chunk c-2: its copy must be done before it is rewritten
        if (c >= 2) HK_HIP(ctx, hipEventSynchronize(ctx->ev_copied[x]), "hipEventSynchronize");
        order_lines(&chunks[c], scan[(size_t)c].sorted, ctx->pin[x]);
        if (c > 0) {  // device buffer and lane x hold chunk c
            std::swap(ctx->lines, ctx->lines_alt);
            std::swap(ctx->ln, ctx->ln_alt);
        }
        for (const auto& f : present_fields(&chunks[c]))
            HK_HIP(ctx, hipMemcpyAsync(static_cast<double*>(ctx->lines.p) + f.first * n, ctx->pin[x] + f.first * n,
                                       (size_t)f.second * n * sizeof(double), hipMemcpyHostToDevice, ctx->stream),
                   "copying a chunk");
        HK_HIP(ctx, hipEventRecord(ctx->ev_copied[x], ctx->stream), "hipEventRecord");
        ctx->n_lines = n;
        ctx->li = info[(size_t)c];
        ctx->lines_loaded = true;
        // the series and the wing trade streams from chunk to chunk, so that
        // the wing of chunk c+1 need not wait for that of chunk c to end
        const hipStream_t ws = x ? ctx->side : ctx->wing_s, cs = x ? ctx->wing_s : ctx->side;
        Flight f;
        if (int rc = opacity_launch(ctx, st, grid, precision, kappa, (accumulate || c > 0) ? 1 : 0, ctx->stream,
                                    cs, ctx->ev_cfork[x], ctx->ev_ccore[x], &f))
            return rc;
        hipEvent_t kappa_ready = nullptr;
        if (c > 0) {
            if (int rc = finish(c - 1, prev)) return rc;
            if (precision == HK_F64) {
                HK_HIP(ctx, hipEventRecord(ctx->ev_kappa, ctx->stream), "hipEventRecord");
                kappa_ready = ctx->ev_kappa;
            }
        }
        if (int rc = flight_wing(ctx, f, ws, kappa_ready, ctx->ev_cwing[x])) return rc;
        prev = f;
        return HK_OK;
    };
    int rc = HK_OK;
    for (int32_t c = 0; c < n_chunks && rc == HK_OK; ++c) rc = one_chunk(c);
    if (rc == HK_OK) rc = finish(n_chunks - 1, prev);
    if (rc != HK_OK) {  // nothing may still run on the other streams
        (void)hipStreamSynchronize(ctx->wing_s);
        (void)hipStreamSynchronize(ctx->side);
        return rc;
    }
    ctx->last_stream_chunks = n_chunks;
    ctx->stream_lines = n_total;
    return HK_OK;
}

int hk_kdist(hk_ctx* ctx, const void* kappa, int precision, int64_t n_points, const hk_bins* bins,
             double* k_out, void* sorted_out)
{
    GValues gv;
    if (int rc = check_bins(ctx, bins, &gv)) return rc;
    if (precision != HK_F64 && precision != HK_F32_KAHAN)
        return fail(ctx, HK_EINVAL, "unknown precision %d", precision);
    if (n_points < 0 || n_points > HK_MAX_POINTS) return fail(ctx, HK_EINVAL, "n_points out of range");
    if (n_points > 0 && (!kappa || !k_out)) return fail(ctx, HK_EINVAL, "kappa and k_out must not be NULL");
    if (int rc = check_ctx(ctx)) return rc;
    HK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    const int eb = precision == HK_F64 ? 8 : 4;
    const size_t sb = kdist_scratch_bytes(eb, n_points, bins->points_per_bin, ctx->lds_bytes, ctx->lds_max);
    if (sb) HK_HIP(ctx, ctx->kscratch.ensure(sb), "allocating sort scratch");
    StageTimer tm(ctx, HK_STAGE_KDIST);
    HK_HIP(ctx, launch_kdist(kappa, eb, n_points, bins->points_per_bin, gv, k_out, sorted_out,
                             ctx->kscratch.p, ctx->lds_bytes, ctx->lds_max, 1, ctx->stream),
           "kdist");
    tm.stop();
    return HK_OK;
}

static_assert((size_t)HK_KDIST_NOALLOC_SCRATCH_BYTES == kNoAllocScratchBytes, "no-allocation scratch size");

int hk_kdist_noalloc(hk_ctx* ctx, const void* kappa, int precision, int64_t n_points, const hk_bins* bins,
                     double* k_out, void* sorted_out)
{
    GValues gv;
    if (int rc = check_bins(ctx, bins, &gv)) return rc;
    if (precision != HK_F64 && precision != HK_F32_KAHAN)
        return fail(ctx, HK_EINVAL, "unknown precision %d", precision);
    if (n_points < 0 || n_points > HK_MAX_POINTS) return fail(ctx, HK_EINVAL, "n_points out of range");
    if (n_points > 0 && (!kappa || !k_out)) return fail(ctx, HK_EINVAL, "kappa and k_out must not be NULL");
    if (int rc = check_ctx(ctx)) return rc;
    const int eb = precision == HK_F64 ? 8 : 4;
    const size_t sb = kdist_scratch_bytes(eb, n_points, bins->points_per_bin, ctx->lds_bytes, ctx->lds_max);
    if (sb > kNoAllocScratchBytes)
        return fail(ctx, HK_EINVAL,
                    "hk_kdist_noalloc: bins of %lld points above one LDS sort need %zu bytes of scratch, more than "
                    "its fixed %zu (n_points * key bytes * 2)",
                    (long long)bins->points_per_bin, sb, kNoAllocScratchBytes);
    if (!ctx->noalloc_scratch) return fail(ctx, HK_EDEVICE, "no fixed sort scratch on this device");
    HK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    HK_HIP(ctx, launch_kdist(kappa, eb, n_points, bins->points_per_bin, gv, k_out, sorted_out, ctx->noalloc_scratch,
                             ctx->lds_bytes, ctx->lds_max, 1, ctx->stream),
           "kdist");
    return HK_OK;
}

int hk_tables(hk_ctx* ctx, const hk_state* states, int32_t n_states, const hk_grid* grid, const hk_bins* bins,
              int precision, double* k_out)
{
    if (n_states < 0) return fail(ctx, HK_EINVAL, "n_states must be >= 0 (got %d)", n_states);
    if (n_states > 0 && !states) return fail(ctx, HK_EINVAL, "states is NULL");
    for (int32_t i = 0; i < n_states; ++i) {
        if (check_state(ctx, &states[i])) {
            const std::string m = hk_last_error(ctx);
            return fail(ctx, HK_EINVAL, "states[%d]: %s", i, m.c_str());
        }
    }
    if (int rc = check_grid(ctx, grid)) return rc;
    GValues gv;
    if (int rc = check_bins(ctx, bins, &gv)) return rc;
    if (precision == HK_F32_SURROGATE)
        return fail(ctx, HK_EUNSUPPORTED, "hk_tables supports HK_F64 and HK_F32_KAHAN");
    if (precision != HK_F64 && precision != HK_F32_KAHAN)
        return fail(ctx, HK_EINVAL, "unknown precision %d", precision);
    if (precision == HK_F32_KAHAN && !(grid->cutoff_lorentz > 0.0) && !(grid->cutoff / grid->dnu < 8388608.0))
        return fail(ctx, HK_EINVAL, "HK_F32_KAHAN needs cutoff/dnu < 2^23 (got %g)", grid->cutoff / grid->dnu);
    const int32_t np = (int32_t)grid->n_points;
    const int64_t n_bins = ((int64_t)np + bins->points_per_bin - 1) / bins->points_per_bin;
    if (n_states > 0 && np > 0 && !k_out) return fail(ctx, HK_EINVAL, "k_out is NULL");
    if (int rc = check_ctx(ctx)) return rc;
    if (!ctx->lines_loaded) return fail(ctx, HK_ENOTREADY, "no line list loaded (call hk_load_lines first)");
    if (precision == HK_F32_KAHAN)
        for (int32_t i = 0; i < n_states; ++i)
            if (!(max_cutoff(ctx, &states[i], grid) / grid->dnu < 8388608.0))
                return fail(ctx, HK_EINVAL, "states[%d]: binary32 profiles need (largest cutoff)/dnu < 2^23", i);
    HK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    ctx->last_tables_states = 0;
    ctx->last_stream_chunks = 0;
    if (n_states == 0 || np == 0) return HK_OK;

    const int64_t n = ctx->n_lines;
    const bool f64 = precision == HK_F64;
    const LinesDev L = lines_dev(ctx);
    const int32_t tpc = f64 ? core_f64_tile_points() : core_f32_tile_points();
    const int64_t n_tiles_c = ((int64_t)np + tpc - 1) / tpc;
    const int64_t n_tiles_max = ((int64_t)np + opacity_f64_tile_points(2) - 1) / opacity_f64_tile_points(2);
    const int64_t n_tiles_max32 = ((int64_t)np + opacity_f32_tile_points(2) - 1) / opacity_f32_tile_points(2);
    const int64_t ranges_per_state = 2 * std::max(n_tiles_max, n_tiles_max32);

    // states per launch: the option, or as many as the memory budget holds
    const int64_t rec_bytes = f64 ? (int64_t)(sizeof(WingRec) + sizeof(WingIdx) + sizeof(CoreRec))
                                  : (int64_t)(sizeof(WingIdx) + sizeof(WingRec32) + sizeof(CoreRec32));
    // records, tile ranges, the opacity grid and the series grid (binary32:
    // sums, compensations and series in binary32)
    const int64_t per_state = n * rec_bytes + (ranges_per_state + 2 * n_tiles_c) * 8 + (int64_t)np * (f64 ? 16 : 20);
    int64_t B = ctx->tables_batch > 0 ? ctx->tables_batch : std::max<int64_t>(1, ctx->tables_mem / per_state);
    B = std::min<int64_t>(B, n_states);
    const int64_t n_batches = (n_states + B - 1) / B;
    B = (n_states + n_batches - 1) / n_batches;

    const size_t nb = (size_t)std::max<int64_t>(n, 1) * (size_t)B;
    HK_HIP(ctx, ctx->tb_idx.ensure(nb * sizeof(WingIdx)), "allocating batch records");
    if (f64) {
        HK_HIP(ctx, ctx->tb_wing.ensure(nb * sizeof(WingRec)), "allocating batch records");
        HK_HIP(ctx, ctx->tb_core.ensure(nb * sizeof(CoreRec)), "allocating batch records");
    } else {
        HK_HIP(ctx, ctx->tb_w32.ensure(nb * sizeof(WingRec32)), "allocating batch records");
        HK_HIP(ctx, ctx->tb_c32.ensure(nb * sizeof(CoreRec32)), "allocating batch records");
        HK_HIP(ctx, ctx->tb_comp.ensure((size_t)B * np * sizeof(float)), "allocating batch sums");
        HK_HIP(ctx, ctx->tb_scale.ensure((size_t)B * sizeof(int32_t)), "allocating batch scales");
        HK_HIP(ctx, ctx->tb_kappa.ensure((size_t)B * np * sizeof(double)), "allocating the opacities");
        HK_HIP(ctx, ctx->ln.f32partial.ensure((size_t)256 * B * sizeof(double)), "allocating the scale");
    }
    // per-state constants and reaches of a batch, on the device
    HK_HIP(ctx, ctx->tb_prep.ensure((size_t)B * (sizeof(PrepParams) + 2 * sizeof(double))), "allocating batch constants");
    HK_HIP(ctx, ctx->tb_out.ensure((size_t)B * np * (f64 ? sizeof(double) : sizeof(float))),
           "allocating batch opacities");
    HK_HIP(ctx, ctx->tb_series.ensure((size_t)B * np * (f64 ? sizeof(double) : sizeof(float))),
           "allocating batch series grids");
    HK_HIP(ctx, ctx->tb_ranges.ensure((size_t)B * ranges_per_state * sizeof(int64_t)), "allocating tile ranges");
    HK_HIP(ctx, ctx->tb_ranges_c.ensure((size_t)B * 2 * n_tiles_c * sizeof(int64_t)), "allocating tile ranges");
    HK_HIP(ctx, ctx->tb_counts.ensure((size_t)n_states * kCountBlocks * 3 * sizeof(int64_t)),
           "allocating counters");
    const size_t sb = kdist_scratch_bytes(8, np, bins->points_per_bin, ctx->lds_bytes, ctx->lds_max);
    if (sb) HK_HIP(ctx, ctx->kscratch.ensure(sb), "allocating sort scratch");
    // bins of one LDS radix sort: every state of a batch in one sort launch
    const bool sort_batched = bins->points_per_bin <= kdist_radix_max_keys(8, ctx->lds_max);

    WingIdx* tidx = static_cast<WingIdx*>(ctx->tb_idx.p);
    int64_t* rc_all = static_cast<int64_t*>(ctx->tb_ranges_c.p);
    int64_t* counts = static_cast<int64_t*>(ctx->tb_counts.p);

    // tile shape: cached, or timed on the first batch
    const int64_t cut_steps = grid->cutoff_lorentz > 0.0 ? -(int64_t)std::llround(grid->cutoff_lorentz * 1e3)
                                                         : (int64_t)std::llround(grid->cutoff / grid->dnu);
    int ppl = f64 ? ctx->f64_points_per_lane : ctx->f32_points_per_lane;
    bool tune = false;
    if (ctx->tables_autotune) {
        tune = true;
        for (const auto& t : ctx->tuned)
            if (t.precision == precision && t.n_lines == n && t.n_points == np && t.cut_steps == cut_steps) {
                ppl = t.ppl;
                tune = false;
            }
    }

    for (int64_t b0 = 0; b0 < n_states; b0 += B) {
        const int32_t nbat = (int32_t)std::min<int64_t>(B, n_states - b0);
        std::vector<double> reach_c((size_t)nbat), reach((size_t)nbat);
        std::vector<PrepParams> pps((size_t)nbat);
        for (int32_t s = 0; s < nbat; ++s) {
            pps[(size_t)s] = prep_params(ctx, &states[b0 + s], grid);
            reach_c[(size_t)s] = core_reach(ctx, &states[b0 + s], grid, pps[(size_t)s]);
            reach[(size_t)s] = wing_reach(ctx, &states[b0 + s], grid);
        }
        PrepParams* d_pps = static_cast<PrepParams*>(ctx->tb_prep.p);
        double* d_reach_c = reinterpret_cast<double*>(d_pps + B);
        double* d_reach = d_reach_c + B;
        {
            // the host arrays live until the batch's plans are read back
            // (a synchronisation), after these copies have run
            HK_HIP(ctx, hipMemcpyAsync(d_pps, pps.data(), pps.size() * sizeof(PrepParams), hipMemcpyHostToDevice,
                                       ctx->stream),
                   "copying batch constants");
            HK_HIP(ctx, hipMemcpyAsync(d_reach_c, reach_c.data(), reach_c.size() * sizeof(double),
                                       hipMemcpyHostToDevice, ctx->stream),
                   "copying batch constants");
            HK_HIP(ctx, hipMemcpyAsync(d_reach, reach.data(), reach.size() * sizeof(double), hipMemcpyHostToDevice,
                                       ctx->stream),
                   "copying batch constants");
        }
        {
            // every state of the batch in one launch per step
            StageTimer tm(ctx, HK_STAGE_LINE_PREP);
            if (f64) {
                HK_HIP(ctx, launch_line_prep_f64_batch(L, d_pps, nbat, static_cast<WingRec*>(ctx->tb_wing.p), tidx,
                                                       static_cast<CoreRec*>(ctx->tb_core.p), ctx->stream),
                       "line_prep_f64");
            } else {
                // the binary32 records straight from the line list: the
                // states' scales from a pass over the peaks, then the records
                int32_t* scale = static_cast<int32_t*>(ctx->tb_scale.p);
                HK_HIP(ctx, launch_f32_scale_lines(L, d_pps, static_cast<double*>(ctx->ln.f32partial.p), 256, scale,
                                                   ctx->stream, nbat),
                       "f32_scale");
                HK_HIP(ctx, launch_line_prep_f32_direct(L, d_pps, nbat, grid->nu_min, grid->dnu, scale, tidx,
                                                        static_cast<WingRec32*>(ctx->tb_w32.p),
                                                        static_cast<CoreRec32*>(ctx->tb_c32.p), ctx->stream),
                       "line_prep_f32");
            }
            HK_HIP(ctx, launch_eval_counts(tidx, n, counts + b0 * kCountBlocks * 3, kCountBlocks, ctx->stream, nbat),
                   "eval_counts");
            HK_HIP(ctx, launch_tile_ranges(L.nu, n, n_tiles_c, tpc, grid->nu_min, grid->dnu, np, 0.0, rc_all,
                                           ctx->stream, d_reach_c, nbat),
                   "tile_ranges");
            tm.stop();
        }
        if (tune) {
            const int32_t n_try = std::min<int32_t>(nbat, 4);
            if (int rc = autotune_wing(ctx, precision, &states[b0], n_try, grid, &ppl)) return rc;
            ctx->tuned.push_back({precision, n, np, cut_steps, ppl});
            tune = false;
        }
        const int32_t tp = f64 ? opacity_f64_tile_points(ppl) : opacity_f32_tile_points(ppl);
        const int64_t n_tiles = ((int64_t)np + tp - 1) / tp;
        int64_t* rw = static_cast<int64_t*>(ctx->tb_ranges.p);
        WorkPlan wwp, cwp;
        {
            StageTimer tm(ctx, HK_STAGE_LINE_PREP);
            HK_HIP(ctx, launch_tile_ranges(L.nu, n, n_tiles, tp, grid->nu_min, grid->dnu, np, 0.0, rw, ctx->stream,
                                           d_reach, nbat),
                   "tile_ranges");
            // the plans of the whole batch, read back to size the launches
            if (int rc = make_plan(ctx, ctx->ln.wplan, rw, n_tiles, nbat, reach.data(), tp, f64 ? 64 : 256, grid, true,
                                   &wwp, ctx->stream, d_reach))
                return rc;
            if (int rc = make_plan(ctx, ctx->ln.cplan, rc_all, n_tiles_c, nbat, reach_c.data(), tpc, 64, grid, true, &cwp,
                                   ctx->stream, d_reach_c))
                return rc;
            tm.stop();
        }
        // the series of the batch into its own grids: on the second stream
        // while the wing runs (tables_overlap = 1), or before the wing on the
        // caller's stream
        const bool overlap = ctx->tables_overlap != 0;
        hipStream_t cs = ctx->stream;
        if (overlap) {
            if (int rc = ensure_side(ctx)) return rc;
            cs = ctx->side;
            HK_HIP(ctx, hipEventRecord(ctx->ev_fork, ctx->stream), "hipEventRecord");
            HK_HIP(ctx, hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0), "hipStreamWaitEvent");
        }
        {
            StageTimer tm(ctx, HK_STAGE_CORE, cs);
            if (f64)
                HK_HIP(ctx, launch_core_f64(static_cast<WingRec*>(ctx->tb_wing.p), tidx,
                                            static_cast<CoreRec*>(ctx->tb_core.p), rc_all, n, n_tiles_c, nbat, cwp,
                                            grid->nu_min, grid->dnu, np, static_cast<double*>(ctx->tb_series.p),
                                            static_cast<double*>(ctx->ln.cplan.partial.p), cs),
                       "core_f64");
            else
                HK_HIP(ctx, launch_core_f32(tidx, static_cast<CoreRec32*>(ctx->tb_c32.p), rc_all, n, n_tiles_c, nbat,
                                            cwp, np, static_cast<float*>(ctx->tb_series.p),
                                            static_cast<float*>(ctx->ln.cplan.partial.p), nullptr, nullptr, nullptr,
                                            0, cs),
                       "core_f32");
            tm.stop();
        }
        if (overlap) HK_HIP(ctx, hipEventRecord(ctx->ev_join, ctx->side), "hipEventRecord");
        {
            StageTimer tm(ctx, HK_STAGE_OPACITY);
            if (f64)
                HK_HIP(ctx, launch_wing_f64(ppl, static_cast<WingRec*>(ctx->tb_wing.p), tidx, rw, n, n_tiles, nbat, wwp,
                                            grid->nu_min, grid->dnu, np, static_cast<double*>(ctx->tb_out.p),
                                            static_cast<double*>(ctx->ln.wplan.partial.p), 0, ctx->wing_edge_paths, ctx->stream),
                       "wing_f64");
            else
                HK_HIP(ctx, launch_wing_f32(ppl, static_cast<WingRec32*>(ctx->tb_w32.p), tidx, rw, n, n_tiles, nbat,
                                            wwp, np, static_cast<float*>(ctx->tb_out.p),
                                            static_cast<float*>(ctx->tb_comp.p),
                                            static_cast<float2*>(ctx->ln.wplan.partial.p), ctx->wing_edge_paths, ctx->stream),
                       "wing_f32");
            tm.stop();
        }
        if (overlap) HK_HIP(ctx, hipStreamWaitEvent(ctx->stream, ctx->ev_join, 0), "hipStreamWaitEvent");
        if (f64)
            HK_HIP(ctx, launch_add_f64(static_cast<double*>(ctx->tb_out.p), static_cast<double*>(ctx->tb_series.p),
                                       (int64_t)nbat * np, ctx->stream),
                   "add_f64");
        {
            StageTimer tm(ctx, HK_STAGE_KDIST);
            // the batch's binary64 opacities: the wing grids (binary64), or
            // the binary32 Kahan pairs and series finished into tb_kappa
            const double* kap = static_cast<double*>(ctx->tb_out.p);
            if (!f64) {
                HK_HIP(ctx, launch_f32_finish(static_cast<float*>(ctx->tb_out.p), static_cast<float*>(ctx->tb_comp.p),
                                              static_cast<float*>(ctx->tb_series.p),
                                              static_cast<int32_t*>(ctx->tb_scale.p), np,
                                              static_cast<double*>(ctx->tb_kappa.p), 0, ctx->stream, nbat),
                       "f32_finish");
                kap = static_cast<double*>(ctx->tb_kappa.p);
            }
            if (sort_batched) {
                HK_HIP(ctx, launch_kdist(kap, 8, np, bins->points_per_bin, gv, k_out + b0 * n_bins * gv.n, nullptr,
                                         ctx->kscratch.p, ctx->lds_bytes, ctx->lds_max, nbat, ctx->stream),
                       "kdist");
            } else {
                for (int32_t s = 0; s < nbat; ++s)
                    HK_HIP(ctx, launch_kdist(kap + (int64_t)s * np, 8, np, bins->points_per_bin, gv,
                                             k_out + (b0 + s) * n_bins * gv.n, nullptr, ctx->kscratch.p,
                                             ctx->lds_bytes, ctx->lds_max, 1, ctx->stream),
                           "kdist");
            }
            tm.stop();
        }
    }
    ctx->last_tables_states = n_states;
    ctx->tables_ppl_used = ppl;
    ctx->have_run = true;
    return HK_OK;
}

static int sg_ready(hk_ctx* ctx)
{
    if (!ctx->sg_loaded) return fail(ctx, HK_ENOTREADY, "no surrogate parameters (hk_surrogate_set_params)");
    return HK_OK;
}

static int check_samples(hk_ctx* ctx, const float* x, const float* y, int64_t n)
{
    if (n < 0 || n > HK_MAX_POINTS) return fail(ctx, HK_EINVAL, "sample count %lld out of range", (long long)n);
    if (n > 0 && (!x || !y)) return fail(ctx, HK_EINVAL, "x and y must not be NULL");
    return HK_OK;
}

int hk_surrogate_labels(hk_ctx* ctx, const float* x, const float* y, int64_t n, float* z)
{
    if (int rc = check_samples(ctx, x, y, n)) return rc;
    if (n > 0 && !z) return fail(ctx, HK_EINVAL, "z is NULL");
    if (int rc = check_ctx(ctx)) return rc;
    HK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    HK_HIP(ctx, launch_surrogate_labels(x, y, n, z, ctx->stream), "surrogate_labels");
    return HK_OK;
}

int hk_surrogate_set_params(hk_ctx* ctx, const float* theta)
{
    if (!theta) return fail(ctx, HK_EINVAL, "theta is NULL");
    for (int i = 0; i < HK_SURR_N_PARAMS; ++i)
        if (!std::isfinite(theta[i])) return fail(ctx, HK_EINVAL, "theta[%d] is not finite", i);
    if (int rc = check_ctx(ctx)) return rc;
    HK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    const size_t nb = (size_t)HK_SURR_N_PARAMS * sizeof(float);
    HK_HIP(ctx, ctx->sg_theta.ensure(nb), "allocating parameters");
    HK_HIP(ctx, ctx->sg_m.ensure(nb), "allocating parameters");
    HK_HIP(ctx, ctx->sg_v.ensure(nb), "allocating parameters");
    HK_HIP(ctx, ctx->sg_copy.ensure(surrogate_params_bytes()), "allocating parameters");
    HK_HIP(ctx, hipMemcpyAsync(ctx->sg_theta.p, theta, nb, hipMemcpyHostToDevice, ctx->stream), "copying parameters");
    HK_HIP(ctx, launch_zero(ctx->sg_m.p, nb, ctx->stream), "zero");
    HK_HIP(ctx, launch_zero(ctx->sg_v.p, nb, ctx->stream), "zero");
    HK_HIP(ctx, launch_surrogate_pack(static_cast<float*>(ctx->sg_theta.p), ctx->sg_copy.p, ctx->stream),
           "surrogate_pack");
    HK_HIP(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    ctx->sg_loaded = true;
    ctx->sg_certified = false;
    ctx->sg_step = 0;
    ctx->sg_cursor = 0;
    return HK_OK;
}

int hk_surrogate_get_params(hk_ctx* ctx, float* theta)
{
    if (!theta) return fail(ctx, HK_EINVAL, "theta is NULL");
    if (int rc = check_ctx(ctx)) return rc;
    if (int rc = sg_ready(ctx)) return rc;
    HK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    HK_HIP(ctx, hipMemcpyAsync(theta, ctx->sg_theta.p, (size_t)HK_SURR_N_PARAMS * sizeof(float),
                               hipMemcpyDeviceToHost, ctx->stream),
           "copying parameters");
    HK_HIP(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    return HK_OK;
}

static int sg_partials(hk_ctx* ctx, int32_t batch)
{
    const int64_t n_wg = (batch + 63) / 64;
    HK_HIP(ctx, ctx->sg_part.ensure((size_t)n_wg * HK_SURR_N_PARAMS * sizeof(float)), "allocating gradients");
    HK_HIP(ctx, ctx->sg_ploss.ensure((size_t)n_wg * sizeof(float)), "allocating gradients");
    return HK_OK;
}

int hk_surrogate_grad(hk_ctx* ctx, const float* x, const float* y, const float* z, int64_t n, double wscale,
                      float* grad, float* loss)
{
    if (!(wscale >= 0.0) || !std::isfinite(wscale)) return fail(ctx, HK_EINVAL, "wscale must be finite and >= 0");
    if (int rc = check_samples(ctx, x, y, n)) return rc;
    if (n < 1 || n > HK_SURR_MAX_BATCH)
        return fail(ctx, HK_EINVAL, "n must be in [1, %d] (got %lld)", HK_SURR_MAX_BATCH, (long long)n);
    if (!z || !grad) return fail(ctx, HK_EINVAL, "z and grad must not be NULL");
    if (int rc = check_ctx(ctx)) return rc;
    if (int rc = sg_ready(ctx)) return rc;
    HK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (int rc = sg_partials(ctx, (int32_t)n)) return rc;
    float* part = static_cast<float*>(ctx->sg_part.p);
    float* pl = static_cast<float*>(ctx->sg_ploss.p);
    HK_HIP(ctx, launch_surrogate_train_step(ctx->sg_copy.p, x, y, z, n, 0, (int32_t)n, (float)wscale, part, pl,
                                            ctx->stream),
           "surrogate_train_step");
    HK_HIP(ctx, launch_surrogate_reduce(part, (int32_t)n, grad, pl, loss, ctx->stream), "surrogate_reduce");
    return HK_OK;
}

int hk_surrogate_train(hk_ctx* ctx, const float* x, const float* y, const float* z, int64_t n,
                       const hk_train_cfg* cfg, float* loss_hist)
{
    if (int rc = check_samples(ctx, x, y, n)) return rc;
    if (n < 1 || !z) return fail(ctx, HK_EINVAL, "need n >= 1 samples with targets z");
    if (!cfg) return fail(ctx, HK_EINVAL, "cfg is NULL");
    if (cfg->batch < 1 || cfg->batch > HK_SURR_MAX_BATCH)
        return fail(ctx, HK_EINVAL, "batch must be in [1, %d]", HK_SURR_MAX_BATCH);
    if (cfg->steps < 0) return fail(ctx, HK_EINVAL, "steps must be >= 0");
    if (!(cfg->lr > 0.0) || !(cfg->beta1 >= 0.0 && cfg->beta1 < 1.0) || !(cfg->beta2 >= 0.0 && cfg->beta2 < 1.0) ||
        !(cfg->eps > 0.0) || !(cfg->wscale >= 0.0) || !std::isfinite(cfg->wscale))
        return fail(ctx, HK_EINVAL, "need lr > 0, 0 <= beta1, beta2 < 1, eps > 0, wscale >= 0");
    if (int rc = check_ctx(ctx)) return rc;
    if (int rc = sg_ready(ctx)) return rc;
    HK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (int rc = sg_partials(ctx, cfg->batch)) return rc;
    float* part = static_cast<float*>(ctx->sg_part.p);
    float* pl = static_cast<float*>(ctx->sg_ploss.p);
    for (int32_t s = 0; s < cfg->steps; ++s) {
        const int64_t t = ctx->sg_step + 1;
        const float c1 = (float)(1.0 / (1.0 - std::pow(cfg->beta1, (double)t)));
        const float c2 = (float)(1.0 / (1.0 - std::pow(cfg->beta2, (double)t)));
        HK_HIP(ctx, launch_surrogate_train_step(ctx->sg_copy.p, x, y, z, n, ctx->sg_cursor, cfg->batch,
                                                (float)cfg->wscale, part, pl, ctx->stream),
               "surrogate_train_step");
        HK_HIP(ctx, launch_surrogate_adam(static_cast<float*>(ctx->sg_theta.p), static_cast<float*>(ctx->sg_m.p),
                                          static_cast<float*>(ctx->sg_v.p), part, cfg->batch, (float)cfg->lr,
                                          (float)cfg->beta1, (float)cfg->beta2, (float)cfg->eps, c1, c2,
                                          ctx->sg_copy.p, pl, loss_hist ? loss_hist + s : nullptr, ctx->stream),
               "surrogate_adam");
        ctx->sg_step = t;
        ctx->sg_cursor = (ctx->sg_cursor + cfg->batch) % n;
    }
    ctx->sg_certified = false;
    return HK_OK;
}

int hk_surrogate_eval(hk_ctx* ctx, const float* x, const float* y, int64_t n, float* z, float* K)
{
    if (int rc = check_samples(ctx, x, y, n)) return rc;
    if (n > 0 && !z) return fail(ctx, HK_EINVAL, "z is NULL");
    if (int rc = check_ctx(ctx)) return rc;
    if (int rc = sg_ready(ctx)) return rc;
    HK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    HK_HIP(ctx, launch_surrogate_eval(ctx->sg_copy.p, x, y, n, z, K, ctx->stream), "surrogate_eval");
    return HK_OK;
}

int hk_surrogate_certify(hk_ctx* ctx, double budget, double* err, int32_t* n_certified)
{
    if (!(budget > 0.0) || !std::isfinite(budget)) return fail(ctx, HK_EINVAL, "budget must be finite and > 0");
    if (int rc = check_ctx(ctx)) return rc;
    if (int rc = sg_ready(ctx)) return rc;
    HK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    const int nc = surrogate_cells();
    HK_HIP(ctx, ctx->sg_err.ensure((size_t)nc * sizeof(double)), "allocating certification");
    HK_HIP(ctx, ctx->sg_mask.ensure((size_t)nc), "allocating certification");
    HK_HIP(ctx, launch_surrogate_certify(ctx->sg_copy.p, static_cast<double*>(ctx->sg_err.p), ctx->stream),
           "surrogate_certify");
    std::vector<double> e((size_t)nc);
    HK_HIP(ctx, hipMemcpyAsync(e.data(), ctx->sg_err.p, e.size() * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream),
           "copying certification");
    HK_HIP(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    std::vector<uint8_t> mask((size_t)nc);
    int32_t cnt = 0;
    for (int c = 0; c < nc; ++c) {
        mask[(size_t)c] = e[(size_t)c] <= budget ? 1 : 0;
        cnt += mask[(size_t)c];
    }
    HK_HIP(ctx, hipMemcpy(ctx->sg_mask.p, mask.data(), mask.size(), hipMemcpyHostToDevice), "copying the mask");
    if (err) std::memcpy(err, e.data(), e.size() * sizeof(double));
    if (n_certified) *n_certified = cnt;
    ctx->sg_certified = true;
    ctx->sg_budget = budget;
    return HK_OK;
}

namespace {
// The surrogate blob: a 32-byte header, the binary32 parameters and, when
// certified, the binary64 cell errors (the mask is err <= budget).
constexpr char kSurrMagic[8] = {'H', 'K', 'S', 'U', 'R', 'R', '0', '1'};
struct SurrHeader {
    char magic[8];
    int32_t n_params, n_cells, certified, reserved;
    double budget;
};
static_assert(sizeof(SurrHeader) == 32, "surrogate blob header");
size_t surr_blob_bytes(bool certified)
{
    return sizeof(SurrHeader) + (size_t)HK_SURR_N_PARAMS * sizeof(float) +
           (certified ? (size_t)HK_SURR_CELLS_X * HK_SURR_CELLS_Y * sizeof(double) : 0);
}
}  // namespace

int hk_surrogate_save(hk_ctx* ctx, void* blob, size_t capacity, size_t* size)
{
    if (int rc = check_ctx(ctx)) return rc;
    if (int rc = sg_ready(ctx)) return rc;
    if (!size) return fail(ctx, HK_EINVAL, "size is NULL");
    const size_t need = surr_blob_bytes(ctx->sg_certified);
    *size = need;
    if (!blob) return HK_OK;
    if (capacity < need) return fail(ctx, HK_EINVAL, "blob capacity %zu < %zu bytes", capacity, need);
    HK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    SurrHeader h{};
    std::memcpy(h.magic, kSurrMagic, sizeof kSurrMagic);
    h.n_params = HK_SURR_N_PARAMS;
    h.n_cells = HK_SURR_CELLS_X * HK_SURR_CELLS_Y;
    h.certified = ctx->sg_certified ? 1 : 0;
    h.budget = ctx->sg_certified ? ctx->sg_budget : 0.0;
    char* out = static_cast<char*>(blob);
    std::memcpy(out, &h, sizeof h);
    HK_HIP(ctx, hipMemcpyAsync(out + sizeof h, ctx->sg_theta.p, (size_t)HK_SURR_N_PARAMS * sizeof(float),
                               hipMemcpyDeviceToHost, ctx->stream),
           "copying parameters");
    if (ctx->sg_certified)
        HK_HIP(ctx, hipMemcpyAsync(out + sizeof h + (size_t)HK_SURR_N_PARAMS * sizeof(float), ctx->sg_err.p,
                                   (size_t)h.n_cells * sizeof(double), hipMemcpyDeviceToHost, ctx->stream),
               "copying certification");
    HK_HIP(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    return HK_OK;
}

int hk_surrogate_load(hk_ctx* ctx, const void* blob, size_t size)
{
    if (!blob) return fail(ctx, HK_EINVAL, "blob is NULL");
    if (size < sizeof(SurrHeader)) return fail(ctx, HK_EINVAL, "blob of %zu bytes has no header", size);
    SurrHeader h;
    std::memcpy(&h, blob, sizeof h);
    if (std::memcmp(h.magic, kSurrMagic, sizeof kSurrMagic) != 0)
        return fail(ctx, HK_EINVAL, "not a surrogate blob (magic)");
    if (h.n_params != HK_SURR_N_PARAMS || h.n_cells != HK_SURR_CELLS_X * HK_SURR_CELLS_Y ||
        (h.certified != 0 && h.certified != 1))
        return fail(ctx, HK_EINVAL, "surrogate blob layout (%d parameters, %d cells) differs from this library's",
                    h.n_params, h.n_cells);
    if (size != surr_blob_bytes(h.certified != 0))
        return fail(ctx, HK_EINVAL, "blob of %zu bytes, expected %zu", size, surr_blob_bytes(h.certified != 0));
    if (h.certified && !(h.budget > 0.0 && std::isfinite(h.budget)))
        return fail(ctx, HK_EINVAL, "blob's certification budget is not finite and > 0");
    const char* in = static_cast<const char*>(blob);
    std::vector<float> theta((size_t)HK_SURR_N_PARAMS);
    std::memcpy(theta.data(), in + sizeof h, theta.size() * sizeof(float));
    std::vector<double> err;
    if (h.certified) {
        err.resize((size_t)h.n_cells);
        std::memcpy(err.data(), in + sizeof h + theta.size() * sizeof(float), err.size() * sizeof(double));
        for (double e : err)
            if (std::isnan(e) || e < 0.0) return fail(ctx, HK_EINVAL, "blob holds an invalid cell error");
    }
    if (int rc = hk_surrogate_set_params(ctx, theta.data())) return rc;
    if (!h.certified) return HK_OK;
    const int nc = h.n_cells;
    HK_HIP(ctx, ctx->sg_err.ensure((size_t)nc * sizeof(double)), "allocating certification");
    HK_HIP(ctx, ctx->sg_mask.ensure((size_t)nc), "allocating certification");
    std::vector<uint8_t> mask((size_t)nc);
    for (int c = 0; c < nc; ++c) mask[(size_t)c] = err[(size_t)c] <= h.budget ? 1 : 0;
    HK_HIP(ctx, hipMemcpy(ctx->sg_err.p, err.data(), err.size() * sizeof(double), hipMemcpyHostToDevice),
           "copying certification");
    HK_HIP(ctx, hipMemcpy(ctx->sg_mask.p, mask.data(), mask.size(), hipMemcpyHostToDevice), "copying the mask");
    ctx->sg_certified = true;
    ctx->sg_budget = h.budget;
    return HK_OK;
}

static_assert(HK_MAX_COEF == kMaxCoef, "coefficient bound");
static_assert(HK_RULE_STEP == kRuleStep && HK_RULE_LINEAR == kRuleLinear, "k(g) rules");
static_assert(HK_TRANSMISSION_NODES <= kMaxQuad, "quadrature bound");

int hk_resample(hk_ctx* ctx, const void* sorted, int precision, int64_t n_points, int64_t points_per_bin,
                int32_t n_coef, double* coef_out)
{
    if (precision != HK_F64 && precision != HK_F32_KAHAN)
        return fail(ctx, HK_EINVAL, "unknown precision %d", precision);
    if (n_points < 0 || n_points > HK_MAX_POINTS) return fail(ctx, HK_EINVAL, "n_points out of range");
    if (points_per_bin < 1) return fail(ctx, HK_EINVAL, "points_per_bin must be >= 1");
    if (n_coef < 1 || n_coef > HK_MAX_COEF) return fail(ctx, HK_EINVAL, "n_coef must be in [1, %d]", HK_MAX_COEF);
    const int64_t ml = n_points % points_per_bin;
    if ((n_points >= points_per_bin && points_per_bin < n_coef) || (ml > 0 && ml < n_coef))
        return fail(ctx, HK_EINVAL, "every bin needs at least n_coef = %d points", n_coef);
    if (n_points > 0 && (!sorted || !coef_out)) return fail(ctx, HK_EINVAL, "sorted and coef_out must not be NULL");
    if (int rc = check_ctx(ctx)) return rc;
    if (n_points == 0) return HK_OK;
    HK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    const int64_t m = std::min(points_per_bin, n_points);
    if (ctx->rs_m != m || ctx->rs_nc != n_coef) {
        HK_HIP(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        if (int rc = upload_qr(ctx, m, n_coef, ctx->rs_Q, ctx->rs_R)) return rc;
        ctx->rs_m = m;
        ctx->rs_ml = -1;
        ctx->rs_nc = n_coef;
    }
    const bool ragged = n_points > points_per_bin && ml > 0;
    if (ragged && ctx->rs_ml != ml) {
        HK_HIP(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        if (int rc = upload_qr(ctx, ml, n_coef, ctx->rs_Ql, ctx->rs_Rl)) return rc;
        ctx->rs_ml = ml;
    }
    const double* Ql = ragged ? static_cast<const double*>(ctx->rs_Ql.p) : static_cast<const double*>(ctx->rs_Q.p);
    const double* Rl = ragged ? static_cast<const double*>(ctx->rs_Rl.p) : static_cast<const double*>(ctx->rs_R.p);
    HK_HIP(ctx, launch_resample(sorted, precision == HK_F64 ? 8 : 4, n_points, points_per_bin, n_coef,
                                static_cast<const double*>(ctx->rs_Q.p), static_cast<const double*>(ctx->rs_R.p), Ql,
                                Rl, coef_out, ctx->stream),
           "resample");
    return HK_OK;
}

int hk_transmission(hk_ctx* ctx, const double* coef, int64_t n_bins, int32_t n_coef, const double* m_col,
                    int32_t n_m, double* T_out)
{
    if (n_bins < 0 || n_bins > HK_MAX_POINTS) return fail(ctx, HK_EINVAL, "n_bins out of range");
    if (n_coef < 1 || n_coef > HK_MAX_COEF) return fail(ctx, HK_EINVAL, "n_coef must be in [1, %d]", HK_MAX_COEF);
    if (n_m < 0 || n_m > HK_MAX_COLUMNS) return fail(ctx, HK_EINVAL, "n_m must be in [0, %d]", HK_MAX_COLUMNS);
    if (n_bins > 0 && n_m > 0 && (!coef || !m_col || !T_out))
        return fail(ctx, HK_EINVAL, "coef, m and T_out must not be NULL");
    if (int rc = check_ctx(ctx)) return rc;
    if (n_bins == 0 || n_m == 0) return HK_OK;
    HK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    if (!ctx->rs_quad_ready) {
        std::vector<double> q(2 * HK_TRANSMISSION_NODES);
        if (int rc = hk_gauss_legendre(HK_TRANSMISSION_NODES, q.data(), q.data() + HK_TRANSMISSION_NODES)) return rc;
        HK_HIP(ctx, ctx->rs_quad.ensure(q.size() * sizeof(double)), "allocating the quadrature");
        HK_HIP(ctx, hipMemcpy(ctx->rs_quad.p, q.data(), q.size() * sizeof(double), hipMemcpyHostToDevice),
               "copying the quadrature");
        ctx->rs_quad_ready = true;
    }
    const double* yq = static_cast<const double*>(ctx->rs_quad.p);
    HK_HIP(ctx, launch_transmission_fit(coef, n_bins, n_coef, yq, yq + HK_TRANSMISSION_NODES, HK_TRANSMISSION_NODES,
                                        m_col, n_m, T_out, ctx->stream),
           "transmission");
    return HK_OK;
}

int hk_transmission_direct(hk_ctx* ctx, const void* sorted, int precision, int64_t n_points, int64_t points_per_bin,
                           const double* m_col, int32_t n_m, double* T_out)
{
    if (precision != HK_F64 && precision != HK_F32_KAHAN)
        return fail(ctx, HK_EINVAL, "unknown precision %d", precision);
    if (n_points < 0 || n_points > HK_MAX_POINTS) return fail(ctx, HK_EINVAL, "n_points out of range");
    if (points_per_bin < 1) return fail(ctx, HK_EINVAL, "points_per_bin must be >= 1");
    if (n_m < 0 || n_m > HK_MAX_COLUMNS) return fail(ctx, HK_EINVAL, "n_m must be in [0, %d]", HK_MAX_COLUMNS);
    if (n_points > 0 && n_m > 0 && (!sorted || !m_col || !T_out))
        return fail(ctx, HK_EINVAL, "sorted, m and T_out must not be NULL");
    if (int rc = check_ctx(ctx)) return rc;
    if (n_points == 0 || n_m == 0) return HK_OK;
    HK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    HK_HIP(ctx, launch_transmission_direct(sorted, precision == HK_F64 ? 8 : 4, n_points, points_per_bin, m_col, n_m,
                                           T_out, ctx->stream),
           "transmission_direct");
    return HK_OK;
}

int hk_stats(hk_ctx* ctx, hk_run_stats* out)
{
    if (int rc = check_ctx(ctx)) return rc;
    if (!out) return fail(ctx, HK_EINVAL, "out is NULL");
    std::memset(out, 0, sizeof *out);
    const bool streamed = ctx->last_stream_chunks > 0;
    out->n_lines = streamed ? ctx->stream_lines : ctx->n_lines;
    if (!ctx->have_run) return fail(ctx, HK_ENOTREADY, "no hk_opacity call yet");
    HK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    // hk_opacity: count from the state's records now; hk_tables and
    // hk_opacity_stream: the per-state or per-chunk counters they left
    const bool tables = ctx->last_tables_states > 0;
    const int64_t nblk = tables     ? (int64_t)kCountBlocks * ctx->last_tables_states
                         : streamed ? (int64_t)kCountBlocks * ctx->last_stream_chunks
                                    : kCountBlocks;
    HK_HIP(ctx, ctx->partial.ensure((size_t)kCountBlocks * 3 * sizeof(int64_t)), "allocating counters");
    if (out->n_lines > 0) {
        if (!tables && !streamed)
            HK_HIP(ctx, launch_eval_counts(static_cast<WingIdx*>(ctx->ln.widx.p), ctx->n_lines,
                                           static_cast<int64_t*>(ctx->partial.p), kCountBlocks, ctx->stream),
                   "eval_counts");
        std::vector<int64_t> h((size_t)nblk * 3);
        const void* src = tables ? ctx->tb_counts.p : streamed ? ctx->st_counts.p : ctx->partial.p;
        HK_HIP(ctx, hipMemcpyAsync(h.data(), src, h.size() * sizeof(int64_t),
                                   hipMemcpyDeviceToHost, ctx->stream),
               "copying counters");
        HK_HIP(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        int64_t e = 0, c = 0, g = 0;
        for (int64_t b = 0; b < nblk; ++b) {
            e += h[3 * b];
            c += h[3 * b + 1];
            g += h[3 * b + 2];
        }
        out->evals = e;
        out->evals_core = c;
        out->evals_gh3 = g - c;
        out->evals_gh1 = e - g;
        if (!tables && ctx->sg_used_total.p) {  // 0 after hk_tables, which has no surrogate
            int64_t u = 0;
            HK_HIP(ctx, hipMemcpyAsync(&u, ctx->sg_used_total.p, sizeof u, hipMemcpyDeviceToHost, ctx->stream),
                   "copying counters");
            HK_HIP(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
            out->evals_surrogate = u;
        }
    }
    return HK_OK;
}

int hk_set_option(hk_ctx* ctx, const char* name, int64_t value)
{
    if (!name) return fail(ctx, HK_EINVAL, "option name is NULL");
    const bool f64 = std::strcmp(name, "f64_points_per_lane") == 0;
    const bool f32 = std::strcmp(name, "f32_points_per_lane") == 0;
    if (f64 || f32) {
        // binary64 points form groups of four within a lane
        if (f64 && value != 4 && value != 8)
            return fail(ctx, HK_EINVAL, "%s must be 4 or 8 (got %lld)", name, (long long)value);
        if (value != 2 && value != 4 && value != 8)
            return fail(ctx, HK_EINVAL, "%s must be 2, 4 or 8 (got %lld)", name, (long long)value);
        if (int rc = check_ctx(ctx)) return rc;
        (f64 ? ctx->f64_points_per_lane : ctx->f32_points_per_lane) = (int)value;
        return HK_OK;
    }
    if (std::strcmp(name, "tables_batch") == 0) {
        if (value < 0 || value > INT32_MAX) return fail(ctx, HK_EINVAL, "tables_batch must be >= 0");
        if (int rc = check_ctx(ctx)) return rc;
        ctx->tables_batch = value;
        return HK_OK;
    }
    if (std::strcmp(name, "tables_mem_mib") == 0) {
        if (value < 1 || value > ((int64_t)1 << 30)) return fail(ctx, HK_EINVAL, "tables_mem_mib must be >= 1");
        if (int rc = check_ctx(ctx)) return rc;
        ctx->tables_mem = value << 20;
        return HK_OK;
    }
    if (std::strcmp(name, "tables_overlap") == 0) {
        if (value != 0 && value != 1) return fail(ctx, HK_EINVAL, "tables_overlap must be 0 or 1");
        ctx->tables_overlap = (int)value;
        return HK_OK;
    }
    if (std::strcmp(name, "wing_edge_paths") == 0) {
        if (value != 0 && value != 1) return fail(ctx, HK_EINVAL, "wing_edge_paths must be 0 or 1");
        if (int rc = check_ctx(ctx)) return rc;
        ctx->wing_edge_paths = (int)value;
        return HK_OK;
    }
    if (std::strcmp(name, "tables_autotune") == 0) {
        if (value != 0 && value != 1) return fail(ctx, HK_EINVAL, "tables_autotune must be 0 or 1");
        if (int rc = check_ctx(ctx)) return rc;
        ctx->tables_autotune = (int)value;
        if (!value) ctx->tuned.clear();
        return HK_OK;
    }
    return fail(ctx, HK_EINVAL, "unknown option '%s'", name);
}

int hk_get_option(hk_ctx* ctx, const char* name, int64_t* value)
{
    if (!name || !value) return fail(ctx, HK_EINVAL, "name and value must not be NULL");
    if (int rc = check_ctx(ctx)) return rc;
    if (std::strcmp(name, "f64_points_per_lane") == 0) *value = ctx->f64_points_per_lane;
    else if (std::strcmp(name, "f32_points_per_lane") == 0) *value = ctx->f32_points_per_lane;
    else if (std::strcmp(name, "tables_batch") == 0) *value = ctx->tables_batch;
    else if (std::strcmp(name, "tables_mem_mib") == 0) *value = ctx->tables_mem >> 20;
    else if (std::strcmp(name, "tables_autotune") == 0) *value = ctx->tables_autotune;
    else if (std::strcmp(name, "wing_edge_paths") == 0) *value = ctx->wing_edge_paths;
    else if (std::strcmp(name, "tables_overlap") == 0) *value = ctx->tables_overlap;
    else if (std::strcmp(name, "tables_points_per_lane") == 0) *value = ctx->tables_ppl_used;
    else if (std::strcmp(name, "wing_items") == 0 || std::strcmp(name, "wing_segment_lines") == 0) {
        // the last wing stage's plan (for its first state), read back
        *value = 0;
        if (!ctx->ln.wplan.total.p) return HK_OK;
        HK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
        const bool items = name[5] == 'i';
        HK_HIP(ctx, hipMemcpyAsync(value, items ? ctx->ln.wplan.total.p : ctx->ln.wplan.seg.p, sizeof *value,
                                   hipMemcpyDeviceToHost, ctx->stream),
               "reading the work plan");
        HK_HIP(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
        if (!items && *value == kNoSplit) *value = 0;
    } else
        return fail(ctx, HK_EINVAL, "unknown option '%s'", name);
    return HK_OK;
}

int hk_set_timing(hk_ctx* ctx, int enable)
{
    if (int rc = check_ctx(ctx)) return rc;
    HK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    HK_HIP(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    for (auto& p : ctx->pending) {
        ctx->free_events.push_back(p.second.first);
        ctx->free_events.push_back(p.second.second);
    }
    ctx->pending.clear();
    ctx->tsum = hk_timing{};
    ctx->timing = enable != 0;
    return HK_OK;
}

int hk_get_timing(hk_ctx* ctx, hk_timing* out)
{
    if (int rc = check_ctx(ctx)) return rc;
    if (!out) return fail(ctx, HK_EINVAL, "out is NULL");
    HK_HIP(ctx, hipSetDevice(ctx->device), "hipSetDevice");
    HK_HIP(ctx, hipStreamSynchronize(ctx->stream), "hipStreamSynchronize");
    for (auto& p : ctx->pending) {
        float ms = 0.0f;
        HK_HIP(ctx, hipEventElapsedTime(&ms, p.second.first, p.second.second), "hipEventElapsedTime");
        ctx->tsum.ms[p.first] += ms;
        ctx->tsum.calls[p.first] += 1;
        ctx->free_events.push_back(p.second.first);
        ctx->free_events.push_back(p.second.second);
    }
    ctx->pending.clear();
    *out = ctx->tsum;
    return HK_OK;
}

// Gauss-Legendre rule on (0, 1).  Each node of P_n on [-1, 1] is refined by
// Newton's method from the Chebyshev-like start cos(pi (k - 1/4)/(n + 1/2)),
// with P_n and its derivative from Bonnet's recurrence; weight
// 2 / ((1 - x^2) P_n'(x)^2).  Mapped to (0, 1): g = (1 + x)/2, w/2.
int hk_gauss_legendre(int32_t n, double* g, double* w)
{
    if (n < 1 || n > 256) return fail(nullptr, HK_EINVAL, "n must be in [1, 256]");
    if (!g || !w) return fail(nullptr, HK_EINVAL, "g and w must not be NULL");
    for (int k = 1; k <= n; ++k) {
        double x = std::cos(kPi * (k - 0.25) / (n + 0.5));
        double pn = 0.0, dpn = 1.0;
        for (int it = 0; it < 50; ++it) {
            double pkm1 = 1.0, pk = x;  // P_0, P_1
            for (int m = 2; m <= n; ++m) {
                double pkp1 = ((2 * m - 1) * x * pk - (m - 1) * pkm1) / m;
                pkm1 = pk;
                pk = pkp1;
            }
            pn = n == 1 ? x : pk;
            double pnm1 = n == 1 ? 1.0 : pkm1;
            dpn = n * (pnm1 - x * pn) / (1.0 - x * x);
            double dx = pn / dpn;
            x -= dx;
            if (std::fabs(dx) <= 1e-16 * std::max(1.0, std::fabs(x))) break;
        }
        {
            double pkm1 = 1.0, pk = x;
            for (int m = 2; m <= n; ++m) {
                double pkp1 = ((2 * m - 1) * x * pk - (m - 1) * pkm1) / m;
                pkm1 = pk;
                pk = pkp1;
            }
            pn = n == 1 ? x : pk;
            double pnm1 = n == 1 ? 1.0 : pkm1;
            dpn = n * (pnm1 - x * pn) / (1.0 - x * x);
        }
        // x is the k-th largest root: store ascending
        g[n - k] = 0.5 * (1.0 + x);
        w[n - k] = 1.0 / ((1.0 - x * x) * dpn * dpn);
    }
    return HK_OK;
}

}  // extern "C"
