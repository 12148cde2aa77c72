// extern "C" entry points of liblw.so: argument validation, workspace checks, dispatch.
#include "lw_internal.h"

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <vector>

namespace lw {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

lw_status fail(lw_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

lw_status check_launch(const char *what)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(LW_E_HIP, "%s: %s", what, hipGetErrorString(e));
    g_err[0] = 0;
    return LW_OK;
}

// ---- kernel timing (lw_timing_enable / lw_timing_read)
namespace {
struct TimedLaunch {
    int which;
    hipEvent_t a, b;
};
std::mutex g_tm;
bool g_timing = false;
std::vector<TimedLaunch> g_timed;  // recorded, not yet read
std::vector<hipEvent_t> g_pool;    // idle events

hipEvent_t pool_event()
{
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}
}  // namespace

hipEvent_t timing_begin(int which, hipStream_t s)
{
    (void)which;
    std::lock_guard<std::mutex> lk(g_tm);
    if (!g_timing) return nullptr;
    hipEvent_t e = pool_event();
    if (e && hipEventRecord(e, s) != hipSuccess) {
        g_pool.push_back(e);
        return nullptr;
    }
    return e;
}

void timing_end(int which, hipEvent_t start, hipStream_t s)
{
    if (!start) return;
    std::lock_guard<std::mutex> lk(g_tm);
    hipEvent_t e = pool_event();
    if (!g_timing || !e || hipEventRecord(e, s) != hipSuccess) {
        g_pool.push_back(start);
        if (e) g_pool.push_back(e);
        return;
    }
    g_timed.push_back({which, start, e});
}

namespace {

constexpr int64_t kMaxSamples = int64_t(1) << 31;

bool finite_pos(double v) { return v > 0.0 && v < 1e300; }

lw_status check_traj_samples(const lw_traj_t *t, const char *fn)
{
    if (!t) return fail(LW_E_ARG, "%s: traj is NULL", fn);
    if (t->kind != LW_TRAJ_SAMPLES)
        return fail(LW_E_UNSUPPORTED, "%s: traj->kind must be LW_TRAJ_SAMPLES", fn);
    if (t->span != 0) return fail(LW_E_ARG, "%s: traj->span must be 0 for stored samples", fn);
    if (t->n_particles < 0 || t->n_samples < 1 || t->n_samples >= kMaxSamples)
        return fail(LW_E_SHAPE, "%s: need n_particles >= 0 and 1 <= n_samples < 2^31 (got %lld, %lld)", fn,
                    (long long)t->n_particles, (long long)t->n_samples);
    if (!finite_pos(t->dt) || !(t->t_start > -1e300 && t->t_start < 1e300))
        return fail(LW_E_ARG, "%s: dt must be positive and finite, t_start finite", fn);
    if (t->n_particles > 0) {
        if (!t->r || !t->beta || !t->beta_dot) return fail(LW_E_ARG, "%s: r, beta, beta_dot must be non-NULL", fn);
        if (!aligned(t->r, 8) || !aligned(t->beta, 8) || !aligned(t->beta_dot, 8) ||
            (t->charge && !aligned(t->charge, 8)))
            return fail(LW_E_ALIGN, "%s: trajectory arrays must be 8-byte aligned", fn);
    }
    return LW_OK;
}

lw_status check_grid(const lw_grid_t *g, const char *fn, bool need_grid)
{
    if (!g) return fail(LW_E_ARG, "%s: grid is NULL", fn);
    if (g->n_pix < 0) return fail(LW_E_SHAPE, "%s: n_pix < 0", fn);
    if (g->n_pix > 0 && !g->x_det) return fail(LW_E_ARG, "%s: x_det is NULL", fn);
    if (g->x_det && !aligned(g->x_det, 8)) return fail(LW_E_ALIGN, "%s: x_det must be 8-byte aligned", fn);
    if (!(g->t0 > -1e300 && g->t0 < 1e300)) return fail(LW_E_ARG, "%s: t0 must be finite", fn);
    if (need_grid) {
        if (!finite_pos(g->dt_obs)) return fail(LW_E_ARG, "%s: dt_obs must be positive and finite", fn);
        if (g->n_obs < 1 || g->n_obs > 0x7fffffff) return fail(LW_E_SHAPE, "%s: n_obs out of range [1, 2^31)", fn);
    }
    return LW_OK;
}

bool pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// spans: whether this call pushes in spans (the deposit and its adjoint), where traj->span
// may also be >= 2
lw_status check_traj_boris(const lw_traj_t *t, const char *fn, bool spans = false)
{
    if (!t) return fail(LW_E_ARG, "%s: traj is NULL", fn);
    if (t->kind != LW_TRAJ_BORIS) return fail(LW_E_ARG, "%s: traj->kind must be LW_TRAJ_BORIS", fn);
    if (t->span != 0 && !(spans && t->span >= 2))
        return fail(LW_E_ARG, "%s: traj->span must be 0%s", fn, spans ? " or >= 2" : "");
    if (t->n_particles < 0 || t->n_particles > (int64_t(1) << 28) || t->n_samples < 1 || t->n_samples >= kMaxSamples)
        return fail(LW_E_SHAPE, "%s: bad sizes", fn);
    if (!finite_pos(t->dt) || !(t->t_start > -1e300 && t->t_start < 1e300))
        return fail(LW_E_ARG, "%s: dt must be positive and finite, t_start finite", fn);
    const lw_laser_t &L = t->laser;
    if (!finite_pos(L.lambda) || !(L.n_cycles > 0.0) || !(L.a0 >= 0.0 && L.a0 < 1e6) || !(L.w0 < 1e300))
        return fail(LW_E_ARG, "%s: laser parameters out of range", fn);
    if (t->n_particles > 0 && !t->init) return fail(LW_E_ARG, "%s: init is NULL", fn);
    if ((t->init && !aligned(t->init, 8)) || (t->charge && !aligned(t->charge, 8)))
        return fail(LW_E_ALIGN, "%s: init and charge must be 8-byte aligned", fn);
    return LW_OK;
}

}  // namespace
}  // namespace lw

using namespace lw;

extern "C" {

const char *lw_last_error(void) { return g_err; }

lw_status lw_timing_enable(int on)
{
    std::lock_guard<std::mutex> lk(g_tm);
    g_timing = on != 0;
    if (!g_timing) {
        for (const TimedLaunch &t : g_timed) {
            (void)hipEventSynchronize(t.b);
            g_pool.push_back(t.a);
            g_pool.push_back(t.b);
        }
        g_timed.clear();
    }
    return LW_OK;
}

lw_status lw_timing_read(int which, double *total_ms, int64_t *launches)
{
    if (which != LW_KERNEL_DEPOSIT && which != LW_KERNEL_DEPOSIT_BWD && which != LW_KERNEL_BORIS_TANGENT)
        return fail(LW_E_ARG, "lw_timing_read: unknown kernel %d", which);
    if (!total_ms || !launches) return fail(LW_E_ARG, "lw_timing_read: NULL output");
    std::lock_guard<std::mutex> lk(g_tm);
    double sum = 0.0;
    int64_t n = 0;
    lw_status st = LW_OK;
    std::vector<TimedLaunch> keep;
    for (const TimedLaunch &t : g_timed) {
        if (t.which != which) {
            keep.push_back(t);
            continue;
        }
        float ms = 0.0f;
        if (hipEventSynchronize(t.b) != hipSuccess || hipEventElapsedTime(&ms, t.a, t.b) != hipSuccess)
            st = fail(LW_E_HIP, "lw_timing_read: event query failed");
        sum += ms;
        ++n;
        g_pool.push_back(t.a);
        g_pool.push_back(t.b);
    }
    g_timed.swap(keep);
    *total_ms = sum;
    *launches = n;
    return st;
}

const char *lw_version(void) { return "liblw 0.1 (gfx950)"; }

size_t lw_workspace_bytes(int which, int64_t n_a, int64_t n_b, int prec)
{
    switch (which) {
    case LW_WS_DEPOSIT:
        return deposit_ws_bytes(n_a, n_b, prec);
    case LW_WS_DEPOSIT_BWD:
        return deposit_bwd_ws_bytes(n_a);
    case LW_WS_FFT:
    case LW_WS_FFT_BWD:
        return fft_ws_bytes(n_a, n_b, prec);
    case LW_WS_DIRECT_FD:
    case LW_WS_DIRECT_FD_BWD:
        return direct_fd_ws_bytes(n_a, n_b);
    case LW_WS_DEPOSIT_BORIS:
        return n_b >= 1 ? boris_plan_ws_bytes(boris_plan_default(n_a, n_b, prec), prec) : 0;
    case LW_WS_DEPOSIT_BWD_BORIS:
        return n_b >= 1 ? boris_plan_ws_bytes(boris_plan_default(n_a, n_b, LW_PREC_FP64, true), LW_PREC_FP64, true)
                        : 0;
    case LW_WS_DEPOSIT_DET_ACC:
        return n_a >= 0 && n_b >= 0 ? det_acc_bytes(n_a, n_b) : 0;
    default:
        return 0;
    }
}

// lw_deposit_td and lw_deposit_td_det (acc != nullptr: the order-independent FP64 deposit)
static lw_status deposit_entry(const char *fn, const lw_traj_t *traj, const lw_grid_t *grid, int prec, int field_mask,
                               int geom, void *E, int64_t *diag, void *acc, size_t acc_bytes, void *ws,
                               size_t ws_bytes, hipStream_t stream)
{
    const bool boris = traj && traj->kind == LW_TRAJ_BORIS;
    lw_status st = boris ? check_traj_boris(traj, fn, true) : check_traj_samples(traj, fn);
    if (st != LW_OK) return st;
    if ((st = check_grid(grid, fn, true)) != LW_OK) return st;
    if (prec != LW_PREC_FP64 && prec != LW_PREC_MIXED) return fail(LW_E_ARG, "%s: unknown prec %d", fn, prec);
    if (field_mask <= 0 || (field_mask & ~(LW_FIELD_ACCEL | LW_FIELD_VELOCITY)))
        return fail(LW_E_ARG, "%s: field_mask must be a non-empty combination of LW_FIELD_*", fn);
    const bool accum = (geom & LW_ACCUMULATE) != 0;
    const int g = geom & ~(LW_ACCUMULATE | LW_CULL);
    if (g != LW_GEOM_EXACT && g != LW_GEOM_FARFIELD) return fail(LW_E_ARG, "%s: unknown geometry %d", fn, g);
    const int gc = g | (geom & LW_CULL);  // geometry and culling for the launchers
    if (grid->n_pix > 0 && !E) return fail(LW_E_ARG, "%s: E is NULL", fn);
    if (E && !aligned(E, 16)) return fail(LW_E_ALIGN, "%s: E must be 16-byte aligned", fn);
    if (diag && !aligned(diag, 8)) return fail(LW_E_ALIGN, "%s: diag must be 8-byte aligned", fn);
    if (grid->n_pix > (int64_t(1) << 31) || traj->n_particles > (int64_t(1) << 40))
        return fail(LW_E_SHAPE, "%s: too many pixels or particles", fn);
    if (ws && !aligned(ws, 256)) return fail(LW_E_ALIGN, "%s: workspace must be 256-byte aligned", fn);
    const bool det = acc_bytes > 0 || acc;
    if (det) {
        if (geom & (LW_ACCUMULATE | LW_CULL)) return fail(LW_E_ARG, "%s: LW_ACCUMULATE and LW_CULL are not taken", fn);
        const size_t need = det_acc_bytes(grid->n_pix, grid->n_obs);
        if (!acc || acc_bytes < need)
            return fail(LW_E_WORKSPACE, "%s: accumulator buffer of %zu bytes < %zu needed", fn, acc_bytes, need);
        if (!aligned(acc, 256)) return fail(LW_E_ALIGN, "%s: accumulator buffer must be 256-byte aligned", fn);
    }
    if (boris) {
        const bool work = traj->n_particles > 0 && grid->n_pix > 0;
        const BorisPlan plan = boris_plan_fit(traj->n_particles, traj->n_samples, traj->span, ws_bytes, prec);
        const int64_t lmin = std::min<int64_t>(traj->n_samples, 2);
        if (work && (!ws || plan.batch < 1 || plan.span < lmin))
            return fail(LW_E_WORKSPACE, "%s: workspace of %zu bytes holds no span (one particle needs %zu)", fn,
                        ws_bytes, boris_plan_ws_bytes(BorisPlan{1, traj->span > 0 ? traj->span : lmin}, prec));
        if (det) return launch_deposit_det(traj, grid, field_mask, g, (double *)E, diag, acc, ws, ws_bytes, stream);
        return launch_deposit_boris(traj, grid, prec, field_mask, gc, accum, E, diag, ws, ws_bytes, stream);
    }
    // any workspace that holds one particle's records is accepted (the particles are then taken
    // in chunks); lw_workspace_bytes gives the size that takes them all at once
    const size_t need = deposit_ws_bytes(1, traj->n_samples, prec);
    if (traj->n_particles > 0 && grid->n_pix > 0 && (!ws || ws_bytes < need))
        return fail(LW_E_WORKSPACE, "%s: workspace of %zu bytes < %zu needed", fn, ws_bytes, need);
    if (det) return launch_deposit_det(traj, grid, field_mask, g, (double *)E, diag, acc, ws, ws_bytes, stream);
    return launch_deposit(traj, grid, prec, field_mask, gc, accum, E, diag, ws, ws_bytes, stream);
}

lw_status lw_deposit_td(const lw_traj_t *traj, const lw_grid_t *grid, int prec, int field_mask, int geom, void *E,
                        int64_t *diag, void *ws, size_t ws_bytes, hipStream_t stream)
{
    return deposit_entry("lw_deposit_td", traj, grid, prec, field_mask, geom, E, diag, nullptr, 0, ws, ws_bytes,
                         stream);
}

lw_status lw_deposit_td_det(const lw_traj_t *traj, const lw_grid_t *grid, int field_mask, int geom, double *E,
                            int64_t *diag, void *acc, size_t acc_bytes, void *ws, size_t ws_bytes, hipStream_t stream)
{
    if (!acc && acc_bytes == 0) return fail(LW_E_WORKSPACE, "lw_deposit_td_det: no accumulator buffer");
    return deposit_entry("lw_deposit_td_det", traj, grid, LW_PREC_FP64, field_mask, geom, E, diag, acc, acc_bytes, ws,
                         ws_bytes, stream);
}

lw_status lw_spectrum_fft(const void *E, int64_t n_pix, int64_t n_obs, double dt_obs, int prec, void *S, void *ws,
                          size_t ws_bytes, hipStream_t stream)
{
    const char *fn = "lw_spectrum_fft";
    if (prec != LW_PREC_FP64 && prec != LW_PREC_MIXED) return fail(LW_E_ARG, "%s: unknown prec %d", fn, prec);
    if (n_pix < 0) return fail(LW_E_SHAPE, "%s: n_pix < 0", fn);
    if (!pow2(n_obs) || n_obs < 4 || n_obs > (int64_t(1) << 22))
        return fail(LW_E_SHAPE, "%s: n_obs must be a power of two in [4, 2^22] (got %lld)", fn, (long long)n_obs);
    if (!finite_pos(dt_obs)) return fail(LW_E_ARG, "%s: dt_obs must be positive and finite", fn);
    if (n_pix > 0 && (!E || !S)) return fail(LW_E_ARG, "%s: E and S must be non-NULL", fn);
    if ((E && !aligned(E, 16)) || (S && !aligned(S, 16)) || (ws && !aligned(ws, 256)))
        return fail(LW_E_ALIGN, "%s: E, S must be 16-byte and ws 256-byte aligned", fn);
    return launch_fft(E, n_pix, n_obs, dt_obs, prec, S, ws, ws_bytes, stream);
}

lw_status lw_spectrum_fft_noalloc(const void *E, int64_t n_pix, int64_t n_obs, double dt_obs, int prec, void *S,
                                  hipStream_t stream)
{
    const char *fn = "lw_spectrum_fft_noalloc";
    if (prec != LW_PREC_FP64 && prec != LW_PREC_MIXED) return fail(LW_E_ARG, "%s: unknown prec %d", fn, prec);
    if (n_pix < 0) return fail(LW_E_SHAPE, "%s: n_pix < 0", fn);
    if (!pow2(n_obs) || n_obs < 4 || n_obs > (int64_t(1) << 22))
        return fail(LW_E_SHAPE, "%s: n_obs must be a power of two in [4, 2^22] (got %lld)", fn, (long long)n_obs);
    if (!finite_pos(dt_obs)) return fail(LW_E_ARG, "%s: dt_obs must be positive and finite", fn);
    if (n_pix > 0 && (!E || !S)) return fail(LW_E_ARG, "%s: E and S must be non-NULL", fn);
    if ((E && !aligned(E, 16)) || (S && !aligned(S, 16)))
        return fail(LW_E_ALIGN, "%s: E and S must be 16-byte aligned", fn);
    return launch_fft_noalloc(E, n_pix, n_obs, dt_obs, prec, S, stream);
}

size_t lw_noalloc_scratch_bytes(void) { return fft_noalloc_scratch_bytes(); }

lw_status lw_direct_fd(const lw_traj_t *traj, const lw_grid_t *grid, const double *omega, int64_t n_omega, int prec,
                       int field_mask, int geom, double *S, void *ws, size_t ws_bytes, hipStream_t stream)
{
    const char *fn = "lw_direct_fd";
    lw_status st = check_traj_samples(traj, fn);
    if (st != LW_OK) return st;
    if ((st = check_grid(grid, fn, false)) != LW_OK) return st;
    if (prec != LW_PREC_FP64 && prec != LW_PREC_MIXED) return fail(LW_E_ARG, "%s: unknown prec %d", fn, prec);
    if (field_mask <= 0 || (field_mask & ~(LW_FIELD_ACCEL | LW_FIELD_VELOCITY)))
        return fail(LW_E_ARG, "%s: field_mask must be a non-empty combination of LW_FIELD_*", fn);
    if (geom != LW_GEOM_EXACT && geom != LW_GEOM_FARFIELD) return fail(LW_E_ARG, "%s: unknown geometry %d", fn, geom);
    if (n_omega < 0) return fail(LW_E_SHAPE, "%s: n_omega < 0", fn);
    if (n_omega > 0 && !omega) return fail(LW_E_ARG, "%s: omega is NULL", fn);
    if (n_omega > 0 && grid->n_pix > 0 && !S) return fail(LW_E_ARG, "%s: S is NULL", fn);
    if ((omega && !aligned(omega, 8)) || (S && !aligned(S, 8)) || (ws && !aligned(ws, 256)))
        return fail(LW_E_ALIGN, "%s: misaligned pointer", fn);
    const size_t need = direct_fd_ws_bytes(grid->n_pix, n_omega);
    if (n_omega > 0 && grid->n_pix > 0 && (!ws || ws_bytes < need))
        return fail(LW_E_WORKSPACE, "%s: workspace of %zu bytes < %zu needed", fn, ws_bytes, need);
    return launch_direct_fd(traj, grid, omega, n_omega, prec, field_mask, geom, S, ws, ws_bytes, stream);
}

lw_status lw_trajectory_boris(const lw_traj_t *traj, double *r, double *beta, double *beta_dot, hipStream_t stream)
{
    const char *fn = "lw_trajectory_boris";
    if (!traj) return fail(LW_E_ARG, "%s: traj is NULL", fn);
    if (traj->kind != LW_TRAJ_BORIS) return fail(LW_E_ARG, "%s: traj->kind must be LW_TRAJ_BORIS", fn);
    if (traj->span != 0) return fail(LW_E_ARG, "%s: traj->span must be 0", fn);
    if (traj->n_particles < 0 || traj->n_samples < 1 || traj->n_samples >= (int64_t(1) << 31))
        return fail(LW_E_SHAPE, "%s: bad sizes", fn);
    if (!finite_pos(traj->dt)) return fail(LW_E_ARG, "%s: dt must be positive and finite", fn);
    const lw_laser_t &L = traj->laser;
    if (!finite_pos(L.lambda) || !(L.n_cycles > 0.0) || !(L.a0 >= 0.0 && L.a0 < 1e6) || !(L.w0 < 1e300))
        return fail(LW_E_ARG, "%s: laser parameters out of range", fn);
    if (traj->n_particles > 0 && (!traj->init || !r || !beta || !beta_dot))
        return fail(LW_E_ARG, "%s: NULL array", fn);
    if ((traj->init && !aligned(traj->init, 8)) || (r && !aligned(r, 8)) || (beta && !aligned(beta, 8)) ||
        (beta_dot && !aligned(beta_dot, 8)))
        return fail(LW_E_ALIGN, "%s: arrays must be 8-byte aligned", fn);
    return launch_boris(traj, r, beta, beta_dot, stream);
}

lw_status lw_trajectory_boris_bwd(const lw_traj_t *traj, const double *g_r, const double *g_beta,
                                  const double *g_beta_dot, double *grad_init, double *grad_a0, hipStream_t stream)
{
    const char *fn = "lw_trajectory_boris_bwd";
    if (!traj) return fail(LW_E_ARG, "%s: traj is NULL", fn);
    if (traj->kind != LW_TRAJ_BORIS) return fail(LW_E_ARG, "%s: traj->kind must be LW_TRAJ_BORIS", fn);
    if (traj->span != 0) return fail(LW_E_ARG, "%s: traj->span must be 0", fn);
    if (traj->n_particles < 0 || traj->n_samples < 1 || traj->n_samples >= (int64_t(1) << 31) ||
        traj->n_particles > (int64_t(1) << 28))
        return fail(LW_E_SHAPE, "%s: bad sizes", fn);
    if (!finite_pos(traj->dt)) return fail(LW_E_ARG, "%s: dt must be positive and finite", fn);
    const lw_laser_t &L = traj->laser;
    if (!finite_pos(L.lambda) || !(L.n_cycles > 0.0) || !(L.a0 >= 0.0 && L.a0 < 1e6) || !(L.w0 < 1e300))
        return fail(LW_E_ARG, "%s: laser parameters out of range", fn);
    if (traj->n_particles > 0 && (!traj->init || !g_r || !g_beta || !g_beta_dot || !grad_init || !grad_a0))
        return fail(LW_E_ARG, "%s: NULL array", fn);
    for (const void *p : {(const void *)traj->init, (const void *)g_r, (const void *)g_beta, (const void *)g_beta_dot,
                          (const void *)grad_init, (const void *)grad_a0})
        if (p && !aligned(p, 8)) return fail(LW_E_ALIGN, "%s: arrays must be 8-byte aligned", fn);
    return launch_boris_bwd(traj, g_r, g_beta, g_beta_dot, grad_init, grad_a0, stream);
}

lw_status lw_spectrum_fft_bwd(const void *E, const void *dS, int64_t n_pix, int64_t n_obs, double dt_obs, int prec,
                              void *dE, void *ws, size_t ws_bytes, hipStream_t stream)
{
    const char *fn = "lw_spectrum_fft_bwd";
    if (prec != LW_PREC_FP64 && prec != LW_PREC_MIXED) return fail(LW_E_ARG, "%s: unknown prec %d", fn, prec);
    if (n_pix < 0) return fail(LW_E_SHAPE, "%s: n_pix < 0", fn);
    if (!pow2(n_obs) || n_obs < 4 || n_obs > (int64_t(1) << 22))
        return fail(LW_E_SHAPE, "%s: n_obs must be a power of two in [4, 2^22] (got %lld)", fn, (long long)n_obs);
    if (!finite_pos(dt_obs)) return fail(LW_E_ARG, "%s: dt_obs must be positive and finite", fn);
    if (n_pix > 0 && (!E || !dS || !dE)) return fail(LW_E_ARG, "%s: E, dS and dE must be non-NULL", fn);
    if ((E && !aligned(E, 16)) || (dS && !aligned(dS, 16)) || (dE && !aligned(dE, 16)) || (ws && !aligned(ws, 256)))
        return fail(LW_E_ALIGN, "%s: E, dS, dE must be 16-byte and ws 256-byte aligned", fn);
    if (E == (const void *)dE) return fail(LW_E_ARG, "%s: dE must not alias E", fn);
    return launch_fft_bwd(E, dS, n_pix, n_obs, dt_obs, prec, dE, ws, ws_bytes, stream);
}

lw_status lw_deposit_td_bwd(const lw_traj_t *traj, const lw_grid_t *grid, int prec, int field_mask, int geom,
                            const void *dE, double *d_r, double *d_beta, double *d_beta_dot, void *ws,
                            size_t ws_bytes, hipStream_t stream)
{
    const char *fn = "lw_deposit_td_bwd";
    lw_status st = check_traj_samples(traj, fn);
    if (st != LW_OK) return st;
    if ((st = check_grid(grid, fn, true)) != LW_OK) return st;
    if (prec == LW_PREC_MIXED) return fail(LW_E_UNSUPPORTED, "%s: only LW_PREC_FP64 is supported", fn);
    if (prec != LW_PREC_FP64) return fail(LW_E_ARG, "%s: unknown prec %d", fn, prec);
    if (field_mask <= 0 || (field_mask & ~(LW_FIELD_ACCEL | LW_FIELD_VELOCITY)))
        return fail(LW_E_ARG, "%s: field_mask must be a non-empty combination of LW_FIELD_*", fn);
    if (geom != LW_GEOM_EXACT && geom != LW_GEOM_FARFIELD) return fail(LW_E_ARG, "%s: unknown geometry %d", fn, geom);
    if (traj->n_particles > 0 && grid->n_pix > 0 && (!dE || !d_r || !d_beta || !d_beta_dot))
        return fail(LW_E_ARG, "%s: dE, d_r, d_beta, d_beta_dot must be non-NULL", fn);
    if ((dE && !aligned(dE, 16)) || (d_r && !aligned(d_r, 8)) || (d_beta && !aligned(d_beta, 8)) ||
        (d_beta_dot && !aligned(d_beta_dot, 8)) || (ws && !aligned(ws, 256)))
        return fail(LW_E_ALIGN, "%s: misaligned pointer", fn);
    const size_t need = deposit_bwd_ws_bytes(traj->n_particles);
    if (traj->n_particles > 0 && grid->n_pix > 0 && traj->n_samples >= 2 && (!ws || ws_bytes < need))
        return fail(LW_E_WORKSPACE, "%s: workspace of %zu bytes < %zu needed", fn, ws_bytes, need);
    return launch_deposit_bwd(traj, grid, field_mask, geom, (const double *)dE, d_r, d_beta, d_beta_dot, ws, ws_bytes,
                              stream);
}

lw_status lw_deposit_td_bwd_boris(const lw_traj_t *traj, const lw_grid_t *grid, int prec, int field_mask, int geom,
                                  const void *dE, double *grad_init, double *grad_a0, void *ws, size_t ws_bytes,
                                  hipStream_t stream)
{
    const char *fn = "lw_deposit_td_bwd_boris";
    lw_status st = check_traj_boris(traj, fn, true);
    if (st != LW_OK) return st;
    if ((st = check_grid(grid, fn, true)) != LW_OK) return st;
    if (prec == LW_PREC_MIXED) return fail(LW_E_UNSUPPORTED, "%s: only LW_PREC_FP64 is supported", fn);
    if (prec != LW_PREC_FP64) return fail(LW_E_ARG, "%s: unknown prec %d", fn, prec);
    if (field_mask <= 0 || (field_mask & ~(LW_FIELD_ACCEL | LW_FIELD_VELOCITY)))
        return fail(LW_E_ARG, "%s: field_mask must be a non-empty combination of LW_FIELD_*", fn);
    if (geom != LW_GEOM_EXACT && geom != LW_GEOM_FARFIELD) return fail(LW_E_ARG, "%s: unknown geometry %d", fn, geom);
    const bool work = traj->n_particles > 0;
    if (work && (!grad_init || !grad_a0 || (grid->n_pix > 0 && !dE))) return fail(LW_E_ARG, "%s: NULL array", fn);
    if ((dE && !aligned(dE, 16)) || (grad_init && !aligned(grad_init, 8)) || (grad_a0 && !aligned(grad_a0, 8)) ||
        (ws && !aligned(ws, 256)))
        return fail(LW_E_ALIGN, "%s: misaligned pointer", fn);
    if (work && grid->n_pix > 0 && traj->n_samples >= 2) {
        const BorisPlan plan =
            boris_plan_fit(traj->n_particles, traj->n_samples, traj->span, ws_bytes, LW_PREC_FP64, true);
        if (!ws || plan.batch < 1 || plan.span < 2)
            return fail(LW_E_WORKSPACE, "%s: workspace of %zu bytes holds no span (one particle needs %zu)", fn,
                        ws_bytes,
                        boris_plan_ws_bytes(BorisPlan{1, traj->span > 0 ? traj->span : 2}, LW_PREC_FP64, true));
    }
    return launch_deposit_bwd_boris(traj, grid, field_mask, geom, (const double *)dE, grad_init, grad_a0, ws, ws_bytes,
                                    stream);
}

lw_status lw_direct_fd_bwd(const lw_traj_t *traj, const lw_grid_t *grid, const double *omega, int64_t n_omega,
                           int prec, int field_mask, int geom, const double *dS, double *d_r, double *d_beta,
                           double *d_beta_dot, void *ws, size_t ws_bytes, hipStream_t stream)
{
    const char *fn = "lw_direct_fd_bwd";
    lw_status st = check_traj_samples(traj, fn);
    if (st != LW_OK) return st;
    if ((st = check_grid(grid, fn, false)) != LW_OK) return st;
    if (prec == LW_PREC_MIXED) return fail(LW_E_UNSUPPORTED, "%s: only LW_PREC_FP64 is supported", fn);
    if (prec != LW_PREC_FP64) return fail(LW_E_ARG, "%s: unknown prec %d", fn, prec);
    if (field_mask <= 0 || (field_mask & ~(LW_FIELD_ACCEL | LW_FIELD_VELOCITY)))
        return fail(LW_E_ARG, "%s: field_mask must be a non-empty combination of LW_FIELD_*", fn);
    if (geom != LW_GEOM_EXACT && geom != LW_GEOM_FARFIELD) return fail(LW_E_ARG, "%s: unknown geometry %d", fn, geom);
    if (n_omega < 0) return fail(LW_E_SHAPE, "%s: n_omega < 0", fn);
    const bool work = n_omega > 0 && grid->n_pix > 0 && traj->n_particles > 0;
    if (work && (!omega || !dS || !d_r || !d_beta || !d_beta_dot)) return fail(LW_E_ARG, "%s: NULL array", fn);
    for (const void *p : {(const void *)omega, (const void *)dS, (const void *)d_r, (const void *)d_beta,
                          (const void *)d_beta_dot})
        if (p && !aligned(p, 8)) return fail(LW_E_ALIGN, "%s: arrays must be 8-byte aligned", fn);
    if (ws && !aligned(ws, 256)) return fail(LW_E_ALIGN, "%s: ws must be 256-byte aligned", fn);
    const size_t need = direct_fd_ws_bytes(grid->n_pix, n_omega);
    if (work && (!ws || ws_bytes < need))
        return fail(LW_E_WORKSPACE, "%s: workspace of %zu bytes < %zu needed", fn, ws_bytes, need);
    return launch_direct_fd_bwd(traj, grid, omega, n_omega, field_mask, geom, dS, d_r, d_beta, d_beta_dot, ws,
                                ws_bytes, stream);
}

}  // extern "C"
