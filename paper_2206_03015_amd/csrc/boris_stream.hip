// Deposit and its adjoint for trajectories given as initial conditions plus a laser pulse
// (LW_TRAJ_BORIS): the FP64 Boris pusher recomputes the samples inside the library, so the
// whole trajectory set is never stored (the paper's time-domain method with the trajectory
// update inside the particle loop, and its on-the-fly evaluation over time).  The deposit
// pushes a batch of particles over a span of samples into the workspace, deposits it
// (accumulating after the first) and reuses the space for the next span: spans share their
// boundary sample, the pusher's state (position and the two momenta) is kept between them, so
// the samples are those of one uninterrupted push and the trajectory length is unbounded.
// The adjoint takes the same spans: per span the samples, the deposit adjoint over the span's
// intervals, then the pusher's tangents over the span, their dual-number state kept between
// spans like the pusher's.
#include "lw_internal.h"

#include <algorithm>

namespace lw {
namespace {

// default workspace budget of a plan
constexpr size_t kBatchBytes = size_t(16) << 30;
// the pusher runs one lane per particle through every step of a span, so its time is the
// per-step latency of one wavefront times the span length for up to one wavefront per SIMD
// (1024 SIMDs x 64 lanes): batches of up to that many particles, spans as long as fit
constexpr int64_t kFillParticles = 65536;
// spans shorter than this give way to smaller batches (each span is one deposit launch)
constexpr int64_t kMinSpan = 1024;
// longest span one deposit launch takes (its pre-pass grid covers 8192 samples per block row)
constexpr int64_t kMaxSpan = int64_t(1) << 28;
constexpr int kStateBytes = 9 * sizeof(double);
// the adjoint runs seven tangent lanes per particle: batches of up to three wavefronts of them per
// SIMD (3 x 1024 x 64 / 7 particles).  Larger batches also push each trajectory's first pass
// (max |r|^2) fewer times.  Deposit-and-pusher adjoint of the large workload: 16384 particles
// 787 ms, 28086 633-640 ms, 40960 654 ms, 65536 648 ms
constexpr int64_t kFillParticlesBwd = 28086;
constexpr int kTanStateBytes = 7 * 18 * sizeof(double);

inline size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// workspace of a plan.  Forward: deposit scratch (records of the span), pusher states, the
// particles' max |r|^2, r, beta, beta_dot of the span.  Adjoint (bwd): tangent states, pusher
// states, the particles' max |r|^2, the span's samples and their gradients.
size_t plan_bytes(int64_t B, int64_t L, int prec, bool bwd)
{
    const size_t arr = align256((size_t)B * (size_t)L * 3 * sizeof(double));
    const size_t rb = align256((size_t)B * sizeof(double));
    if (bwd) return align256((size_t)B * kTanStateBytes) + align256((size_t)B * kStateBytes) + rb + 6 * arr;
    return align256(deposit_ws_bytes(B, L, prec)) + align256((size_t)B * kStateBytes) + rb + 3 * arr;
}

// bytes per (particle, sample) of a plan: samples (72), records (forward) or gradients (adjoint)
size_t per_sample_bytes(int prec, bool bwd) { return bwd ? 144 : 72 + (prec == LW_PREC_FP64 ? 80 : 64); }

// longest span (<= lmax) of B particles within `bytes` (0 if not even one sample fits)
int64_t fit_span(int64_t B, int64_t lmax, size_t bytes, int prec, bool bwd)
{
    const size_t fixed = plan_bytes(B, 1, prec, bwd);
    if (fixed > bytes) return 0;
    const size_t per_sample = (size_t)B * per_sample_bytes(prec, bwd);
    int64_t L = std::min<int64_t>(lmax, 1 + (int64_t)((bytes - fixed) / per_sample));
    while (L > 1 && plan_bytes(B, L, prec, bwd) > bytes) --L;
    return L;
}

// largest batch (<= bmax) with spans of L samples within `bytes` (0 if none)
int64_t fit_batch(int64_t bmax, int64_t L, size_t bytes, int prec, bool bwd)
{
    const size_t fixed = plan_bytes(1, L, prec, bwd);
    if (fixed > bytes) return 0;
    const size_t per_particle_bytes = (size_t)L * per_sample_bytes(prec, bwd) + kStateBytes + 3 * sizeof(double) +
                                      (bwd ? kTanStateBytes : 0);
    int64_t B = std::min<int64_t>(bmax, 1 + (int64_t)((bytes - fixed) / per_particle_bytes));
    while (B > 1 && plan_bytes(B, L, prec, bwd) > bytes) --B;
    return B;
}

__global__ void k_zero(double *__restrict__ p, int64_t n)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        p[j] = 0.0;
}

}  // namespace

// Batch and span from the workspace: batches of min(n_p, kFillParticles) particles over the
// longest spans that fit (whole trajectories when they do); spans shorter than kMinSpan give
// way to smaller batches; a requested span fixes L and leaves the batch to the workspace.
BorisPlan boris_plan_fit(int64_t n_p, int64_t ns, int64_t span_req, size_t ws_bytes, int prec, bool bwd)
{
    const int64_t b0 = std::max<int64_t>(1, std::min<int64_t>(n_p, bwd ? kFillParticlesBwd : kFillParticles));
    const int64_t lmax = std::min<int64_t>(ns, kMaxSpan);
    const int64_t lmin = std::min<int64_t>(lmax, 2);  // a span must advance (one interval at least)
    if (span_req > 0) {
        const int64_t L = std::max<int64_t>(lmin, std::min<int64_t>(span_req, lmax));
        return {fit_batch(b0, L, ws_bytes, prec, bwd), L};
    }
    const int64_t L0 = fit_span(b0, lmax, ws_bytes, prec, bwd);
    if (L0 >= std::min<int64_t>(lmax, kMinSpan)) return {b0, L0};
    const int64_t Lm = std::min<int64_t>(lmax, kMinSpan);
    const int64_t B = fit_batch(b0, Lm, ws_bytes, prec, bwd);
    if (B >= 1) return {B, Lm};
    const int64_t L1 = fit_span(1, lmax, ws_bytes, prec, bwd);
    if (L1 >= lmin) return {1, L1};
    return {0, 0};
}

BorisPlan boris_plan_default(int64_t n_p, int64_t ns, int prec, bool bwd)
{
    const BorisPlan p = boris_plan_fit(n_p, ns, 0, kBatchBytes, prec, bwd);
    // a budget too small for even one particle's two-sample span cannot happen at 16 GiB
    return p.batch > 0 ? p : BorisPlan{1, std::min<int64_t>(ns, 2)};
}

size_t boris_plan_ws_bytes(const BorisPlan &p, int prec, bool bwd)
{
    return plan_bytes(std::max<int64_t>(p.batch, 1), p.span, prec, bwd);
}

lw_status launch_deposit_boris(const lw_traj_t *t, const lw_grid_t *gr, int prec, int fmask, int geom,
                               bool accumulate, void *E, int64_t *diag, void *ws, size_t ws_bytes, hipStream_t s,
                               int acc_mode, DetAcc det)
{
    const int64_t n_p = t->n_particles, ns = t->n_samples;
    if (n_p == 0 || gr->n_pix == 0) {  // nothing to push: only the trace and diag reset of the plain call
        lw_traj_t sub = *t;
        sub.kind = LW_TRAJ_SAMPLES;
        sub.span = 0;
        sub.n_particles = 0;
        sub.r = sub.beta = sub.beta_dot = nullptr;
        return launch_deposit(&sub, gr, prec, fmask, geom, accumulate, E, diag, ws, ws_bytes, s, 0, nullptr, acc_mode,
                              det);
    }
    const BorisPlan P = boris_plan_fit(n_p, ns, t->span, ws_bytes, prec);
    if (P.batch < 1 || (ns > 1 && P.span < 2)) return fail(LW_E_WORKSPACE, "lw_deposit_td: workspace holds no span");
    const size_t dep_bytes = align256(deposit_ws_bytes(P.batch, P.span, prec));
    char *p = (char *)ws + dep_bytes;
    double *state = (double *)p;
    p += align256((size_t)P.batch * kStateBytes);
    double *rb2 = (double *)p;
    p += align256((size_t)P.batch * sizeof(double));
    const size_t arr = align256((size_t)P.batch * (size_t)P.span * 3 * sizeof(double));
    double *r = (double *)p, *b = (double *)(p + arr), *bd = (double *)(p + 2 * arr);
    for (int64_t b0 = 0; b0 < n_p; b0 += P.batch) {
        const int64_t nb = std::min<int64_t>(P.batch, n_p - b0);
        lw_traj_t push = *t;
        push.n_particles = nb;
        push.init = t->init + 6 * b0;
        // max |r|^2 over each whole trajectory: every span takes the same arrival-time forms
        lw_status st = launch_boris_rmax2(&push, rb2, s);
        if (st != LW_OK) return st;
        for (int64_t s0 = 0;;) {
            const int64_t n_span = std::min<int64_t>(P.span, ns - s0);
            st = launch_boris_span(&push, s0, n_span, state, r, b, bd, s);
            if (st != LW_OK) return st;
            lw_traj_t sub = *t;
            sub.kind = LW_TRAJ_SAMPLES;
            sub.span = 0;
            sub.n_particles = nb;
            sub.n_samples = n_span;
            sub.r = r;
            sub.beta = b;
            sub.beta_dot = bd;
            sub.init = nullptr;
            sub.charge = t->charge ? t->charge + b0 : nullptr;
            st = launch_deposit(&sub, gr, prec, fmask, geom, accumulate || b0 > 0 || s0 > 0, E, diag, ws, dep_bytes,
                                s, s0, rb2, acc_mode, det);
            if (st != LW_OK) return st;
            if (s0 + n_span >= ns) break;
            s0 += n_span - 1;  // the next span starts at this span's last sample
        }
    }
    return LW_OK;
}

lw_status launch_deposit_bwd_boris(const lw_traj_t *t, const lw_grid_t *gr, int fmask, int geom, const double *dE,
                                   double *grad_init, double *grad_a0, void *ws, size_t ws_bytes, hipStream_t s)
{
    const int64_t n_p = t->n_particles, ns = t->n_samples;
    if (n_p == 0) return LW_OK;
    if (gr->n_pix == 0 || ns < 2) {  // no pixels or no interval: the gradient is zero
        k_zero<<<(int)std::min<int64_t>((6 * n_p + 255) / 256, 65536), 256, 0, s>>>(grad_init, 6 * n_p);
        k_zero<<<(int)std::min<int64_t>((n_p + 255) / 256, 65536), 256, 0, s>>>(grad_a0, n_p);
        return check_launch("lw_deposit_td_bwd_boris");
    }
    const BorisPlan P = boris_plan_fit(n_p, ns, t->span, ws_bytes, LW_PREC_FP64, true);
    if (P.batch < 1 || P.span < 2) return fail(LW_E_WORKSPACE, "lw_deposit_td_bwd_boris: workspace holds no span");
    char *p = (char *)ws;
    double *tstate = (double *)p;
    p += align256((size_t)P.batch * kTanStateBytes);
    double *pstate = (double *)p;
    p += align256((size_t)P.batch * kStateBytes);
    double *rb2 = (double *)p;
    p += align256((size_t)P.batch * sizeof(double));
    const size_t arr = align256((size_t)P.batch * (size_t)P.span * 3 * sizeof(double));
    double *r = (double *)p, *b = (double *)(p + arr), *bd = (double *)(p + 2 * arr);
    double *gr_ = (double *)(p + 3 * arr), *gb = (double *)(p + 4 * arr), *ga = (double *)(p + 5 * arr);
    for (int64_t b0 = 0; b0 < n_p; b0 += P.batch) {
        const int64_t nb = std::min<int64_t>(P.batch, n_p - b0);
        lw_traj_t push = *t;
        push.n_particles = nb;
        push.init = t->init + 6 * b0;
        lw_status st = launch_boris_rmax2(&push, rb2, s);
        if (st != LW_OK) return st;
        for (int64_t s0 = 0;;) {
            const int64_t n_span = std::min<int64_t>(P.span, ns - s0);
            // the span's samples, the deposit adjoint over its intervals (dJ/d samples), then
            // the tangents of the same span contracted with them
            st = launch_boris_span(&push, s0, n_span, pstate, r, b, bd, s);
            if (st != LW_OK) return st;
            const int64_t nz = nb * n_span * 3;
            for (double *z : {gr_, gb, ga})
                k_zero<<<(int)std::min<int64_t>((nz + 255) / 256, 65536), 256, 0, s>>>(z, nz);
            lw_traj_t sub = *t;
            sub.kind = LW_TRAJ_SAMPLES;
            sub.span = 0;
            sub.n_particles = nb;
            sub.n_samples = n_span;
            sub.r = r;
            sub.beta = b;
            sub.beta_dot = bd;
            sub.init = nullptr;
            sub.charge = t->charge ? t->charge + b0 : nullptr;
            st = launch_deposit_bwd(&sub, gr, fmask, geom, dE, gr_, gb, ga, nullptr, 0, s, s0, rb2);
            if (st != LW_OK) return st;
            st = launch_boris_bwd_span(&push, s0, n_span, tstate, gr_, gb, ga, grad_init + 6 * b0, grad_a0 + b0, s);
            if (st != LW_OK) return st;
            if (s0 + n_span >= ns) break;
            s0 += n_span - 1;  // the next span starts at this span's last sample
        }
    }
    return check_launch("lw_deposit_td_bwd_boris");
}

}  // namespace lw
