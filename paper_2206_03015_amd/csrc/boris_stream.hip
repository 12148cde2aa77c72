// Deposit and its adjoint for trajectories given as initial conditions plus a laser pulse
// (LW_TRAJ_BORIS): the FP64 Boris pusher recomputes the samples batch by batch of particles
// inside the library, so the whole trajectory set is never stored (the paper's time-domain
// method with the trajectory update inside the particle loop).  Each batch is pushed into
// the workspace, deposited (accumulating after the first batch) and discarded.
#include "lw_internal.h"

#include <algorithm>

namespace lw {
namespace {

// default trajectory batch (all three arrays): the pusher runs one lane per particle through
// every step, so a batch must hold enough particles to occupy the GPU (16 GiB: ~12k particles
// at 2e4 steps)
constexpr size_t kBatchBytes = size_t(16) << 30;

inline size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// bytes of one particle's batch buffers: `arrays` sample arrays of [n_samples][3] doubles
inline size_t per_particle(int64_t ns, int arrays) { return align256((size_t)ns * 3 * sizeof(double)) * arrays; }

__global__ void k_zero(double *__restrict__ p, int64_t n)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        p[j] = 0.0;
}

}  // namespace

int64_t boris_batch_default(int64_t n_p, int64_t ns, int arrays)
{
    const int64_t b = (int64_t)(kBatchBytes / per_particle(ns, arrays));
    return std::max<int64_t>(1, std::min<int64_t>(n_p, b));
}

size_t boris_stream_ws_bytes(int64_t n_p, int64_t ns, int64_t batch, int arrays)
{
    const size_t dep = arrays == 3 ? deposit_ws_bytes(batch, ns) : 0;
    return align256(dep) + (size_t)batch * per_particle(ns, arrays);
}

// largest batch that fits ws_bytes (0 if none does)
int64_t boris_batch_fit(int64_t n_p, int64_t ns, size_t ws_bytes, int arrays)
{
    int64_t b = boris_batch_default(n_p, ns, arrays);
    while (b > 0 && boris_stream_ws_bytes(n_p, ns, b, arrays) > ws_bytes) {
        const size_t pp = per_particle(ns, arrays);
        const size_t fixed = boris_stream_ws_bytes(n_p, ns, 0, arrays) + 4096;
        const int64_t guess = ws_bytes > fixed ? (int64_t)((ws_bytes - fixed) / (pp + 64)) : 0;
        b = std::min<int64_t>(b - 1, guess);
    }
    return std::max<int64_t>(b, 0);
}

lw_status launch_deposit_boris(const lw_traj_t *t, const lw_grid_t *gr, int prec, int fmask, int geom,
                               bool accumulate, void *E, int64_t *diag, void *ws, size_t ws_bytes, hipStream_t s)
{
    const int64_t n_p = t->n_particles, ns = t->n_samples;
    if (n_p == 0 || gr->n_pix == 0) {  // nothing to push: only the trace and diag reset of the plain call
        lw_traj_t sub = *t;
        sub.kind = LW_TRAJ_SAMPLES;
        sub.n_particles = 0;
        sub.r = sub.beta = sub.beta_dot = nullptr;
        return launch_deposit(&sub, gr, prec, fmask, geom, accumulate, E, diag, ws, ws_bytes, s);
    }
    const int64_t B = boris_batch_fit(n_p, ns, ws_bytes, 3);
    if (B < 1) return fail(LW_E_WORKSPACE, "lw_deposit_td: workspace holds no trajectory batch");
    const size_t dep_bytes = align256(deposit_ws_bytes(B, ns));
    char *p = (char *)ws + dep_bytes;
    const size_t arr = align256((size_t)ns * 3 * sizeof(double)) * (size_t)B;
    double *r = (double *)p, *b = (double *)(p + arr), *bd = (double *)(p + 2 * arr);
    for (int64_t b0 = 0; b0 < n_p; b0 += B) {
        const int64_t nb = std::min<int64_t>(B, n_p - b0);
        lw_traj_t push = *t;
        push.n_particles = nb;
        push.init = t->init + 6 * b0;
        lw_status st = launch_boris(&push, r, b, bd, s);
        if (st != LW_OK) return st;
        lw_traj_t sub = *t;
        sub.kind = LW_TRAJ_SAMPLES;
        sub.n_particles = nb;
        sub.r = r;
        sub.beta = b;
        sub.beta_dot = bd;
        sub.init = nullptr;
        sub.charge = t->charge ? t->charge + b0 : nullptr;
        st = launch_deposit(&sub, gr, prec, fmask, geom, accumulate || b0 > 0, E, diag, ws, dep_bytes, s);
        if (st != LW_OK) return st;
    }
    return LW_OK;
}

lw_status launch_deposit_bwd_boris(const lw_traj_t *t, const lw_grid_t *gr, int fmask, int geom, const double *dE,
                                   double *grad_init, double *grad_a0, void *ws, size_t ws_bytes, hipStream_t s)
{
    const int64_t n_p = t->n_particles, ns = t->n_samples;
    if (n_p == 0) return LW_OK;
    if (gr->n_pix == 0) {  // no pixels: the gradient is zero
        k_zero<<<(int)std::min<int64_t>((6 * n_p + 255) / 256, 65536), 256, 0, s>>>(grad_init, 6 * n_p);
        k_zero<<<(int)std::min<int64_t>((n_p + 255) / 256, 65536), 256, 0, s>>>(grad_a0, n_p);
        return check_launch("lw_deposit_td_bwd_boris");
    }
    const int64_t B = boris_batch_fit(n_p, ns, ws_bytes, 6);
    if (B < 1) return fail(LW_E_WORKSPACE, "lw_deposit_td_bwd_boris: workspace holds no trajectory batch");
    const size_t arr = align256((size_t)ns * 3 * sizeof(double)) * (size_t)B;
    char *p = (char *)ws;
    double *r = (double *)p, *b = (double *)(p + arr), *bd = (double *)(p + 2 * arr);
    double *gr_ = (double *)(p + 3 * arr), *gb = (double *)(p + 4 * arr), *ga = (double *)(p + 5 * arr);
    for (int64_t b0 = 0; b0 < n_p; b0 += B) {
        const int64_t nb = std::min<int64_t>(B, n_p - b0);
        lw_traj_t push = *t;
        push.n_particles = nb;
        push.init = t->init + 6 * b0;
        lw_status st = launch_boris(&push, r, b, bd, s);
        if (st != LW_OK) return st;
        const int64_t nz = nb * ns * 3;
        for (double *z : {gr_, gb, ga})
            k_zero<<<(int)std::min<int64_t>((nz + 255) / 256, 65536), 256, 0, s>>>(z, nz);
        lw_traj_t sub = *t;
        sub.kind = LW_TRAJ_SAMPLES;
        sub.n_particles = nb;
        sub.r = r;
        sub.beta = b;
        sub.beta_dot = bd;
        sub.init = nullptr;
        sub.charge = t->charge ? t->charge + b0 : nullptr;
        st = launch_deposit_bwd(&sub, gr, fmask, geom, dE, gr_, gb, ga, s);
        if (st != LW_OK) return st;
        st = launch_boris_bwd(&push, gr_, gb, ga, grad_init + 6 * b0, grad_a0 + b0, s);
        if (st != LW_OK) return st;
    }
    return check_launch("lw_deposit_td_bwd_boris");
}

}  // namespace lw
