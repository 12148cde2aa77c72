// FP64 Boris trajectories of electrons in the laser pulse (the trajectory source of
// the time-domain method; the paper integrates the equations of motion with the
// Boris method), and their forward-mode tangents with respect to the initial phase
// space and the laser amplitude a0.  One lane per particle; samples are
// r, beta, beta_dot [n_particles][n_samples][3].
#include "lw_internal.h"

#include <algorithm>

namespace lw {
namespace {

// ---- dual numbers: value and ND directional derivatives --------------------------------------
template <int ND>
struct Dual {
    double v;
    double d[ND];
    Dual() = default;
    __device__ __forceinline__ Dual(double x) : v(x)
    {
#pragma unroll
        for (int j = 0; j < ND; ++j) d[j] = 0.0;
    }
};
template <int ND>
__device__ __forceinline__ Dual<ND> operator+(Dual<ND> a, Dual<ND> b)
{
    Dual<ND> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int j = 0; j < ND; ++j) r.d[j] = a.d[j] + b.d[j];
    return r;
}
template <int ND>
__device__ __forceinline__ Dual<ND> operator-(Dual<ND> a, Dual<ND> b)
{
    Dual<ND> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int j = 0; j < ND; ++j) r.d[j] = a.d[j] - b.d[j];
    return r;
}
template <int ND>
__device__ __forceinline__ Dual<ND> operator-(Dual<ND> a)
{
    Dual<ND> r;
    r.v = -a.v;
#pragma unroll
    for (int j = 0; j < ND; ++j) r.d[j] = -a.d[j];
    return r;
}
template <int ND>
__device__ __forceinline__ Dual<ND> operator*(Dual<ND> a, Dual<ND> b)
{
    Dual<ND> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int j = 0; j < ND; ++j) r.d[j] = a.d[j] * b.v + a.v * b.d[j];
    return r;
}
template <int ND>
__device__ __forceinline__ Dual<ND> operator/(Dual<ND> a, Dual<ND> b)
{
    Dual<ND> r;
    r.v = a.v / b.v;
#pragma unroll
    for (int j = 0; j < ND; ++j) r.d[j] = (a.d[j] - r.v * b.d[j]) / b.v;
    return r;
}
template <int ND>
__device__ __forceinline__ Dual<ND> operator*(double a, Dual<ND> b)
{
    Dual<ND> r;
    r.v = a * b.v;
#pragma unroll
    for (int j = 0; j < ND; ++j) r.d[j] = a * b.d[j];
    return r;
}
template <int ND>
__device__ __forceinline__ Dual<ND> operator*(Dual<ND> b, double a)
{
    return a * b;
}
template <int ND>
__device__ __forceinline__ Dual<ND> operator/(Dual<ND> b, double a)
{
    Dual<ND> r;
    r.v = b.v / a;
#pragma unroll
    for (int j = 0; j < ND; ++j) r.d[j] = b.d[j] / a;
    return r;
}
template <int ND>
__device__ __forceinline__ Dual<ND> operator/(double a, Dual<ND> b)
{
    Dual<ND> r;
    r.v = a / b.v;
#pragma unroll
    for (int j = 0; j < ND; ++j) r.d[j] = -r.v * b.d[j] / b.v;
    return r;
}
template <int ND>
__device__ __forceinline__ Dual<ND> operator+(Dual<ND> a, double b)
{
    a.v += b;
    return a;
}
template <int ND>
__device__ __forceinline__ Dual<ND> operator+(double b, Dual<ND> a)
{
    a.v += b;
    return a;
}
template <int ND>
__device__ __forceinline__ Dual<ND> operator-(double b, Dual<ND> a)
{
    return b + (-a);
}
using ::exp;  // the double overloads stay visible beside the dual ones
using ::sincos;
using ::sqrt;
template <int ND>
__device__ __forceinline__ Dual<ND> sqrt(Dual<ND> a)
{
    Dual<ND> r;
    r.v = ::sqrt(a.v);
#pragma unroll
    for (int j = 0; j < ND; ++j) r.d[j] = a.d[j] / (2.0 * r.v);
    return r;
}
template <int ND>
__device__ __forceinline__ Dual<ND> exp(Dual<ND> a)
{
    Dual<ND> r;
    r.v = ::exp(a.v);
#pragma unroll
    for (int j = 0; j < ND; ++j) r.d[j] = a.d[j] * r.v;
    return r;
}
template <int ND>
__device__ __forceinline__ void sincos(Dual<ND> a, Dual<ND> *s, Dual<ND> *c)
{
    double sv, cv;
    ::sincos(a.v, &sv, &cv);
    s->v = sv;
    c->v = cv;
#pragma unroll
    for (int j = 0; j < ND; ++j) {
        s->d[j] = a.d[j] * cv;
        c->d[j] = -a.d[j] * sv;
    }
}
__device__ __forceinline__ double val(double a) { return a; }
template <int ND>
__device__ __forceinline__ double val(const Dual<ND> &a)
{
    return a.v;
}

// ---- the laser pulse and the pusher, written once for double and for dual numbers -----------
struct LaserDev {
    double a0, wl, w0, nc, e0_per_a0;  // wl = 2 pi c / lambda, E0 = a0 e0_per_a0, e0_per_a0 = m_e c wl / e
};

// Pulse written through its normalised vector potential a_x = a0 g(phi) sin(phi),
// g = cos^2(phi/(2 nc)) on |phi| < pi nc, phi = wl (t + z/c):
// E_x = -E0 T(rho) d(g sin)/dphi, B_y = -E_x / c, T = exp(-rho^2/w0^2) (w0 > 0).
template <typename R>
__device__ __forceinline__ void laser_eb(const LaserDev &L, R a0, R x, R y, R z, double t, R &Ex, R &By)
{
    const R phi = L.wl * (t + z / kC);
    Ex = 0.0;
    By = 0.0;
    if (!(fabs(val(phi)) < kPi * L.nc)) return;
    R sh, ch, sp, cp;
    sincos(phi / (2.0 * L.nc), &sh, &ch);
    sincos(phi, &sp, &cp);
    const R g = ch * ch;
    // g' = -sin(phi/nc)/(2 nc) = -sh ch / nc (double angle: one sin/cos pair fewer per step)
    const R gp = -((sh * ch) / L.nc);
    const R dS = gp * sp + g * cp;
    R T = 1.0;
    if (L.w0 > 0.0) T = exp(-((x * x + y * y) / (L.w0 * L.w0)));
    Ex = -(L.e0_per_a0 * (a0 * T * dS));
    By = -(Ex / kC);
}

// Boris update of u = gamma beta over time h for an electron, with E = (Ex,0,0), B = (0,By,0).
template <typename R>
__device__ __forceinline__ void kick(R &ux, R &uy, R &uz, R Ex, R By, double h)
{
    const double q = -kQe, m = kMe;
    const double a = q * h / (2.0 * m * kC);
    const R mx = ux + a * Ex, my = uy, mz = uz;
    const R gm = sqrt(1.0 + (mx * mx + my * my + mz * mz));
    const R ty = (q * h / (2.0 * m)) * By / gm;  // rotation vector (0, ty, 0)
    const R sy = 2.0 * ty / (1.0 + ty * ty);
    // u' = u- + u- x t ;  u+ = u- + u' x s
    const R px = mx - mz * ty, pz = mz + mx * ty;
    const R nx = mx - pz * sy, nz = mz + px * sy;
    ux = nx + a * Ex;
    uy = my;
    uz = nz;
}

// State of one particle's pusher at sample i: position, u = gamma beta at the sample time, u
// half a step later, and the field at (r_i, t_i).  The field is a function of the position and
// the time only, so a state saved without it and resumed at sample i recomputes it bit for bit.
template <typename R>
struct PushState {
    R x, y, z, usx, usy, usz, uhx, uhy, uhz, Ex, By;
};

template <typename R>
__device__ __forceinline__ void push_start(const LaserDev &L, R a0, const R *init, double t_start, double dt,
                                           PushState<R> &S)
{
    S.x = init[0];
    S.y = init[1];
    S.z = init[2];
    S.usx = init[3];
    S.usy = init[4];
    S.usz = init[5];
    S.uhx = S.usx;
    S.uhy = S.usy;
    S.uhz = S.usz;
    laser_eb(L, a0, S.x, S.y, S.z, t_start, S.Ex, S.By);
    kick(S.uhx, S.uhy, S.uhz, S.Ex, S.By, 0.5 * dt);
}

// r, beta and beta_dot of the sample the state stands at
template <typename R>
__device__ __forceinline__ void push_sample(const PushState<R> &S, R *rr, R *bb, R *aa)
{
    const double q = -kQe, m = kMe;
    const R g = sqrt(1.0 + (S.usx * S.usx + S.usy * S.usy + S.usz * S.usz));
    const R ig = 1.0 / g;  // one division for the four quotients by gamma
    const R bx = S.usx * ig, by = S.usy * ig, bz = S.usz * ig;
    // d beta/dt = q/(gamma m c) [E + c beta x B - beta (beta.E)],  E = (Ex,0,0), B = (0,By,0)
    const R f = (q / (m * kC)) * ig;
    const R be = bx * S.Ex;
    rr[0] = S.x;
    rr[1] = S.y;
    rr[2] = S.z;
    bb[0] = bx;
    bb[1] = by;
    bb[2] = bz;
    aa[0] = f * (S.Ex - kC * (bz * S.By) - bx * be);
    aa[1] = f * (-(by * be));
    aa[2] = f * (kC * (bx * S.By) - bz * be);
}

// one Boris step from sample i to sample i + 1 (t_next = t_start + (i + 1) dt)
template <typename R>
__device__ __forceinline__ void push_step(const LaserDev &L, R a0, double t_next, double dt, PushState<R> &S)
{
    const R gh = sqrt(1.0 + (S.uhx * S.uhx + S.uhy * S.uhy + S.uhz * S.uhz));
    const R cg = (kC * dt) / gh;  // c dt / gamma at the half step
    S.x = S.x + cg * S.uhx;
    S.y = S.y + cg * S.uhy;
    S.z = S.z + cg * S.uhz;
    R nx = S.uhx, ny = S.uhy, nz = S.uhz;
    // the field at (r_{i+1}, t_{i+1}) drives the kick and is the next sample's field
    laser_eb(L, a0, S.x, S.y, S.z, t_next, S.Ex, S.By);
    kick(nx, ny, nz, S.Ex, S.By, dt);
    S.usx = 0.5 * (S.uhx + nx);
    S.usy = 0.5 * (S.uhy + ny);
    S.usz = 0.5 * (S.uhz + nz);
    S.uhx = nx;
    S.uhy = ny;
    S.uhz = nz;
}

// Runs the pusher of one particle and calls emit(i, r[3], beta[3], beta_dot[3]) per sample.
template <typename R, typename Emit>
__device__ __forceinline__ void push_particle(const LaserDev &L, R a0, const R *init, int64_t n_samples,
                                              double t_start, double dt, Emit emit)
{
    PushState<R> S;
    push_start(L, a0, init, t_start, dt, S);
    for (int64_t i = 0; i < n_samples; ++i) {
        R rr[3], bb[3], aa[3];
        push_sample(S, rr, bb, aa);
        emit(i, rr, bb, aa);
        if (i + 1 == n_samples) break;
        push_step(L, a0, t_start + (double)(i + 1) * dt, dt, S);
    }
}

__global__ __launch_bounds__(256) void k_boris(const double *__restrict__ init, int64_t n_particles,
                                               int64_t n_samples, double t_start, double dt, LaserDev L,
                                               double *__restrict__ r, double *__restrict__ beta,
                                               double *__restrict__ beta_dot)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_particles) return;
    double in[6];
    for (int c = 0; c < 6; ++c) in[c] = init[6 * k + c];
    push_particle<double>(L, L.a0, in, n_samples, t_start, dt,
                          [&](int64_t i, const double *rr, const double *bb, const double *aa) {
                              const size_t o = (size_t)(k * n_samples + i) * 3;
                              for (int c = 0; c < 3; ++c) {
                                  r[o + c] = rr[c];
                                  beta[o + c] = bb[c];
                                  beta_dot[o + c] = aa[c];
                              }
                          });
}

// max_i |r_i|^2 over every sample of each particle's trajectory (nothing stored; the sum in the
// order of the deposit's pre-pass, z^2 + (y^2 + x^2) with fused multiply-adds), so that
// choices made per particle over its whole trajectory agree between the spans of a deposit
// and its adjoint and with those of the stored samples
__global__ __launch_bounds__(256) void k_boris_rmax2(const double *__restrict__ init, int64_t n_particles,
                                                     int64_t n_samples, double t_start, double dt, LaserDev L,
                                                     double *__restrict__ rmax2)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_particles) return;
    double in[6];
    for (int c = 0; c < 6; ++c) in[c] = init[6 * k + c];
    PushState<double> S;
    push_start(L, L.a0, in, t_start, dt, S);
    double mx = fma(S.z, S.z, fma(S.y, S.y, S.x * S.x));
    for (int64_t i = 1; i < n_samples; ++i) {
        push_step(L, L.a0, t_start + (double)i * dt, dt, S);
        mx = fmax(mx, fma(S.z, S.z, fma(S.y, S.y, S.x * S.x)));
    }
    rmax2[k] = mx;
}

// Samples s0 .. s0 + n_span - 1 of each particle into r, beta, beta_dot [n_particles][n_span][3].
// The pusher starts from init (s0 = 0) or from the state saved by the previous span, which ends
// at sample s0 (spans share their boundary sample), and saves its state at the last sample it
// writes: x, y, z, u at the sample and u half a step later, [n_particles][9].
constexpr int kStateDoubles = 9;

__global__ __launch_bounds__(256) void k_boris_span(const double *__restrict__ init, int64_t n_particles,
                                                    int64_t s0, int64_t n_span, double t_start, double dt,
                                                    LaserDev L, double *__restrict__ state, double *__restrict__ r,
                                                    double *__restrict__ beta, double *__restrict__ beta_dot)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_particles) return;
    PushState<double> S;
    double *st = state + kStateDoubles * k;
    if (s0 == 0) {
        double in[6];
        for (int c = 0; c < 6; ++c) in[c] = init[6 * k + c];
        push_start(L, L.a0, in, t_start, dt, S);
    } else {
        S.x = st[0];
        S.y = st[1];
        S.z = st[2];
        S.usx = st[3];
        S.usy = st[4];
        S.usz = st[5];
        S.uhx = st[6];
        S.uhy = st[7];
        S.uhz = st[8];
        // the same arguments as the step that reached sample s0: the same field
        laser_eb(L, L.a0, S.x, S.y, S.z, t_start + (double)s0 * dt, S.Ex, S.By);
    }
    for (int64_t j = 0; j < n_span; ++j) {
        double rr[3], bb[3], aa[3];
        push_sample(S, rr, bb, aa);
        const size_t o = (size_t)(k * n_span + j) * 3;
        for (int c = 0; c < 3; ++c) {
            r[o + c] = rr[c];
            beta[o + c] = bb[c];
            beta_dot[o + c] = aa[c];
        }
        if (j + 1 == n_span) break;
        push_step(L, L.a0, t_start + (double)(s0 + j + 1) * dt, dt, S);
    }
    st[0] = S.x;
    st[1] = S.y;
    st[2] = S.z;
    st[3] = S.usx;
    st[4] = S.usy;
    st[5] = S.usz;
    st[6] = S.uhx;
    st[7] = S.uhy;
    st[8] = S.uhz;
}

// Gradient through the pusher by forward-mode tangents: lane l handles particle k = l / 7
// and parameter p = l % 7 (init[k][0..5], then a0), runs the pusher in dual numbers seeded
// with d/dp = 1 and accumulates sum_i g_r.dr_i/dp + g_beta.dbeta_i/dp + g_bd.dbeta_dot_i/dp.
// Every trajectory depends only on its own initial condition and on a0, so these seven
// tangents per particle are the whole gradient.
constexpr int kParams = 7;

__global__ __launch_bounds__(64) void k_boris_tangent(const double *__restrict__ init, int64_t n_particles,
                                                      int64_t n_samples, double t_start, double dt, LaserDev L,
                                                      const double *__restrict__ g_r, const double *__restrict__ g_b,
                                                      const double *__restrict__ g_a, double *__restrict__ grad_init,
                                                      double *__restrict__ grad_a0)
{
    using D = Dual<1>;
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n_particles * kParams) return;
    const int64_t k = l / kParams;
    const int p = (int)(l - k * kParams);
    D in[6];
    for (int c = 0; c < 6; ++c) {
        in[c] = D(init[6 * k + c]);
        in[c].d[0] = (c == p) ? 1.0 : 0.0;
    }
    D a0(L.a0);
    a0.d[0] = (p == 6) ? 1.0 : 0.0;
    double acc = 0.0;
    push_particle<D>(L, a0, in, n_samples, t_start, dt, [&](int64_t i, const D *rr, const D *bb, const D *aa) {
        const size_t o = (size_t)(k * n_samples + i) * 3;
        for (int c = 0; c < 3; ++c) acc += g_r[o + c] * rr[c].d[0] + g_b[o + c] * bb[c].d[0] + g_a[o + c] * aa[c].d[0];
    });
    if (p < 6)
        grad_init[6 * k + p] = acc;
    else
        grad_a0[k] = acc;
}

// The tangents over samples s0 .. s0 + n_span - 1 only, kTanND of the seven per lane: lane l
// takes particle k = l / G and parameters p = kTanND (l % G) + j (j < kTanND, p < 7), G =
// ceil(7 / kTanND) lanes per particle, so each lane runs the pusher's values once for kTanND
// tangents (the laser's sin, cos and exp serve them all).  Each lane starts from its seeded
// initial state (s0 = 0) or from the dual-number state the previous span left at sample s0
// ([lane][9 (1 + kTanND)]: the 9 state values, then their derivatives), contracts the span's
// gradients g_* [n_particles][n_span][3], saves its state at the span's last sample, and writes
// (s0 = 0) or adds its sums.  Spans share their boundary sample; the gradients of a boundary
// sample are split between the two spans' deposit adjoints (each gathers its own intervals), so
// the two contractions add up to the whole.
// One tangent per lane: two or four per lane (values computed once for them) measured slower on
// the large workload's adjoint (444 and 448 against 326 ms): their registers (221, 324) leave
// fewer wavefronts to hide the pusher's serial chain of steps.
constexpr int kTanND = 1;
constexpr int kTanLanes = (kParams + kTanND - 1) / kTanND;          // lanes per particle
constexpr int kTanStateDoubles = 9 * (1 + kTanND);                  // per lane
static_assert(kTanLanes * kTanStateDoubles <= 7 * 18, "the workspace holds 126 doubles of state per particle");

__global__ __launch_bounds__(64) void k_boris_tangent_span(const double *__restrict__ init, int64_t n_particles,
                                                           int64_t s0, int64_t n_span, double t_start, double dt,
                                                           LaserDev L, double *__restrict__ tstate,
                                                           const double *__restrict__ g_r,
                                                           const double *__restrict__ g_b,
                                                           const double *__restrict__ g_a,
                                                           double *__restrict__ grad_init,
                                                           double *__restrict__ grad_a0)
{
    using D = Dual<kTanND>;
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= n_particles * kTanLanes) return;
    const int64_t k = l / kTanLanes;
    const int p0 = (int)(l - k * kTanLanes) * kTanND;  // parameters p0 .. p0 + kTanND - 1
    D a0(L.a0);
#pragma unroll
    for (int j = 0; j < kTanND; ++j) a0.d[j] = (p0 + j == 6) ? 1.0 : 0.0;
    PushState<D> S;
    double *st = tstate + kTanStateDoubles * l;
    if (s0 == 0) {
        D in[6];
        for (int c = 0; c < 6; ++c) {
            in[c] = D(init[6 * k + c]);
#pragma unroll
            for (int j = 0; j < kTanND; ++j) in[c].d[j] = (c == p0 + j) ? 1.0 : 0.0;
        }
        push_start(L, a0, in, t_start, dt, S);
    } else {
        D *f[9] = {&S.x, &S.y, &S.z, &S.usx, &S.usy, &S.usz, &S.uhx, &S.uhy, &S.uhz};
        for (int c = 0; c < 9; ++c) {
            f[c]->v = st[c];
#pragma unroll
            for (int j = 0; j < kTanND; ++j) f[c]->d[j] = st[9 + 9 * j + c];
        }
        // the same arguments as the step that reached sample s0: the same field and derivative
        laser_eb(L, a0, S.x, S.y, S.z, t_start + (double)s0 * dt, S.Ex, S.By);
    }
    double acc[kTanND];
#pragma unroll
    for (int j = 0; j < kTanND; ++j) acc[j] = 0.0;
    for (int64_t i = 0; i < n_span; ++i) {
        D rr[3], bb[3], aa[3];
        push_sample(S, rr, bb, aa);
        const size_t o = (size_t)(k * n_span + i) * 3;
        for (int c = 0; c < 3; ++c) {
            const double gr = g_r[o + c], gb = g_b[o + c], ga = g_a[o + c];
#pragma unroll
            for (int j = 0; j < kTanND; ++j) acc[j] += gr * rr[c].d[j] + gb * bb[c].d[j] + ga * aa[c].d[j];
        }
        if (i + 1 == n_span) break;
        push_step(L, a0, t_start + (double)(s0 + i + 1) * dt, dt, S);
    }
    {
        const D *f[9] = {&S.x, &S.y, &S.z, &S.usx, &S.usy, &S.usz, &S.uhx, &S.uhy, &S.uhz};
        for (int c = 0; c < 9; ++c) {
            st[c] = f[c]->v;
#pragma unroll
            for (int j = 0; j < kTanND; ++j) st[9 + 9 * j + c] = f[c]->d[j];
        }
    }
#pragma unroll
    for (int j = 0; j < kTanND; ++j) {
        const int p = p0 + j;
        if (p >= kParams) break;
        double *out = p < 6 ? grad_init + 6 * k + p : grad_a0 + k;
        *out = s0 == 0 ? acc[j] : *out + acc[j];
    }
}

LaserDev laser_dev(const lw_laser_t &l)
{
    LaserDev L;
    L.a0 = l.a0;
    L.wl = 2.0 * kPi * kC / l.lambda;
    L.w0 = l.w0;
    L.nc = l.n_cycles;
    L.e0_per_a0 = kMe * kC * L.wl / kQe;
    return L;
}

}  // namespace

lw_status launch_boris(const lw_traj_t *t, double *r, double *beta, double *beta_dot, hipStream_t s)
{
    if (t->n_particles == 0) return LW_OK;
    const LaserDev L = laser_dev(t->laser);
    const int64_t blocks = (t->n_particles + 63) / 64;
    k_boris<<<(unsigned)blocks, 64, 0, s>>>(t->init, t->n_particles, t->n_samples, t->t_start, t->dt, L, r, beta,
                                           beta_dot);
    return check_launch("lw_trajectory_boris");
}

lw_status launch_boris_rmax2(const lw_traj_t *t, double *rmax2, hipStream_t s)
{
    if (t->n_particles == 0) return LW_OK;
    const LaserDev L = laser_dev(t->laser);
    const int64_t blocks = (t->n_particles + 63) / 64;
    k_boris_rmax2<<<(unsigned)blocks, 64, 0, s>>>(t->init, t->n_particles, t->n_samples, t->t_start, t->dt, L, rmax2);
    return check_launch("max |r|^2 of the pushed trajectories");
}

lw_status launch_boris_span(const lw_traj_t *t, int64_t s0, int64_t n_span, double *state, double *r, double *beta,
                            double *beta_dot, hipStream_t s)
{
    if (t->n_particles == 0 || n_span == 0) return LW_OK;
    const LaserDev L = laser_dev(t->laser);
    const int64_t blocks = (t->n_particles + 63) / 64;
    k_boris_span<<<(unsigned)blocks, 64, 0, s>>>(t->init, t->n_particles, s0, n_span, t->t_start, t->dt, L, state, r,
                                                beta, beta_dot);
    return check_launch("lw_deposit_td (pusher span)");
}

lw_status launch_boris_bwd_span(const lw_traj_t *t, int64_t s0, int64_t n_span, double *tstate, const double *g_r,
                                const double *g_beta, const double *g_beta_dot, double *grad_init, double *grad_a0,
                                hipStream_t s)
{
    if (t->n_particles == 0 || n_span == 0) return LW_OK;
    const LaserDev L = laser_dev(t->laser);
    const int64_t lanes = t->n_particles * kTanLanes;
    const int64_t blocks = (lanes + 63) / 64;
    hipEvent_t ev = timing_begin(LW_KERNEL_BORIS_TANGENT, s);
    k_boris_tangent_span<<<(unsigned)blocks, 64, 0, s>>>(t->init, t->n_particles, s0, n_span, t->t_start, t->dt, L,
                                                        tstate, g_r, g_beta, g_beta_dot, grad_init, grad_a0);
    timing_end(LW_KERNEL_BORIS_TANGENT, ev, s);
    return check_launch("lw_deposit_td_bwd_boris (tangent span)");
}

lw_status launch_boris_bwd(const lw_traj_t *t, const double *g_r, const double *g_beta, const double *g_beta_dot,
                           double *grad_init, double *grad_a0, hipStream_t s)
{
    if (t->n_particles == 0) return LW_OK;
    const LaserDev L = laser_dev(t->laser);
    const int64_t lanes = t->n_particles * kParams;
    const int64_t blocks = (lanes + 63) / 64;
    k_boris_tangent<<<(unsigned)blocks, 64, 0, s>>>(t->init, t->n_particles, t->n_samples, t->t_start, t->dt, L, g_r,
                                                   g_beta, g_beta_dot, grad_init, grad_a0);
    return check_launch("lw_trajectory_boris_bwd");
}

}  // namespace lw
