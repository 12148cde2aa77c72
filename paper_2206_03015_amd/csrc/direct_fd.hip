// Direct frequency-domain sum (Eq. inty_dft, Algorithm 1), the comparison path.
//
// FP64 (k_direct_fd): a wavefront owns one pixel and 64 frequencies (one per lane) and a
// group of particles.  Per chunk of 64 samples every lane evaluates one sample (arrival
// time and E*kappa, the integrand of Eq. const_phase_drop) into LDS; then every lane sweeps
// the 64 staged samples for its own frequency, forming the phase w*(t_a - t0) in double per
// term and reducing it to one revolution before sin/cos.
//
// Mixed (k_direct_fd_mixed): lane l owns K consecutive frequencies (8, or fewer for short
// frequency lists).  Per chunk and
// lane the phase of the lane's first frequency at a reference arrival time of the chunk is
// formed in double (reduced to one revolution); per sample one float FMA adds nu*(t_a -
// t_ref), a few revolutions at most, and the hardware sin/cos (arguments in revolutions)
// give the first phasor.  When the wavefront's frequencies are equally spaced by dw (checked
// once per wavefront), the others follow by a recurrence over frequency: with the step
// phasor e^{i dw t_a} formed once per sample at staging (phase in double, reduced, then
// float sin/cos), p_1 = p_0 e^{i dw t} and p_{j+1} = 2 cos(dw t) p_j - p_{j-1}, two FMAs per
// further frequency instead of a sin/cos pair.  Otherwise every phasor gets its own sin/cos.
// Terms are summed in float over a chunk, chunks in double.
//
// Partial sums of a wavefront go to a double workspace with atomics; a final kernel forms
// S = (dt^2/2pi) sum_c |F_c|^2.
#include "lw_internal.h"

#include <algorithm>

namespace lw {
namespace {

constexpr int kWavesPerBlock = 4;

// value of lane src (wavefront-uniform src) of a double register
__device__ __forceinline__ double readlane_f64(double v, int src)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, src);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), src);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

struct FdShape {
    int64_t n_particles, n_samples, n_pix, n_omega;
    int64_t n_wblocks, n_groups, parts_per_group;
    double t_start, dt, t0, inv_cdt, cdt;
    int fmask;
};

// most frequencies per lane of the mixed kernel (fewer when there are few frequencies, so
// that the lanes stay busy), and how equal the spacing of a wavefront's frequencies must be
// (relative) for the recurrence over frequency
constexpr int kFdFreq = 8;
constexpr double kFdEqualTol = 1e-13;

// Arrival time relative to t0 (s) and E*kappa of sample i of particle k at pixel g; zeros for
// samples past the end, unusable samples and non-finite results.
template <typename T, int GEOM>
__device__ __forceinline__ void stage_sample(const double *__restrict__ r, const double *__restrict__ beta,
                                             const double *__restrict__ beta_dot, const PixGeo &g, const double *xm,
                                             double q, int64_t k, int64_t i, const FdShape &sh, double &ta, T &ex,
                                             T &ey, T &ez)
{
    ta = 0.0;
    ex = ey = ez = (T)0;
    if (i >= sh.n_samples || !g.ok) return;
    const size_t s = (size_t)(k * sh.n_samples + i) * 3;
    if (!sample_usable(r + s, beta + s, beta_dot + s)) return;
    double kap;
    lw_field<T, GEOM>(g, xm, r[s], r[s + 1], r[s + 2], beta[s], beta[s + 1], beta[s + 2], beta_dot[s], beta_dot[s + 1],
                      beta_dot[s + 2], q, sh.fmask, ex, ey, ez, &kap);
    // arrival time relative to t0 (s), formed in units of u = cdt / c (its compensated base d and
    // the pixel terms, as in the deposit)
    const double u = sh.cdt / kC;
    const double d = arrival_base(sh.t_start, sh.dt, (double)i, sh.t0, u, r[s + 2]);
    ta = arrival_tau<GEOM, kTauSqrt>(pix_const_of(g, sh.inv_cdt), d, r[s], r[s + 1], r[s + 2], 0.0, sh.inv_cdt) * u;
    const T tk = (T)kap;
    ex *= tk;
    ey *= tk;
    ez *= tk;
    if (!(isfinite(ta) && isfinite((double)ex) && isfinite((double)ey) && isfinite((double)ez))) {
        ta = 0.0;
        ex = ey = ez = (T)0;
    }
}

template <int GEOM>
__global__ __launch_bounds__(256) void k_direct_fd(const double *__restrict__ r, const double *__restrict__ beta,
                                                   const double *__restrict__ beta_dot,
                                                   const double *__restrict__ charge, const double *__restrict__ x_det,
                                                   const double *__restrict__ omega, double *__restrict__ acc,
                                                   FdShape sh)
{
    __shared__ double s_ta[kWavesPerBlock][64];
    __shared__ double s_ek[kWavesPerBlock][3][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + wv;
    const int64_t per_pix = sh.n_wblocks * sh.n_groups;
    const int64_t m = wave / per_pix;
    if (m >= sh.n_pix) return;  // whole wavefront idle; no block-level sync below
    const int64_t rem = wave - m * per_pix;
    const int64_t wb = rem / sh.n_groups, grp = rem - wb * sh.n_groups;
    const int64_t w = wb * 64 + lane;
    const bool w_ok = w < sh.n_omega;
    const double nu = w_ok ? omega[w] / (2.0 * kPi) : 0.0;  // cycles per second
    const int64_t k0 = grp * sh.parts_per_group, k1 = std::min(k0 + sh.parts_per_group, sh.n_particles);
    PixGeo g = pix_geo(x_det, m);
    const double *xm = x_det + 3 * m;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0, a4 = 0, a5 = 0;  // Re/Im of F_x, F_y, F_z
    const int64_t ns = sh.n_samples;
    for (int64_t k = k0; k < k1; ++k) {
        const double q = charge ? charge[k] : -kQe;
        for (int64_t i0 = 0; i0 < ns; i0 += 64) {
            // stage: lane -> sample i0 + lane
            {
                double ta = 0.0, ex = 0, ey = 0, ez = 0;
                stage_sample<double, GEOM>(r, beta, beta_dot, g, xm, q, k, i0 + lane, sh, ta, ex, ey, ez);
                s_ta[wv][lane] = ta;
                s_ek[wv][0][lane] = ex;
                s_ek[wv][1][lane] = ey;
                s_ek[wv][2][lane] = ez;
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            const int cnt = (int)std::min<int64_t>(64, ns - i0);
            double b0 = 0, b1 = 0, b2 = 0, b3 = 0, b4 = 0, b5 = 0;
            for (int j = 0; j < cnt; ++j) {
                const double x = nu * s_ta[wv][j];
                const double fr = x - floor(x);  // revolutions in [0, 1)
                double sn, c;
                sincospi(2.0 * fr, &sn, &c);
                const double e0 = s_ek[wv][0][j], e1 = s_ek[wv][1][j], e2 = s_ek[wv][2][j];
                b0 += e0 * c;
                b1 += e0 * sn;
                b2 += e1 * c;
                b3 += e1 * sn;
                b4 += e2 * c;
                b5 += e2 * sn;
            }
            a0 += b0;
            a1 += b1;
            a2 += b2;
            a3 += b3;
            a4 += b4;
            a5 += b5;
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (w_ok && k1 > k0) {
        double *o = acc + ((size_t)m * sh.n_omega + w) * 6;
        atomicAdd(o + 0, a0);
        atomicAdd(o + 1, a1);
        atomicAdd(o + 2, a2);
        atomicAdd(o + 3, a3);
        atomicAdd(o + 4, a4);
        atomicAdd(o + 5, a5);
    }
}

template <int GEOM, int K>
__global__ __launch_bounds__(256) void k_direct_fd_mixed(const double *__restrict__ r,
                                                         const double *__restrict__ beta,
                                                         const double *__restrict__ beta_dot,
                                                         const double *__restrict__ charge,
                                                         const double *__restrict__ x_det,
                                                         const double *__restrict__ omega, double *__restrict__ acc,
                                                         FdShape sh)
{
    __shared__ double s_tref[kWavesPerBlock];
    __shared__ float s_dtf[kWavesPerBlock][64];     // t_a - t_ref (s)
    __shared__ float2 s_step[kWavesPerBlock][64];   // e^{i dw t_a}
    __shared__ float s_ek[kWavesPerBlock][3][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + wv;
    const int64_t per_pix = sh.n_wblocks * sh.n_groups;
    const int64_t m = wave / per_pix;
    if (m >= sh.n_pix) return;  // whole wavefront idle; no block-level sync below
    const int64_t rem = wave - m * per_pix;
    const int64_t wb = rem / sh.n_groups, grp = rem - wb * sh.n_groups;
    const int64_t wfirst = wb * 64 * K, wl = wfirst + (int64_t)lane * K;
    // frequencies in cycles per second; the wavefront's spacing from its first two
    double nu[K];
#pragma unroll
    for (int j = 0; j < K; ++j) nu[j] = wl + j < sh.n_omega ? omega[wl + j] / (2.0 * kPi) : 0.0;
    const double nu_a = omega[wfirst] / (2.0 * kPi);
    const double dnu = wfirst + 1 < sh.n_omega ? omega[wfirst + 1] / (2.0 * kPi) - nu_a : 0.0;
    bool lane_eq = true;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const double pred = nu[0] + (double)j * dnu;
        if (wl + j < sh.n_omega) lane_eq &= fabs(nu[j] - pred) <= kFdEqualTol * fabs(nu[j]);
    }
    const bool equal = __ballot(!lane_eq) == 0;  // wavefront-uniform
    const int64_t k0 = grp * sh.parts_per_group, k1 = std::min(k0 + sh.parts_per_group, sh.n_particles);
    PixGeo g = pix_geo(x_det, m);
    const double *xm = x_det + 3 * m;
    double a[K][6];
#pragma unroll
    for (int j = 0; j < K; ++j)
#pragma unroll
        for (int c = 0; c < 6; ++c) a[j][c] = 0.0;
    const int64_t ns = sh.n_samples;
    for (int64_t k = k0; k < k1; ++k) {
        const double q = charge ? charge[k] : -kQe;
        for (int64_t i0 = 0; i0 < ns; i0 += 64) {
            // stage: lane -> sample i0 + lane
            {
                double ta = 0.0;
                float ex = 0, ey = 0, ez = 0;
                stage_sample<float, GEOM>(r, beta, beta_dot, g, xm, q, k, i0 + lane, sh, ta, ex, ey, ez);
                const bool live = ex != 0.0f || ey != 0.0f || ez != 0.0f;
                // reference arrival time: the first lane with a contribution
                const uint64_t lm = __ballot(live);
                const double tref = lm ? readlane_f64(ta, (int)__builtin_ctzll(lm)) : 0.0;
                s_dtf[wv][lane] = live ? (float)(ta - tref) : 0.0f;
                if (lane == 0) s_tref[wv] = tref;
                float2 st = make_float2(1.0f, 0.0f);
                if (equal && live) {
                    const double x = dnu * ta;
                    const float fr = (float)(x - floor(x));  // revolutions in [0, 1)
                    st = make_float2(__builtin_amdgcn_cosf(fr), __builtin_amdgcn_sinf(fr));
                }
                s_step[wv][lane] = st;
                s_ek[wv][0][lane] = ex;
                s_ek[wv][1][lane] = ey;
                s_ek[wv][2][lane] = ez;
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            const int cnt = (int)std::min<int64_t>(64, ns - i0);
            const double tref = s_tref[wv];
            float b[K][6];
#pragma unroll
            for (int j = 0; j < K; ++j)
#pragma unroll
                for (int c = 0; c < 6; ++c) b[j][c] = 0.0f;
            if (equal) {
                const double x = nu[0] * tref;
                const float base = (float)(x - floor(x));  // revolutions in [0, 1)
                const float nuf = (float)nu[0];
                for (int s = 0; s < cnt; ++s) {
                    const float ph = fmaf(nuf, s_dtf[wv][s], base);
                    // phasors p_j = e^{i(w_0 + j dw)t}: p_1 = p_0 e^{i dw t}, then the two-term
                    // recurrence p_{j+1} = 2 cos(dw t) p_j - p_{j-1} (two FMAs per frequency)
                    float c = __builtin_amdgcn_cosf(ph), sn = __builtin_amdgcn_sinf(ph);
                    const float e0 = s_ek[wv][0][s], e1 = s_ek[wv][1][s], e2 = s_ek[wv][2][s];
                    const float2 st = s_step[wv][s];
                    const float tc = st.x + st.x;
                    float cp = 0.0f, sp = 0.0f;
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        b[j][0] = fmaf(e0, c, b[j][0]);
                        b[j][1] = fmaf(e0, sn, b[j][1]);
                        b[j][2] = fmaf(e1, c, b[j][2]);
                        b[j][3] = fmaf(e1, sn, b[j][3]);
                        b[j][4] = fmaf(e2, c, b[j][4]);
                        b[j][5] = fmaf(e2, sn, b[j][5]);
                        if (j == 0 && K > 1) {
                            cp = c;
                            sp = sn;
                            c = fmaf(cp, st.x, -sp * st.y);
                            sn = fmaf(cp, st.y, sp * st.x);
                        } else if (j + 1 < K) {
                            const float cn = fmaf(tc, c, -cp), sn2 = fmaf(tc, sn, -sp);
                            cp = c;
                            sp = sn;
                            c = cn;
                            sn = sn2;
                        }
                    }
                }
            } else {
                float base[K], nuf[K];
#pragma unroll
                for (int j = 0; j < K; ++j) {
                    const double x = nu[j] * tref;
                    base[j] = (float)(x - floor(x));
                    nuf[j] = (float)nu[j];
                }
                for (int s = 0; s < cnt; ++s) {
                    const float dtf = s_dtf[wv][s];
                    const float e0 = s_ek[wv][0][s], e1 = s_ek[wv][1][s], e2 = s_ek[wv][2][s];
#pragma unroll
                    for (int j = 0; j < K; ++j) {
                        const float ph = fmaf(nuf[j], dtf, base[j]);
                        const float c = __builtin_amdgcn_cosf(ph), sn = __builtin_amdgcn_sinf(ph);
                        b[j][0] = fmaf(e0, c, b[j][0]);
                        b[j][1] = fmaf(e0, sn, b[j][1]);
                        b[j][2] = fmaf(e1, c, b[j][2]);
                        b[j][3] = fmaf(e1, sn, b[j][3]);
                        b[j][4] = fmaf(e2, c, b[j][4]);
                        b[j][5] = fmaf(e2, sn, b[j][5]);
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < K; ++j)
#pragma unroll
                for (int c = 0; c < 6; ++c) a[j][c] += (double)b[j][c];
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (k1 > k0) {
#pragma unroll
        for (int j = 0; j < K; ++j) {
            if (wl + j >= sh.n_omega) continue;
            double *o = acc + ((size_t)m * sh.n_omega + wl + j) * 6;
#pragma unroll
            for (int c = 0; c < 6; ++c) atomicAdd(o + c, a[j][c]);
        }
    }
}

__global__ void k_fd_zero(double *__restrict__ p, int64_t n)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        p[j] = 0.0;
}

__global__ void k_fd_finish(const double *__restrict__ acc, double *__restrict__ S, int64_t n, double f)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x) {
        const double *a = acc + 6 * j;
        S[j] = f * (a[0] * a[0] + a[1] * a[1] + a[2] * a[2] + a[3] * a[3] + a[4] * a[4] + a[5] * a[5]);
    }
}

// Adjoint of the direct sum for FP64 inputs: with R_c, I_c the real and imaginary parts of the
// forward sum F_c(w) (recomputed into acc) and A = E kappa, t = t_i + shift - t0 per (sample, pixel),
//   dJ/dA_c = 2f sum_w dS(w) (R_c cos wt + I_c sin wt),
//   dJ/dt   = 2f sum_w dS(w) w sum_c A_c (I_c cos wt - R_c sin wt),       f = dt^2 / 2pi,
// then dJ/dE = kappa dJ/dA, dJ/dkappa = E.dJ/dA through lw_field_vjp, and dt/dr = -n/c.
// A wavefront owns 64 consecutive samples of one particle (one per lane) and loops over every
// pixel; the frequencies are staged 64 at a time in LDS.  Each sample is owned by one lane, so
// the gradient is added without atomics.
template <int GEOM>
__global__ __launch_bounds__(256) void k_direct_fd_bwd(const double *__restrict__ r, const double *__restrict__ beta,
                                                       const double *__restrict__ beta_dot,
                                                       const double *__restrict__ charge,
                                                       const double *__restrict__ x_det,
                                                       const double *__restrict__ omega,
                                                       const double *__restrict__ acc, const double *__restrict__ dS,
                                                       double *__restrict__ d_r, double *__restrict__ d_beta,
                                                       double *__restrict__ d_beta_dot, FdShape sh, double two_f)
{
    __shared__ double s_w[kWavesPerBlock][64][8];  // dS, w dS, R_x, I_x, R_y, I_y, R_z, I_z
    __shared__ double s_nu[kWavesPerBlock][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + wv;
    const int64_t n_chunks = (sh.n_samples + 63) / 64;
    const int64_t k = wave / n_chunks;
    if (k >= sh.n_particles) return;  // whole wavefront idle; no block-level sync below
    const int64_t i = (wave - k * n_chunks) * 64 + lane;
    const bool in = i < sh.n_samples;
    const size_t s = (size_t)(k * sh.n_samples + (in ? i : 0)) * 3;
    double rs[3], bs[3], as[3];
    for (int c = 0; c < 3; ++c) {
        rs[c] = r[s + c];
        bs[c] = beta[s + c];
        as[c] = beta_dot[s + c];
    }
    const bool usable = in && sample_usable(rs, bs, as);
    const double q = charge ? charge[k] : -kQe;
    const double u = sh.cdt / kC;
    const double d = arrival_base(sh.t_start, sh.dt, (double)i, sh.t0, u, rs[2]);
    double gr[3] = {0, 0, 0}, gb[3] = {0, 0, 0}, ga[3] = {0, 0, 0};
    for (int64_t m = 0; m < sh.n_pix; ++m) {
        const PixGeo g = pix_geo(x_det, m);
        const double *xm = x_det + 3 * m;
        bool ok = usable && g.ok;
        double ta = 0.0, kap = 0.0, E[3] = {0, 0, 0}, A[3] = {0, 0, 0};
        if (ok) {
            lw_field<double, GEOM>(g, xm, rs[0], rs[1], rs[2], bs[0], bs[1], bs[2], as[0], as[1], as[2], q, sh.fmask,
                                   E[0], E[1], E[2], &kap);
            ta = arrival_tau<GEOM, kTauSqrt>(pix_const_of(g, sh.inv_cdt), d, rs[0], rs[1], rs[2], 0.0, sh.inv_cdt) * u;
            for (int c = 0; c < 3; ++c) A[c] = E[c] * kap;
            ok = isfinite(ta) && isfinite(A[0]) && isfinite(A[1]) && isfinite(A[2]);
        }
        double G[3] = {0, 0, 0}, K[3] = {0, 0, 0};
        for (int64_t w0 = 0; w0 < sh.n_omega; w0 += 64) {
            {
                const int64_t w = w0 + lane;
                double *row = s_w[wv][lane];
                if (w < sh.n_omega) {
                    const double *f = acc + ((size_t)m * sh.n_omega + w) * 6;
                    const double d = dS[(size_t)m * sh.n_omega + w];
                    s_nu[wv][lane] = omega[w] / (2.0 * kPi);
                    row[0] = d;
                    row[1] = d * omega[w];
                    for (int c = 0; c < 6; ++c) row[2 + c] = f[c];
                } else {
                    s_nu[wv][lane] = 0.0;
                    for (int c = 0; c < 8; ++c) row[c] = 0.0;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            const int cnt = (int)std::min<int64_t>(64, sh.n_omega - w0);
            if (ok) {
                for (int j = 0; j < cnt; ++j) {
                    const double x = s_nu[wv][j] * ta;
                    double sn, cs;
                    sincospi(2.0 * (x - floor(x)), &sn, &cs);
                    const double *row = s_w[wv][j];
                    for (int c = 0; c < 3; ++c) {
                        const double Rc = row[2 + 2 * c], Ic = row[3 + 2 * c];
                        G[c] = fma(row[0], fma(Rc, cs, Ic * sn), G[c]);
                        K[c] = fma(row[1], fma(Ic, cs, -Rc * sn), K[c]);
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (ok) {
            double gE[3], gk = 0.0, H = 0.0;
            for (int c = 0; c < 3; ++c) {
                G[c] *= two_f;
                gE[c] = kap * G[c];
                gk = fma(E[c], G[c], gk);
                H = fma(A[c], two_f * K[c], H);
            }
            lw_field_vjp<GEOM>(g, xm, rs, bs, as, q, sh.fmask, gE, gr, gb, ga, gk);
            // t = t_i + (|x - r| - |x|)/c - t0 (exact) or t_i - n.r/c - t0 (far field): dt/dr = -n/c
            double n[3] = {g.nx, g.ny, g.nz};
            if (GEOM == LW_GEOM_EXACT) {
                const double d0 = xm[0] - rs[0], d1 = xm[1] - rs[1], d2 = xm[2] - rs[2];
                const double R = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                n[0] = d0 / R;
                n[1] = d1 / R;
                n[2] = d2 / R;
            }
            for (int c = 0; c < 3; ++c) gr[c] -= H * n[c] / kC;
        }
    }
    if (in) {
        for (int c = 0; c < 3; ++c) {
            d_r[s + c] += gr[c];
            d_beta[s + c] += gb[c];
            d_beta_dot[s + c] += ga[c];
        }
    }
}

}  // namespace

size_t direct_fd_ws_bytes(int64_t n_pix, int64_t n_omega)
{
    return (size_t)std::max<int64_t>(n_pix * n_omega, 1) * 6 * sizeof(double);
}

lw_status launch_direct_fd(const lw_traj_t *t, const lw_grid_t *gr, const double *omega, int64_t n_omega, int prec,
                           int fmask, int geom, double *S, void *ws, size_t ws_bytes, hipStream_t s)
{
    const int64_t n_pix = gr->n_pix;
    const int64_t nS = n_pix * n_omega;
    if (nS == 0) return LW_OK;
    double *acc = (double *)ws;
    k_fd_zero<<<(int)std::min<int64_t>((6 * nS + 255) / 256, 65536), 256, 0, s>>>(acc, 6 * nS);
    FdShape sh;
    sh.n_particles = t->n_particles;
    sh.n_samples = t->n_samples;
    sh.n_pix = n_pix;
    sh.n_omega = n_omega;
    // frequencies per lane (mixed): the largest power of two <= kFdFreq that still fills a wavefront
    int K = 1;
    while (K < kFdFreq && 64 * 2 * K <= n_omega) K *= 2;
    const int64_t per_wave = prec == LW_PREC_FP64 ? 64 : 64 * K;  // frequencies per wavefront
    sh.n_wblocks = (n_omega + per_wave - 1) / per_wave;
    const int64_t base = n_pix * sh.n_wblocks;
    int64_t groups = std::max<int64_t>(1, (8192 + base - 1) / base);
    groups = std::min<int64_t>(groups, std::max<int64_t>(t->n_particles, 1));
    sh.parts_per_group = (std::max<int64_t>(t->n_particles, 1) + groups - 1) / groups;
    sh.n_groups = (std::max<int64_t>(t->n_particles, 1) + sh.parts_per_group - 1) / sh.parts_per_group;
    sh.t_start = t->t_start;
    sh.dt = t->dt;
    sh.t0 = gr->t0;
    // any positive grid step gives the same arrival times; use dt (the grid of this call is irrelevant)
    const double dts = t->dt;
    sh.cdt = kC * dts;
    sh.inv_cdt = 1.0 / sh.cdt;
    sh.fmask = fmask;
    if (t->n_particles > 0) {
        const int64_t waves = base * sh.n_groups;
        const int64_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
        if (blocks > 0x7fffffff) return fail(LW_E_SHAPE, "lw_direct_fd: problem too large for one launch");
        if (prec == LW_PREC_FP64) {
            if (geom == LW_GEOM_EXACT)
                k_direct_fd<LW_GEOM_EXACT><<<(unsigned)blocks, 256, 0, s>>>(
                    t->r, t->beta, t->beta_dot, t->charge, gr->x_det, omega, acc, sh);
            else
                k_direct_fd<LW_GEOM_FARFIELD><<<(unsigned)blocks, 256, 0, s>>>(
                    t->r, t->beta, t->beta_dot, t->charge, gr->x_det, omega, acc, sh);
        } else {
#define LW_FD_MIXED(G, KK)                                                                                        \
    k_direct_fd_mixed<G, KK><<<(unsigned)blocks, 256, 0, s>>>(t->r, t->beta, t->beta_dot, t->charge, gr->x_det, omega, \
                                                               acc, sh)
            if (geom == LW_GEOM_EXACT) {
                if (K == 8) LW_FD_MIXED(LW_GEOM_EXACT, 8);
                else if (K == 4) LW_FD_MIXED(LW_GEOM_EXACT, 4);
                else if (K == 2) LW_FD_MIXED(LW_GEOM_EXACT, 2);
                else LW_FD_MIXED(LW_GEOM_EXACT, 1);
            } else {
                if (K == 8) LW_FD_MIXED(LW_GEOM_FARFIELD, 8);
                else if (K == 4) LW_FD_MIXED(LW_GEOM_FARFIELD, 4);
                else if (K == 2) LW_FD_MIXED(LW_GEOM_FARFIELD, 2);
                else LW_FD_MIXED(LW_GEOM_FARFIELD, 1);
            }
#undef LW_FD_MIXED
        }
    }
    const double f = t->dt * t->dt / (2.0 * kPi);
    k_fd_finish<<<(int)std::min<int64_t>((nS + 255) / 256, 65536), 256, 0, s>>>(acc, S, nS, f);
    return check_launch("lw_direct_fd");
}

lw_status launch_direct_fd_bwd(const lw_traj_t *t, const lw_grid_t *gr, const double *omega, int64_t n_omega,
                               int fmask, int geom, const double *dS, double *d_r, double *d_beta, double *d_beta_dot,
                               void *ws, size_t ws_bytes, hipStream_t s)
{
    const int64_t n_pix = gr->n_pix;
    if (n_pix == 0 || n_omega == 0 || t->n_particles == 0) return LW_OK;
    // forward sums F_c(w) in FP64 into the workspace (the |F|^2 pass is not needed)
    double *acc = (double *)ws;
    const int64_t nS = n_pix * n_omega;
    k_fd_zero<<<(int)std::min<int64_t>((6 * nS + 255) / 256, 65536), 256, 0, s>>>(acc, 6 * nS);
    FdShape sh;
    sh.n_particles = t->n_particles;
    sh.n_samples = t->n_samples;
    sh.n_pix = n_pix;
    sh.n_omega = n_omega;
    sh.n_wblocks = (n_omega + 63) / 64;
    const int64_t base = n_pix * sh.n_wblocks;
    int64_t groups = std::max<int64_t>(1, (8192 + base - 1) / base);
    groups = std::min<int64_t>(groups, t->n_particles);
    sh.parts_per_group = (t->n_particles + groups - 1) / groups;
    sh.n_groups = (t->n_particles + sh.parts_per_group - 1) / sh.parts_per_group;
    sh.t_start = t->t_start;
    sh.dt = t->dt;
    sh.t0 = gr->t0;
    sh.cdt = kC * t->dt;
    sh.inv_cdt = 1.0 / sh.cdt;
    sh.fmask = fmask;
    {
        const int64_t waves = base * sh.n_groups;
        const int64_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
        if (blocks > 0x7fffffff) return fail(LW_E_SHAPE, "lw_direct_fd_bwd: problem too large for one launch");
        if (geom == LW_GEOM_EXACT)
            k_direct_fd<LW_GEOM_EXACT><<<(unsigned)blocks, 256, 0, s>>>(t->r, t->beta, t->beta_dot, t->charge,
                                                                              gr->x_det, omega, acc, sh);
        else
            k_direct_fd<LW_GEOM_FARFIELD><<<(unsigned)blocks, 256, 0, s>>>(
                t->r, t->beta, t->beta_dot, t->charge, gr->x_det, omega, acc, sh);
    }
    {
        const int64_t waves = t->n_particles * ((t->n_samples + 63) / 64);
        const int64_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
        if (blocks > 0x7fffffff) return fail(LW_E_SHAPE, "lw_direct_fd_bwd: problem too large for one launch");
        const double two_f = 2.0 * t->dt * t->dt / (2.0 * kPi);
        if (geom == LW_GEOM_EXACT)
            k_direct_fd_bwd<LW_GEOM_EXACT><<<(unsigned)blocks, 256, 0, s>>>(t->r, t->beta, t->beta_dot, t->charge,
                                                                         gr->x_det, omega, acc, dS, d_r, d_beta,
                                                                         d_beta_dot, sh, two_f);
        else
            k_direct_fd_bwd<LW_GEOM_FARFIELD><<<(unsigned)blocks, 256, 0, s>>>(t->r, t->beta, t->beta_dot, t->charge,
                                                                            gr->x_det, omega, acc, dS, d_r, d_beta,
                                                                            d_beta_dot, sh, two_f);
    }
    return check_launch("lw_direct_fd_bwd");
}

}  // namespace lw
