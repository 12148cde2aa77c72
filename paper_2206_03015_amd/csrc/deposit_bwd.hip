// Adjoint of the time-domain deposit with respect to the trajectory samples.
//
// Forward (Algorithm 2, Sec. "Interpolation"): for every interval (tau_{i-1}, tau_i] of
// particle k at pixel m and every grid point u in it,
//   E_tot[m][.][u] += (1 - w) E_{i-1} + w E_i,   w = (u - tau_{i-1}) / (tau_i - tau_{i-1}).
// With g = dJ/dE_tot the interval contributes to its two end samples
//   dJ/dE_{i-1} += (1 - w) g[u],  dJ/dE_i += w g[u],
//   dJ/dtau_{i-1} += -(1 - w) g[u].(E_i - E_{i-1}) / (tau_i - tau_{i-1}),
//   dJ/dtau_i     += -w g[u].(E_i - E_{i-1}) / (tau_i - tau_{i-1}),
// and then flows through the field (lw_field_vjp) and the arrival time
// (dtau/dr = -n/(c dt_obs)) to r, beta, beta_dot.
//
// Gather form, no atomics: a wavefront owns 62 consecutive samples of one particle (lanes
// 1..62; lanes 0 and 63 are halo samples), loops over every pixel, takes the neighbours'
// arrival times and fields by lane shuffles, evaluates the field only where an adjacent
// interval holds grid points, and accumulates its samples' gradients in registers.  Arrival
// times are those of the deposit: the compensated base d of the sample plus the pixel terms,
// with the exact geometry's path term in its third-order series where the particle's max |r|^2
// over the whole trajectory is <= 1e-8 |x_m|^2 (the FP64 deposit's choice), else its square
// root form.
#include "lw_internal.h"

#include <algorithm>

namespace lw {
namespace {

constexpr int kWavesPerBlock = 4;
constexpr int kOwned = 62;
// (|r|/|x|)^2 up to which the series form of the exact-geometry arrival time is used
constexpr double kSeriesBoundBwd = 1e-8;

struct BwdShape {
    int64_t n_particles, n_samples, n_pix, n_obs, n_chunks, sample0;
    double t_start, dt, t0, dt_obs, inv_cdt;
    int fmask;
};

// max_i |r_i|^2 over the usable samples of each particle (the deposit pre-pass's rule and sum
// order): one block per particle
__global__ __launch_bounds__(256) void k_rmax2(const double *__restrict__ r, const double *__restrict__ beta,
                                               const double *__restrict__ beta_dot, int64_t n_samples,
                                               double *__restrict__ rmax2)
{
    __shared__ double s_max[4];
    const int64_t k = blockIdx.x;
    double mx = 0.0;
    for (int64_t i = threadIdx.x; i < n_samples; i += blockDim.x) {
        const size_t o = 3 * (size_t)(k * n_samples + i);
        const double *ri = r + o;
        if (sample_usable(ri, beta + o, beta_dot + o)) mx = fmax(mx, fma(ri[2], ri[2], fma(ri[1], ri[1], ri[0] * ri[0])));
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    if ((threadIdx.x & 63) == 0) s_max[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) m = fmax(m, s_max[w]);
        rmax2[k] = m;
    }
}

__device__ __forceinline__ int64_t grid_count_b(double tau, double n_obs)
{
    return (int64_t)fmin(fmax(floor(tau) + 1.0, 0.0), n_obs);
}

template <int GEOM>
__global__ __launch_bounds__(256) void k_deposit_bwd(const double *__restrict__ r, const double *__restrict__ beta,
                                                     const double *__restrict__ beta_dot,
                                                     const double *__restrict__ charge,
                                                     const double *__restrict__ x_det, const double *__restrict__ dE,
                                                     const double *__restrict__ rbound2, double *__restrict__ d_r,
                                                     double *__restrict__ d_beta, double *__restrict__ d_beta_dot,
                                                     BwdShape sh)
{
    __shared__ PixC s_geo[kWavesPerBlock][64];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t wave = (int64_t)blockIdx.x * kWavesPerBlock + wv;
    const int64_t k = wave / sh.n_chunks;
    if (k >= sh.n_particles) return;  // whole wavefront idle; no block-level sync below
    const int64_t chunk = wave - k * sh.n_chunks;
    const int64_t i = chunk * kOwned + lane - 1;
    const int64_t ns = sh.n_samples;
    const bool in = i >= 0 && i < ns;
    const bool owned = in && lane >= 1 && lane <= kOwned;
    double rs[3] = {0, 0, 0}, bs[3] = {0, 0, 0}, as[3] = {0, 0, 0};
    bool usable = false;
    if (in) {
        const size_t s = (size_t)(k * ns + i) * 3;
        for (int c = 0; c < 3; ++c) {
            rs[c] = r[s + c];
            bs[c] = beta[s + c];
            as[c] = beta_dot[s + c];
        }
        usable = sample_usable(rs, bs, as);
    }
    const double rr = fma(rs[2], rs[2], fma(rs[1], rs[1], rs[0] * rs[0]));
    // sample i of the arrays is sample sample0 + i of the trajectory (spans of a longer one)
    const double dbase = arrival_base(sh.t_start, sh.dt, (double)(sh.sample0 + i), sh.t0, sh.dt_obs, rs[2]);
    const double rb2 = rbound2[k];
    const double q = charge ? charge[k] : -kQe;
    const double nob = (double)sh.n_obs;
    double gr[3] = {0, 0, 0}, gb[3] = {0, 0, 0}, ga[3] = {0, 0, 0};
    PixC *geo = s_geo[wv];

    for (int64_t m0 = 0; m0 < sh.n_pix; m0 += 64) {
        {
            const int64_t mm = std::min<int64_t>(m0 + lane, sh.n_pix - 1);
            geo[lane] = pix_const(x_det, mm, sh.inv_cdt);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const int cnt = (int)std::min<int64_t>(64, sh.n_pix - m0);
        for (int j = 0; j < cnt; ++j) {
            const int64_t m = m0 + j;
            const PixC pcm = geo[j];
            const PixGeo &g = pcm.g;
            const bool ok = usable && g.ok;
            // the exact geometry's correction as its third-order series where the particle's
            // |r|^2 <= 1e-8 |x|^2 over its whole trajectory (exact to rounding, the FP64
            // deposit's form there), else with its square root
            double tau = 0.0;
            if (ok) {
                if (GEOM == LW_GEOM_EXACT && rb2 * (g.invD * g.invD) <= kSeriesBoundBwd)
                    tau = arrival_tau<GEOM, kTauSeries>(pcm, dbase, rs[0], rs[1], rs[2], rr, sh.inv_cdt);
                else
                    tau = arrival_tau<GEOM, kTauSqrt>(pcm, dbase, rs[0], rs[1], rs[2], rr, sh.inv_cdt);
            }
            const double tl = __shfl_up(tau, 1), tr = __shfl_down(tau, 1);
            const int okl = __shfl_up((int)ok, 1), okr = __shfl_down((int)ok, 1);
            const bool left = lane >= 1 && ok && okl && tau > tl;
            const bool right = lane <= 62 && ok && okr && tr > tau;
            const int64_t F = ok ? grid_count_b(tau, nob) : 0;
            const int64_t Fl = left ? grid_count_b(tl, nob) : F, Fr = right ? grid_count_b(tr, nob) : F;
            const bool needE = (left && F > Fl) || (right && Fr > F);
            if (!__ballot(needE)) continue;
            double E[3] = {0, 0, 0};
            const double *xm = x_det + 3 * m;
            if (needE) lw_field<double, GEOM>(g, xm, rs[0], rs[1], rs[2], bs[0], bs[1], bs[2], as[0], as[1], as[2], q,
                                              sh.fmask, E[0], E[1], E[2]);
            double El[3], Er[3];
            for (int c = 0; c < 3; ++c) {
                El[c] = __shfl_up(E[c], 1);
                Er[c] = __shfl_down(E[c], 1);
            }
            if (!owned || !needE) continue;
            const double *dEm = dE + (size_t)m * 3 * sh.n_obs;
            double gE[3] = {0, 0, 0}, gtau = 0.0;
            if (left && F > Fl) {
                const double idt = 1.0 / (tau - tl);
                const double dx = E[0] - El[0], dy = E[1] - El[1], dz = E[2] - El[2];
                for (int64_t u = Fl; u < F; ++u) {
                    const double w = ((double)u - tl) * idt;
                    const double g0 = dEm[u], g1 = dEm[sh.n_obs + u], g2 = dEm[2 * sh.n_obs + u];
                    gE[0] += w * g0;
                    gE[1] += w * g1;
                    gE[2] += w * g2;
                    gtau -= w * (g0 * dx + g1 * dy + g2 * dz) * idt;
                }
            }
            if (right && Fr > F) {
                const double idt = 1.0 / (tr - tau);
                const double dx = Er[0] - E[0], dy = Er[1] - E[1], dz = Er[2] - E[2];
                for (int64_t u = F; u < Fr; ++u) {
                    const double w1 = 1.0 - ((double)u - tau) * idt;
                    const double g0 = dEm[u], g1 = dEm[sh.n_obs + u], g2 = dEm[2 * sh.n_obs + u];
                    gE[0] += w1 * g0;
                    gE[1] += w1 * g1;
                    gE[2] += w1 * g2;
                    gtau -= w1 * (g0 * dx + g1 * dy + g2 * dz) * idt;
                }
            }
            lw_field_vjp<GEOM>(g, xm, rs, bs, as, q, sh.fmask, gE, gr, gb, ga);
            // d tau / d r = -n / (c dt_obs): n = (x - r)/|x - r| (exact) or x/|x| (far field)
            double nx = g.nx, ny = g.ny, nz = g.nz;
            if (GEOM == LW_GEOM_EXACT) {
                const double d0 = xm[0] - rs[0], d1 = xm[1] - rs[1], d2 = xm[2] - rs[2];
                const double R = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                nx = d0 / R;
                ny = d1 / R;
                nz = d2 / R;
            }
            gr[0] -= gtau * nx * sh.inv_cdt;
            gr[1] -= gtau * ny * sh.inv_cdt;
            gr[2] -= gtau * nz * sh.inv_cdt;
        }
        __builtin_amdgcn_wave_barrier();
    }
    if (owned) {
        const size_t s = (size_t)(k * ns + i) * 3;
        for (int c = 0; c < 3; ++c) {
            d_r[s + c] += gr[c];
            d_beta[s + c] += gb[c];
            d_beta_dot[s + c] += ga[c];
        }
    }
}

}  // namespace

size_t deposit_bwd_ws_bytes(int64_t n_particles)
{
    return ((size_t)std::max<int64_t>(n_particles, 1) * sizeof(double) + 255) / 256 * 256;
}

lw_status launch_deposit_bwd(const lw_traj_t *t, const lw_grid_t *gr, int fmask, int geom, const double *dE,
                             double *d_r, double *d_beta, double *d_beta_dot, void *ws, size_t ws_bytes,
                             hipStream_t s, int64_t sample0, const double *rbound2)
{
    if (t->n_particles == 0 || gr->n_pix == 0 || t->n_samples < 2) return LW_OK;
    BwdShape sh;
    sh.n_particles = t->n_particles;
    sh.n_samples = t->n_samples;
    sh.n_pix = gr->n_pix;
    sh.n_obs = gr->n_obs;
    sh.n_chunks = (t->n_samples + kOwned - 1) / kOwned;
    sh.sample0 = sample0;
    sh.t_start = t->t_start;
    sh.dt = t->dt;
    sh.t0 = gr->t0;
    sh.dt_obs = gr->dt_obs;
    sh.inv_cdt = 1.0 / (kC * gr->dt_obs);
    sh.fmask = fmask;
    const int64_t waves = sh.n_particles * sh.n_chunks;
    const int64_t blocks = (waves + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks > 0x7fffffff || sh.n_particles > 0x7fffffff)
        return fail(LW_E_SHAPE, "lw_deposit_td_bwd: problem too large for one launch");
    if (!rbound2) {  // max |r|^2 of each particle over the samples given (its whole trajectory)
        if (!ws || ws_bytes < deposit_bwd_ws_bytes(t->n_particles))
            return fail(LW_E_WORKSPACE, "lw_deposit_td_bwd: workspace of %zu bytes < %zu needed", ws_bytes,
                        deposit_bwd_ws_bytes(t->n_particles));
        k_rmax2<<<(unsigned)t->n_particles, 256, 0, s>>>(t->r, t->beta, t->beta_dot, t->n_samples, (double *)ws);
        rbound2 = (const double *)ws;
    }
    hipEvent_t ev = timing_begin(LW_KERNEL_DEPOSIT_BWD, s);
    if (geom == LW_GEOM_EXACT)
        k_deposit_bwd<LW_GEOM_EXACT><<<(unsigned)blocks, 64 * kWavesPerBlock, 0, s>>>(
            t->r, t->beta, t->beta_dot, t->charge, gr->x_det, dE, rbound2, d_r, d_beta, d_beta_dot, sh);
    else
        k_deposit_bwd<LW_GEOM_FARFIELD><<<(unsigned)blocks, 64 * kWavesPerBlock, 0, s>>>(
            t->r, t->beta, t->beta_dot, t->charge, gr->x_det, dE, rbound2, d_r, d_beta, d_beta_dot, sh);
    timing_end(LW_KERNEL_DEPOSIT_BWD, ev, s);
    return check_launch("lw_deposit_td_bwd");
}

}  // namespace lw
