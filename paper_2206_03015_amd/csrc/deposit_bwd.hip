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
// Gather form, no global atomics: a wavefront owns 62 consecutive samples of one particle (lanes
// 1..62; lanes 0 and 63 are halo samples), loops over every pixel with lanes over samples, and
// finds the intervals (tau_{l-1}, tau_l] that hold window grid points from the neighbour lane's
// arrival time (a DPP lane shift).  Those intervals are queued in LDS and evaluated 64 at a time,
// one per lane (fields at both ends, the adjoint, the field and arrival-time Jacobians); the
// results go to LDS accumulators of the wavefront's samples, written out once at the end.  Arrival
// times are those of the FP64 deposit: for a chunk of pixels all at the records' distance and
// in the series range (the particle's max |r|^2 over its whole trajectory <= 1e-8 |x_m|^2) the
// records' polynomial in b (coefficients from the lane's sample), else per pixel the compensated
// base d plus the pixel terms with the path term as its third-order series in that range, else
// its square root form.
#include "lw_internal.h"

#include <algorithm>

namespace lw {
namespace {

constexpr int kOwned = 62;
constexpr uint32_t kQueue = 128;  // queued intervals (a pixel adds at most 63 to fewer than 64)

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

// Neighbour lanes' values by DPP wavefront shifts (no LDS round trip): lane l gets lane l - 1's
// (up; lane 0 gets 0) or lane l + 1's (down; lane 63 gets 0)
template <int CTRL>
__device__ __forceinline__ double dpp_double(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double lane_up(double v) { return dpp_double<0x138 /* wave_shr:1 */>(v); }
__device__ __forceinline__ double lane_down(double v) { return dpp_double<0x130 /* wave_shl:1 */>(v); }

// Whether (ta, tb] (ta < tb) holds window grid points, i.e. whether the window's grid count
// clamp(floor(t) + 1, 0, n_obs) is larger at tb: floor(tb) > floor(ta), floor(tb) >= 0 and
// floor(ta) <= n_obs - 2
__device__ __forceinline__ bool holds_grid(double fa, double fb, double nob2)
{
    return fb > fa && fb >= 0.0 && fa <= nob2;
}

template <int GEOM>
__global__ __launch_bounds__(64) void k_deposit_bwd(const double *__restrict__ r, const double *__restrict__ beta,
                                                    const double *__restrict__ beta_dot,
                                                    const double *__restrict__ charge,
                                                    const double *__restrict__ x_det, const double *__restrict__ dE,
                                                    const double *__restrict__ rbound2, double *__restrict__ d_r,
                                                    double *__restrict__ d_beta, double *__restrict__ d_beta_dot,
                                                    BwdShape sh)
{
    __shared__ PixGeo geo[64];            // the current chunk of pixels: geometry
    __shared__ double pcs[3][64];         // and o, px, py
    __shared__ uint2 qe[kQueue];          // queued intervals: {right-end lane, pixel in chunk}
    __shared__ double2 qt[kQueue];        // their arrival times {tau_a, tau_b}
    __shared__ double acc[9][64];         // d(r, beta, beta_dot) of the wavefront's samples
    const int lane = threadIdx.x;
    const int64_t wave = blockIdx.x;
    const int64_t k = wave / sh.n_chunks;
    const int64_t chunk = wave - k * sh.n_chunks;
    const int64_t i0 = chunk * kOwned - 1;  // sample of lane 0
    const int64_t i = i0 + lane;
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
#pragma unroll
    for (int c = 0; c < 9; ++c) acc[c][lane] = 0.0;
    const double rr = fma(rs[2], rs[2], fma(rs[1], rs[1], rs[0] * rs[0]));
    // sample i of the arrays is sample sample0 + i of the trajectory (spans of a longer one)
    const double dbase = arrival_base(sh.t_start, sh.dt, (double)(sh.sample0 + i), sh.t0, sh.dt_obs, rs[2]);
    const double rb2 = rbound2[k];
    const double q = charge ? charge[k] : -kQe;
    const double nob = (double)sh.n_obs, nob2 = nob - 2.0;
    // the FP64 deposit's records: tau(b) as a polynomial of degree 5 for pixels at the distance
    // of pixel 0, its coefficients from this lane's sample (the same function and inputs as the
    // deposit's pre-pass, so the same bits of tau where both use them)
    const double Dref = GEOM == LW_GEOM_EXACT ? pix_geo(x_det, 0).D : 1.0;
    double cp[6] = {0, 0, 0, 0, 0, 0};
    if (GEOM == LW_GEOM_EXACT) tau_poly<5>(dbase, rs[0], rs[1], rs[2], sh.inv_cdt, Dref, cp);
    uint32_t qh = 0, qn = 0;
    // this lane and the one below both hold usable samples (the interval ending here has both ends)
    const uint64_t um = __ballot(usable);
    const bool pair_ok = usable && lane >= 1 && ((um >> (lane - 1)) & 1ull);

    // Intervals (tau_{a}, tau_{b}] (b = a + 1 = right-end lane, 1..63) of the queue, one per lane:
    // fields at both ends, the interpolation's adjoint over the interval's grid points, the field
    // and arrival-time adjoints, added to the accumulators of the owned end samples
    auto drain = [&](uint32_t cnt, int64_t m0) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if ((uint32_t)lane < cnt) {
            const uint32_t slot = (qh + (uint32_t)lane) & (kQueue - 1);
            const uint2 e = qe[slot];
            const double2 tt = qt[slot];
            const int lb = (int)e.x, j = (int)e.y;
            const PixGeo g = geo[j];
            const int64_t m = m0 + j;
            const double *xm = x_det + 3 * m;
            const size_t sa = (size_t)(k * ns + i0 + lb - 1) * 3;
            double ra[3], ba[3], da[3], rb[3], bb[3], db[3];
            for (int c = 0; c < 3; ++c) {
                ra[c] = r[sa + c];
                rb[c] = r[sa + 3 + c];
                ba[c] = beta[sa + c];
                bb[c] = beta[sa + 3 + c];
                da[c] = beta_dot[sa + c];
                db[c] = beta_dot[sa + 3 + c];
            }
            double Ea[3], Eb[3];
            lw_field<double, GEOM>(g, xm, ra[0], ra[1], ra[2], ba[0], ba[1], ba[2], da[0], da[1], da[2], q, sh.fmask,
                                   Ea[0], Ea[1], Ea[2]);
            lw_field<double, GEOM>(g, xm, rb[0], rb[1], rb[2], bb[0], bb[1], bb[2], db[0], db[1], db[2], q, sh.fmask,
                                   Eb[0], Eb[1], Eb[2]);
            const double ta = tt.x, tb = tt.y;
            const double idt = 1.0 / (tb - ta);
            const double dx = Eb[0] - Ea[0], dy = Eb[1] - Ea[1], dz = Eb[2] - Ea[2];
            double gEa[3] = {0, 0, 0}, gEb[3] = {0, 0, 0}, gta = 0.0, gtb = 0.0;
            const double *dEm = dE + (size_t)m * 3 * sh.n_obs;
            const int64_t u0 = grid_count_b(ta, nob), u1 = grid_count_b(tb, nob);
            for (int64_t u = u0; u < u1; ++u) {
                const double w = ((double)u - ta) * idt, w1 = 1.0 - w;
                const double g0 = dEm[u], g1 = dEm[sh.n_obs + u], g2 = dEm[2 * sh.n_obs + u];
                gEa[0] += w1 * g0;
                gEa[1] += w1 * g1;
                gEa[2] += w1 * g2;
                gEb[0] += w * g0;
                gEb[1] += w * g1;
                gEb[2] += w * g2;
                const double gd = (g0 * dx + g1 * dy + g2 * dz) * idt;
                gta -= w1 * gd;
                gtb -= w * gd;
            }
            // the end samples this wavefront owns (lanes 1..62): a = lb - 1, b = lb
            auto end = [&](int l, const double *re, const double *be, const double *de, const double *gE,
                           double gt) {
                double gr[3] = {0, 0, 0}, gb[3] = {0, 0, 0}, ga[3] = {0, 0, 0};
                lw_field_vjp<GEOM>(g, xm, re, be, de, q, sh.fmask, gE, gr, gb, ga);
                // d tau / d r = -n / (c dt_obs): n = (x - r)/|x - r| (exact) or x/|x| (far field)
                double nx = g.nx, ny = g.ny, nz = g.nz;
                if (GEOM == LW_GEOM_EXACT) {
                    const double d0 = xm[0] - re[0], d1 = xm[1] - re[1], d2 = xm[2] - re[2];
                    const double R = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                    nx = d0 / R;
                    ny = d1 / R;
                    nz = d2 / R;
                }
                gr[0] -= gt * nx * sh.inv_cdt;
                gr[1] -= gt * ny * sh.inv_cdt;
                gr[2] -= gt * nz * sh.inv_cdt;
                for (int c = 0; c < 3; ++c) {
                    atomicAdd(&acc[c][l], gr[c]);
                    atomicAdd(&acc[3 + c][l], gb[c]);
                    atomicAdd(&acc[6 + c][l], ga[c]);
                }
            };
            if (lb - 1 >= 1) end(lb - 1, ra, ba, da, gEa, gta);
            if (lb <= kOwned) end(lb, rb, bb, db, gEb, gtb);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        qh = (qh + cnt) & (kQueue - 1);
        qn -= cnt;
    };

    for (int64_t m0 = 0; m0 < sh.n_pix; m0 += 64) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        {
            const int64_t mm = std::min<int64_t>(m0 + lane, sh.n_pix - 1);
            const PixC pl = pix_const(x_det, mm, sh.inv_cdt);
            geo[lane] = pl.g;
            pcs[0][lane] = pl.o;
            pcs[1][lane] = pl.px;
            pcs[2][lane] = pl.py;
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const int cnt = (int)std::min<int64_t>(64, sh.n_pix - m0);
        // the records apply to this chunk of pixels if every pixel is at the reference distance
        // and in the series range of this particle (the deposit's rule for its tiles)
        bool rec_chunk = false, rec_low = false;
        if (GEOM == LW_GEOM_EXACT) {
            const PixGeo &gl = geo[lane];
            const bool fits = lane >= cnt || (gl.ok && fabs(gl.D - Dref) <= kSameDistance * Dref &&
                                              rb2 * (gl.invD * gl.invD) <= kSeriesBound);
            rec_chunk = __ballot(!fits) == 0;
            // the forward deposit's lower-degree rule, decided over the same 128-pixel tile (its
            // usable pixels' largest 2 (1 - n_z)), so that both evaluate the same polynomial
            double s2 = lane < cnt && gl.ok ? 2.0 * (1.0 - gl.nz) : 0.0;  // this chunk: half the tile
            const int64_t mo = (m0 ^ 64) + lane;                               // the other half
            if (mo < sh.n_pix) {
                const PixGeo go = pix_geo(x_det, mo);
                if (go.ok) s2 = fmax(s2, 2.0 * (1.0 - go.nz));
            }
            for (int off = 32; off > 0; off >>= 1) s2 = fmax(s2, __shfl_xor(s2, off));
            const bool low = rec_chunk && tail_negligible<true>(rb2, s2, sh.inv_cdt, cp[5], Dref);
            rec_low = __builtin_amdgcn_readfirstlane(low ? 1 : 0) != 0;  // the same in every lane
        }
        for (int j = 0; j < cnt; ++j) {
            // interval (tau_{lane-1}, tau_lane]: both samples usable (and the pixel), increasing,
            // holding window grid points
            double tau = 0.0;
            bool ok2;  // this lane's interval has both ends
            if (rec_chunk) {  // every pixel of the chunk usable: the lanes' flags alone
                const double b = fma(pcs[2][j], rs[1], fma(pcs[1][j], rs[0], pcs[0][j] * rs[2]));
                double u;
                if (rec_low) {  // degree 3 of 5, as the forward where its terms above are negligible
                    u = fma(b, cp[3], cp[2]);
                    u = fma(b, u, cp[1]);
                    u = fma(b, u, cp[0]);
                } else {
                    u = fma(b, cp[5], cp[4]);
#pragma unroll
                    for (int c = 3; c >= 0; --c) u = fma(b, u, cp[c]);
                }
                tau = u;
                ok2 = pair_ok;
            } else {
                PixC pcm;
                pcm.g = geo[j];
                pcm.o = pcs[0][j];
                pcm.px = pcs[1][j];
                pcm.py = pcs[2][j];
                const bool ok = usable && pcm.g.ok;
                if (ok) {
                    if (GEOM == LW_GEOM_EXACT && rb2 * (pcm.g.invD * pcm.g.invD) <= kSeriesBound)
                        tau = arrival_tau<GEOM, kTauSeries>(pcm, dbase, rs[0], rs[1], rs[2], rr, sh.inv_cdt);
                    else
                        tau = arrival_tau<GEOM, kTauSqrt>(pcm, dbase, rs[0], rs[1], rs[2], rr, sh.inv_cdt);
                }
                const uint64_t okm = __ballot(ok);
                ok2 = ok && lane >= 1 && ((okm >> (lane - 1)) & 1ull);
            }
            const double tl = lane_up(tau);
            const bool hit = ok2 && tau > tl && holds_grid(floor(tl), floor(tau), nob2);
            const uint64_t mask = __ballot(hit);
            if (mask) {
                if (hit) {
                    const uint32_t slot = (qh + qn + (uint32_t)lanes_below(mask)) & (kQueue - 1);
                    qe[slot] = make_uint2((uint32_t)lane, (uint32_t)j);
                    qt[slot] = make_double2(tl, tau);
                }
                qn += (uint32_t)__popcll(mask);
                while (qn >= 64) drain(64, m0);
            }
        }
        while (qn > 0) drain(qn < 64 ? qn : 64, m0);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if (owned) {
        const size_t s = (size_t)(k * ns + i) * 3;
        for (int c = 0; c < 3; ++c) {
            d_r[s + c] += acc[c][lane];
            d_beta[s + c] += acc[3 + c][lane];
            d_beta_dot[s + c] += acc[6 + c][lane];
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
    const int64_t blocks = sh.n_particles * sh.n_chunks;  // one wavefront each
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
        k_deposit_bwd<LW_GEOM_EXACT><<<(unsigned)blocks, 64, 0, s>>>(
            t->r, t->beta, t->beta_dot, t->charge, gr->x_det, dE, rbound2, d_r, d_beta, d_beta_dot, sh);
    else
        k_deposit_bwd<LW_GEOM_FARFIELD><<<(unsigned)blocks, 64, 0, s>>>(
            t->r, t->beta, t->beta_dot, t->charge, gr->x_det, dE, rbound2, d_r, d_beta, d_beta_dot, sh);
    timing_end(LW_KERNEL_DEPOSIT_BWD, ev, s);
    return check_launch("lw_deposit_td_bwd");
}

}  // namespace lw
