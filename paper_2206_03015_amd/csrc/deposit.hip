// Time-domain deposit (Algorithm 2 with the piecewise-linear interpolation of
// Sec. "Interpolation"), forward pass.
//
// Work decomposition (one GPU's share of the paper's detector decomposition):
//   * a wavefront owns 64 pixels (one per lane) and a group of particles;
//   * for each particle it streams the trajectory samples through scalar loads
//     (wavefront-uniform), forms every (particle, sample, pixel) arrival time in
//     double and tests whether the interval (tau_{i-1}, tau_i] crosses the next
//     grid point of that pixel's window;
//   * a crossing appends (particle, sample, pixel) to a per-wavefront queue in LDS;
//     whenever 64 entries are queued, all lanes take one entry each, evaluate the
//     Lienard-Wiechert field at the interval's two ends and add the interpolated
//     values at the crossed grid points with global atomics.
// The field is therefore evaluated only at samples that the interpolation reads;
// samples whose interval holds no grid point of the window contribute nothing.
//
// Fast path condition (checked per particle by a pre-pass): every sample usable and
// every step shorter than c*dt by a margin well above the rounding of tau, which makes
// tau strictly increasing for every pixel (|x - r_i| - |x - r_{i-1}| >= -|r_i - r_{i-1}|).
// Particles that fail it take the careful path, which applies the skip rules of
// lw_deposit_td interval by interval.
#include "lw_internal.h"

#include <algorithm>
#include <cmath>

namespace lw {
namespace {

constexpr int kWavesPerBlock = 4;
constexpr int kQCap = 128;
constexpr int kTargetWaves = 16384;

__device__ __forceinline__ double next_grid(double tau, double n_obs)
{
    double f = fmax(floor(tau) + 1.0, 0.0);
    return f >= n_obs ? INFINITY : f;
}

// number of window grid points <= tau: clamp(floor(tau) + 1, 0, n_obs)
__device__ __forceinline__ int64_t grid_count(double tau, double n_obs)
{
    return (int64_t)fmin(fmax(floor(tau) + 1.0, 0.0), n_obs);
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// ---------------------------------------------------------------------------------------------
// pre-pass: arrival-time base alpha_i = (t_i - t0)/dt_obs and the per-particle fast-path flag
__global__ void k_prepass(const double *__restrict__ r, const double *__restrict__ beta,
                          const double *__restrict__ beta_dot, int64_t n_particles, int64_t n_samples,
                          double t_start, double dt, double t0, double dt_obs, double inv_cdt,
                          double *__restrict__ alpha, int *__restrict__ pflag)
{
    const int64_t total = n_particles * n_samples;
    const double cdt_step = kC * dt;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < total;
         s += (int64_t)gridDim.x * blockDim.x) {
        int64_t k = s / n_samples, i = s - k * n_samples;
        if (k == 0) alpha[i] = ((t_start + (double)i * dt) - t0) / dt_obs;
        const double *ri = r + 3 * s, *bi = beta + 3 * s, *ai = beta_dot + 3 * s;
        bool bad = !sample_usable(ri, bi, ai);
        if (!bad && i > 0) {
            const double *rp = ri - 3;
            double dx = ri[0] - rp[0], dy = ri[1] - rp[1], dz = ri[2] - rp[2];
            double step = sqrt(dx * dx + dy * dy + dz * dz);
            double a_i = ((t_start + (double)i * dt) - t0) / dt_obs;
            double scale = fabs(a_i) + (fabs(ri[0]) + fabs(ri[1]) + fabs(ri[2])) * inv_cdt + 1.0;
            double margin = (cdt_step - step) * inv_cdt;  // lower bound of tau_i - tau_{i-1}
            bad = !(margin > 1e-9 + 1e-13 * scale);
        }
        if (bad) atomicOr(pflag + k, 1);
    }
}

template <typename T>
__global__ void k_fill(T *__restrict__ p, int64_t n)
{
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (int64_t)gridDim.x * blockDim.x)
        p[j] = (T)0;
}

// ---------------------------------------------------------------------------------------------
struct DepShape {
    int64_t n_particles, n_samples, n_pix, n_obs;
    int64_t n_tiles, n_tile_blocks, n_groups, parts_per_group;
    double inv_cdt, cdt;
    int fmask;
};

// Evaluate queued crossings: lane j takes entry (qh + j) mod kQCap for j < cnt.
template <typename T, int GEOM>
__device__ __forceinline__ void process_queue(const uint32_t *qi, const uint32_t *qkl, uint32_t qh, uint32_t cnt,
                                              int lane, int64_t tile, int64_t k0, const double *__restrict__ r,
                                              const double *__restrict__ beta, const double *__restrict__ beta_dot,
                                              const double *__restrict__ charge, const double *__restrict__ x_det,
                                              const double *__restrict__ alpha, T *__restrict__ E,
                                              const DepShape &sh)
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    if ((uint32_t)lane < cnt) {
        uint32_t slot = (qh + (uint32_t)lane) & (kQCap - 1);
        uint32_t i = qi[slot], kl = qkl[slot];
        int64_t k = k0 + (int64_t)(kl >> 6);
        int64_t m = tile * 64 + (int64_t)(kl & 63u);
        PixGeo g = pix_geo(x_det, m, sh.inv_cdt);
        const double *xm = x_det + 3 * m;
        const size_t sa = (size_t)(k * sh.n_samples + (int64_t)i - 1) * 3, sb = sa + 3;
        double ta = arrival_tau<GEOM>(g, alpha[i - 1], r[sa], r[sa + 1], r[sa + 2], sh.cdt);
        double tb = arrival_tau<GEOM>(g, alpha[i], r[sb], r[sb + 1], r[sb + 2], sh.cdt);
        double q = charge ? charge[k] : -kQe;
        T eax, eay, eaz, ebx, eby, ebz;
        lw_field<T, GEOM>(g, xm, r[sa], r[sa + 1], r[sa + 2], beta[sa], beta[sa + 1], beta[sa + 2], beta_dot[sa],
                          beta_dot[sa + 1], beta_dot[sa + 2], q, sh.fmask, eax, eay, eaz);
        lw_field<T, GEOM>(g, xm, r[sb], r[sb + 1], r[sb + 2], beta[sb], beta[sb + 1], beta[sb + 2], beta_dot[sb],
                          beta_dot[sb + 1], beta_dot[sb + 2], q, sh.fmask, ebx, eby, ebz);
        const double nob = (double)sh.n_obs;
        int64_t u0 = grid_count(ta, nob), u1 = grid_count(tb, nob);
        double idt = 1.0 / (tb - ta);
        T *Em = E + (size_t)m * 3 * sh.n_obs;
        for (int64_t u = u0; u < u1; ++u) {
            double wd = ((double)u - ta) * idt;
            T w = (T)wd, w1 = (T)(1.0 - wd);
            atomic_add(Em + u, w1 * eax + w * ebx);
            atomic_add(Em + sh.n_obs + u, w1 * eay + w * eby);
            atomic_add(Em + 2 * sh.n_obs + u, w1 * eaz + w * ebz);
        }
    }
    __builtin_amdgcn_wave_barrier();
}

template <typename T, int GEOM>
__global__ __launch_bounds__(256) void k_deposit(const double *__restrict__ r, const double *__restrict__ beta,
                                                 const double *__restrict__ beta_dot,
                                                 const double *__restrict__ charge, const double *__restrict__ x_det,
                                                 const double *__restrict__ alpha, const int *__restrict__ pflag,
                                                 T *__restrict__ E, unsigned long long *__restrict__ diag, DepShape sh)
{
    __shared__ uint32_t q_i[kWavesPerBlock][kQCap];
    __shared__ uint32_t q_kl[kWavesPerBlock][kQCap];
    __shared__ unsigned long long red[4];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wavefront-uniform
    if (threadIdx.x < 4) red[threadIdx.x] = 0ull;
    __syncthreads();

    // block -> (particle group, tile block); consecutive groups on one XCD share trajectory lines in L2
    const int64_t b = blockIdx.x;
    const int64_t xcd = b & 7, slot = b >> 3;
    const int64_t grp = (slot / sh.n_tile_blocks) * 8 + xcd;
    const int64_t tile = (slot % sh.n_tile_blocks) * kWavesPerBlock + wv;
    const int64_t m = tile * 64 + lane;
    const bool pix_in = tile < sh.n_tiles && m < sh.n_pix;
    const int64_t k0 = grp * sh.parts_per_group;
    const int64_t k1 = grp < sh.n_groups ? std::min(k0 + sh.parts_per_group, sh.n_particles) : k0;
    const bool wave_live = tile < sh.n_tiles;

    PixGeo g = pix_geo(x_det, pix_in ? m : 0, sh.inv_cdt);
    const bool lane_ok = pix_in && g.ok;
    const double nob = (double)sh.n_obs;
    unsigned long long c0 = 0, c1 = 0, c2 = 0, c3 = 0;
    uint32_t qh = 0, qn = 0;
    uint32_t *qi = q_i[wv], *qkl = q_kl[wv];
    const int64_t ns = sh.n_samples;

    for (int64_t k = wave_live ? k0 : k1; k < k1; ++k) {
        const double *rk = r + (size_t)k * ns * 3;
        if (pflag[k] == 0) {
            // ---- fast path: tau strictly increasing, all samples usable
            double tau = arrival_tau<GEOM>(g, alpha[0], rk[0], rk[1], rk[2], sh.cdt);
            const double tau0 = tau;
            double gnext = lane_ok ? next_grid(tau, nob) : INFINITY;
            const uint32_t kl_tag = ((uint32_t)(k - k0) << 6) | (uint32_t)lane;
            // one sample: crossing test, queue append, queue drain when 64 entries are pending
            auto step = [&](int64_t i, double ai, double x, double y, double z) {
                tau = arrival_tau<GEOM>(g, ai, x, y, z, sh.cdt);
                const bool hit = tau >= gnext;
                const uint64_t mask = __ballot(hit);
                if (mask) {
                    if (hit) {
                        uint32_t pos = (qh + qn + lanes_below(mask)) & (kQCap - 1);
                        qi[pos] = (uint32_t)i;
                        qkl[pos] = kl_tag;
                        gnext = next_grid(tau, nob);
                    }
                    qn += (uint32_t)__popcll(mask);
                    if (qn >= 64) {
                        process_queue<T, GEOM>(qi, qkl, qh, 64, lane, tile, k0, r, beta, beta_dot, charge, x_det,
                                               alpha, E, sh);
                        qh = (qh + 64) & (kQCap - 1);
                        qn -= 64;
                    }
                }
            };
            int64_t i = 1;
            // four samples per trip; all wavefront-uniform loads issued before the first use
            for (; i + 3 < ns; i += 4) {
                const double a0 = alpha[i], a1 = alpha[i + 1], a2 = alpha[i + 2], a3 = alpha[i + 3];
                const double *rp = rk + 3 * i;
                const double x0 = rp[0], y0 = rp[1], z0 = rp[2], x1 = rp[3], y1 = rp[4], z1 = rp[5];
                const double x2 = rp[6], y2 = rp[7], z2 = rp[8], x3 = rp[9], y3 = rp[10], z3 = rp[11];
                step(i, a0, x0, y0, z0);
                step(i + 1, a1, x1, y1, z1);
                step(i + 2, a2, x2, y2, z2);
                step(i + 3, a3, x3, y3, z3);
            }
            for (; i < ns; ++i) step(i, alpha[i], rk[3 * i], rk[3 * i + 1], rk[3 * i + 2]);
            if (lane_ok) {
                int64_t inside = grid_count(tau, nob) - grid_count(tau0, nob);
                c3 += (unsigned long long)inside;
                c2 += (unsigned long long)((int64_t)(floor(tau) - floor(tau0)) - inside);
            } else if (pix_in) {
                c1 += (unsigned long long)(ns - 1);
            }
        } else {
            // ---- careful path: interval-by-interval skip rules
            const double *bk = beta + (size_t)k * ns * 3, *ak = beta_dot + (size_t)k * ns * 3;
            const double q = charge ? charge[k] : -kQe;
            bool prev_ok = false;
            double tprev = 0.0;
            for (int64_t i = 0; i < ns; ++i) {
                bool ok = lane_ok && sample_usable(rk + 3 * i, bk + 3 * i, ak + 3 * i);
                double tau = NAN;
                if (ok) {
                    tau = arrival_tau<GEOM>(g, alpha[i], rk[3 * i], rk[3 * i + 1], rk[3 * i + 2], sh.cdt);
                    T ex, ey, ez;
                    lw_field<T, GEOM>(g, x_det + 3 * m, rk[3 * i], rk[3 * i + 1], rk[3 * i + 2], bk[3 * i],
                                      bk[3 * i + 1], bk[3 * i + 2], ak[3 * i], ak[3 * i + 1], ak[3 * i + 2], q,
                                      sh.fmask, ex, ey, ez);
                    ok = isfinite(tau) && isfinite((double)ex) && isfinite((double)ey) && isfinite((double)ez);
                }
                bool hit = false;
                if (i > 0 && pix_in) {
                    if (!ok || !prev_ok) {
                        c1 += 1;
                    } else if (!(tau > tprev)) {
                        c0 += 1;
                    } else {
                        int64_t fa = grid_count(tprev, nob), fb = grid_count(tau, nob);
                        c3 += (unsigned long long)(fb - fa);
                        c2 += (unsigned long long)((int64_t)(floor(tau) - floor(tprev)) - (fb - fa));
                        hit = fb > fa;
                    }
                }
                const uint64_t mask = __ballot(hit);
                if (mask) {
                    if (hit) {
                        uint32_t pos = (qh + qn + lanes_below(mask)) & (kQCap - 1);
                        qi[pos] = (uint32_t)i;
                        qkl[pos] = ((uint32_t)(k - k0) << 6) | (uint32_t)lane;
                    }
                    qn += (uint32_t)__popcll(mask);
                    if (qn >= 64) {
                        process_queue<T, GEOM>(qi, qkl, qh, 64, lane, tile, k0, r, beta, beta_dot, charge, x_det,
                                               alpha, E, sh);
                        qh = (qh + 64) & (kQCap - 1);
                        qn -= 64;
                    }
                }
                prev_ok = ok;
                tprev = tau;
            }
        }
    }
    while (qn > 0) {
        uint32_t cnt = qn < 64 ? qn : 64;
        process_queue<T, GEOM>(qi, qkl, qh, cnt, lane, tile, k0, r, beta, beta_dot, charge, x_det, alpha, E, sh);
        qh = (qh + cnt) & (kQCap - 1);
        qn -= cnt;
    }
    // counters: block reduction in LDS, then one global atomic per counter
    if (c0) atomicAdd(&red[0], c0);
    if (c1) atomicAdd(&red[1], c1);
    if (c2) atomicAdd(&red[2], c2);
    if (c3) atomicAdd(&red[3], c3);
    __syncthreads();
    if (diag && threadIdx.x < 4 && red[threadIdx.x]) atomicAdd(diag + threadIdx.x, red[threadIdx.x]);
}

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

size_t deposit_ws_bytes(int64_t n_particles, int64_t n_samples)
{
    return align_up((size_t)std::max<int64_t>(n_particles, 1) * sizeof(int), 256) +
           align_up((size_t)std::max<int64_t>(n_samples, 1) * sizeof(double), 256);
}

lw_status launch_deposit(const lw_traj_t *t, const lw_grid_t *gr, int prec, int fmask, int geom, bool accumulate,
                         void *E, int64_t *diag, void *ws, size_t ws_bytes, hipStream_t s)
{
    const int64_t n_p = t->n_particles, ns = t->n_samples, n_pix = gr->n_pix, n_obs = gr->n_obs;
    const size_t trace_elems = (size_t)n_pix * 3 * (size_t)n_obs;
    const bool f64 = prec == LW_PREC_FP64;
    if (!accumulate) {
        if (trace_elems) {
            int blocks = (int)std::min<size_t>((trace_elems + 255) / 256, 65536);
            if (f64)
                k_fill<double><<<blocks, 256, 0, s>>>((double *)E, (int64_t)trace_elems);
            else
                k_fill<float><<<blocks, 256, 0, s>>>((float *)E, (int64_t)trace_elems);
        }
        if (diag) k_fill<unsigned long long><<<1, 64, 0, s>>>((unsigned long long *)diag, 4);
    }
    if (n_p == 0 || n_pix == 0 || ns == 0) return check_launch("deposit fill");
    int *pflag = (int *)ws;
    double *alpha = (double *)((char *)ws + align_up((size_t)n_p * sizeof(int), 256));
    const double inv_cdt = 1.0 / (kC * gr->dt_obs);
    k_fill<int><<<(int)std::min<int64_t>((n_p + 255) / 256, 65536), 256, 0, s>>>(pflag, n_p);
    {
        int64_t total = n_p * ns;
        int blocks = (int)std::min<int64_t>((total + 255) / 256, 8192);
        k_prepass<<<blocks, 256, 0, s>>>(t->r, t->beta, t->beta_dot, n_p, ns, t->t_start, t->dt, gr->t0, gr->dt_obs,
                                         inv_cdt, alpha, pflag);
    }
    DepShape sh;
    sh.n_particles = n_p;
    sh.n_samples = ns;
    sh.n_pix = n_pix;
    sh.n_obs = n_obs;
    sh.n_tiles = (n_pix + 63) / 64;
    sh.n_tile_blocks = (sh.n_tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    int64_t groups = std::max<int64_t>(1, (kTargetWaves + sh.n_tiles - 1) / sh.n_tiles);
    groups = std::min<int64_t>(groups, n_p);
    sh.parts_per_group = (n_p + groups - 1) / groups;
    sh.n_groups = (n_p + sh.parts_per_group - 1) / sh.parts_per_group;
    sh.inv_cdt = inv_cdt;
    sh.cdt = kC * gr->dt_obs;
    sh.fmask = fmask;
    const int64_t group_slots = (sh.n_groups + 7) / 8 * 8;
    const int64_t blocks = group_slots * sh.n_tile_blocks;
    if (blocks > 0x7fffffff) return fail(LW_E_SHAPE, "lw_deposit_td: problem too large for one launch");
    unsigned long long *dg = (unsigned long long *)diag;
    dim3 grid((unsigned)blocks), block(64 * kWavesPerBlock);
    if (f64) {
        if (geom == LW_GEOM_EXACT)
            k_deposit<double, LW_GEOM_EXACT><<<grid, block, 0, s>>>(t->r, t->beta, t->beta_dot, t->charge,
                                                                    gr->x_det, alpha, pflag, (double *)E, dg, sh);
        else
            k_deposit<double, LW_GEOM_FARFIELD><<<grid, block, 0, s>>>(t->r, t->beta, t->beta_dot, t->charge,
                                                                       gr->x_det, alpha, pflag, (double *)E, dg, sh);
    } else {
        if (geom == LW_GEOM_EXACT)
            k_deposit<float, LW_GEOM_EXACT><<<grid, block, 0, s>>>(t->r, t->beta, t->beta_dot, t->charge, gr->x_det,
                                                                   alpha, pflag, (float *)E, dg, sh);
        else
            k_deposit<float, LW_GEOM_FARFIELD><<<grid, block, 0, s>>>(t->r, t->beta, t->beta_dot, t->charge,
                                                                      gr->x_det, alpha, pflag, (float *)E, dg, sh);
    }
    return check_launch("lw_deposit_td");
}

}  // namespace lw
