// Time-domain deposit (Algorithm 2 with the piecewise-linear interpolation of
// Sec. "Interpolation"), forward pass.
//
// Work decomposition (one GPU's share of the paper's detector decomposition):
//   * a wavefront owns 64 x kPPL pixels (kPPL per lane) and a group of particles;
//   * for each particle it stages 64 samples at a time in LDS (lane j loads sample j),
//     every lane reads each staged sample once (a broadcast) and uses it for each of its
//     pixels: it forms the (particle, sample, pixel) arrival time in double and tests
//     whether the interval (tau_{i-1}, tau_i] crosses the next grid point of that
//     pixel's window (all four tests of a sample pair first, then one branch into the
//     crossing logic if any holds).  With one pixel per lane the broadcast reads bound
//     this loop (LDS returns 128 B per clock); kPPL pixels per lane divide their cost;
//   * a crossing appends (particle, sample, pixel, arrival-time form) to a per-wavefront
//     queue in LDS; whenever 64 entries are queued, all lanes take one entry each,
//     evaluate the Lienard-Wiechert field at the interval's two ends and add the
//     interpolated values at the crossed grid points into a write-combining line of that
//     pixel in LDS (a short run of consecutive grid points of its trace); an interval
//     holding more than kLongRun grid points (an observer grid much finer than the
//     samples) is deposited by the whole wavefront instead, 64 grid points per pass;
//   * a line whose pixel moves past it is added to the trace with global atomics,
//     several lines per instruction (lane l takes value l % 3N of line l / 3N).
// The field is therefore evaluated only at samples that the interpolation reads;
// samples whose interval holds no grid point of the window contribute nothing.  With
// LW_CULL (a separate instantiation) a fast-path particle is skipped when its first and
// last arrival times at the wavefront's pixels bracket no window grid point.
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

constexpr int kPPL = 2;                // pixels per lane
constexpr int kTilePix = 64 * kPPL;     // pixels per wavefront
constexpr int kPixBits = kPPL == 1 ? 6 : kPPL == 2 ? 7 : 8;
static_assert((1 << kPixBits) == kTilePix, "kPPL must be 1, 2 or 4");
constexpr int kWavesPerBlock = 1;
constexpr int kBlockThreads = 64 * kWavesPerBlock;
constexpr uint32_t kQCap = 64 + 2 * 64 * kPPL;  // queue ring per wavefront (63 pending + 2 x kTilePix appended between drains)
// write-combining line per pixel: 16-byte segments of the trace (4 floats or 2 doubles)
template <typename T>
struct WcLine {
    static constexpr int N = 16 / sizeof(T);   // grid points per line
    static constexpr int P = 3 * N + 1;        // LDS stride per pixel (odd: no bank conflicts)
};
constexpr uint32_t kWantNone = 0u;  // below every request (segment + 1)
// queue entry tag: (particle - first particle of the group) << kPixBits | pixel in tile, and this
// bit when the particle's arrival times take the series form
constexpr uint32_t kSerBit = 1u << 31;
// intervals with more grid points than this are deposited by the whole wavefront
constexpr int kLongRun = 8;
constexpr int kStage = 6;  // doubles per staged sample: alpha, x, y, z, |r|^2, pad
// wavefronts per launch to aim for (particle groups x pixel tiles): ~26 rounds of the 3072
// resident wavefronts (12 per CU), so that the last, partly filled round is a small share
// (bunch workload: 16384 wavefronts took 705 ms, 80000 take 655 ms)
constexpr int kTargetWaves = 98304;
// (|r|/|x|)^2 up to which the series form of the exact-geometry arrival time is used
constexpr double kSeriesBound = 1e-8;
constexpr int kPrepassChunk = 8192;

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

// Atomic add into LDS through an LDS-qualified pointer, so that the compiler cannot merge it
// with a global atomic on another path into one flat (address-space generic) atomic.
template <typename T>
__device__ __forceinline__ void lds_add(T *p, T v)
{
    typedef __attribute__((address_space(3))) T lds_t;
    __hip_atomic_fetch_add((lds_t *)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// |r|^2 with the operation order of the pre-pass
__device__ __forceinline__ double sq3(double x, double y, double z) { return fma(z, z, fma(y, y, x * x)); }

__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// value of lane src (wavefront-uniform src) of a double / float / double register
__device__ __forceinline__ double readlane_double(double v, int src)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, src);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), src);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ float readlane_t(float v, int src)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ double readlane_t(double v, int src) { return readlane_double(v, src); }

__device__ __forceinline__ double uniform_double(double v)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct DepWs {
    int *pflag;                 // [n_p] 0 = fast path
    unsigned long long *rmax2;  // [n_p] bits of max_i |r_i|^2 (non-negative doubles order as integers)
    double *alpha;              // [n_s] (t_i - t0)/dt_obs
};

DepWs carve(void *ws, int64_t n_p, int64_t ns)
{
    DepWs w;
    char *p = (char *)ws;
    w.pflag = (int *)p;
    p += align_up((size_t)std::max<int64_t>(n_p, 1) * sizeof(int), 256);
    w.rmax2 = (unsigned long long *)p;
    p += align_up((size_t)std::max<int64_t>(n_p, 1) * sizeof(unsigned long long), 256);
    w.alpha = (double *)p;
    return w;
}

// ---------------------------------------------------------------------------------------------
// pre-pass: one block per (particle, chunk of samples): arrival base alpha_i, sample records,
// per-particle max |r|^2 and the fast-path flag
__global__ __launch_bounds__(256) void k_prepass(const double *__restrict__ r, const double *__restrict__ beta,
                                                 const double *__restrict__ beta_dot, int64_t n_samples,
                                                 int64_t sample0, double t_start, double dt, double t0,
                                                 double dt_obs, double inv_cdt,
                                                 double *__restrict__ alpha, int *__restrict__ pflag,
                                                 unsigned long long *__restrict__ rmax2)
{
    __shared__ unsigned long long s_max[4];
    __shared__ int s_bad[4];
    const int64_t k = blockIdx.x;
    const int64_t i_begin = (int64_t)blockIdx.y * kPrepassChunk;
    const int64_t i_end = std::min<int64_t>(i_begin + kPrepassChunk, n_samples);
    const double cdt_step = kC * dt;
    double mx = 0.0;
    int bad = 0;
    for (int64_t i = i_begin + threadIdx.x; i < i_end; i += blockDim.x) {
        const int64_t s = k * n_samples + i;
        // sample i of the arrays is sample sample0 + i of the trajectory (spans of a longer one)
        const double ai = ((t_start + (double)(sample0 + i) * dt) - t0) / dt_obs;
        if (k == 0) alpha[i] = ai;
        const double *ri = r + 3 * s, *bi = beta + 3 * s, *di = beta_dot + 3 * s;
        const double x = ri[0], y = ri[1], z = ri[2];
        const double rr = sq3(x, y, z);
        bool b = !sample_usable(ri, bi, di);
        if (!b) {
            mx = fmax(mx, rr);
            if (i > 0) {
                const double dx = x - ri[-3], dy = y - ri[-2], dz = z - ri[-1];
                const double step = sqrt(dx * dx + dy * dy + dz * dz);
                const double scale = fabs(ai) + (fabs(x) + fabs(y) + fabs(z)) * inv_cdt + 1.0;
                const double margin = (cdt_step - step) * inv_cdt;  // lower bound of tau_i - tau_{i-1}
                b = !(margin > 1e-9 + 1e-13 * scale);
            }
        }
        bad |= b ? 1 : 0;
    }
    // block reduction
    for (int off = 32; off > 0; off >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, off));
        bad |= __shfl_xor(bad, off);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_max[wv] = (unsigned long long)__double_as_longlong(mx);
        s_bad[wv] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = 0;
        int bb = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            m = std::max(m, s_max[w]);
            bb |= s_bad[w];
        }
        atomicMax(rmax2 + k, m);
        if (bb) atomicOr(pflag + k, 1);
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
    double inv_cdt;
    int fmask;
};

// Per-wavefront state of the deposit kernel.
template <typename T, int GEOM>
struct Wave {

    const double *__restrict__ r;
    const double *__restrict__ beta;
    const double *__restrict__ beta_dot;
    const double *__restrict__ charge;
    const double *__restrict__ x_det;
    const double *__restrict__ alpha;
    const unsigned long long *__restrict__ rmax2;
    T *__restrict__ E;
    DepShape sh;
    double invD2max;  // wavefront maximum of 1/|x_m|^2
    int lane;
    int64_t tile, k0;
    uint2 *q;          // queue ring in LDS: {sample index, (particle - k0) << kPixBits | pixel in tile}
    T *wc;             // write-combining lines in LDS, [kTilePix][WcLine<T>::P] (3 components x N)
    int *wcb;          // [kTilePix] trace segment each line holds (-1: none)
    uint32_t *want;    // [kTilePix] 1 + the furthest segment holding the grid point after a hit in this drain
    int *fpix;         // [64] pixel (in tile) of the j-th line of a flush
    double *stage;     // staged sample records in LDS, [64][kStage]
    PixGeo gl[kPPL];   // geometry of this lane's pixels (lane + 64 h)
    uint32_t qh, qn;   // queue ring head and length
    // arrival-time form of series particles: the short expansion goes with single-precision fields
    static constexpr int kSer = sizeof(T) == 4 ? kTauShort : kTauSeries;

    __device__ __forceinline__ bool series(int64_t k) const
    {
        return GEOM == LW_GEOM_EXACT && __longlong_as_double((long long)rmax2[k]) * invD2max <= kSeriesBound;
    }

    template <int FORM>
    __device__ __forceinline__ double tau_rec(const PixGeo &g, double a, const double *p) const
    {
        return arrival_tau<GEOM, FORM>(g, a, p[0], p[1], p[2], sq3(p[0], p[1], p[2]), sh.inv_cdt);
    }

    __device__ __forceinline__ double tau_any(const PixGeo &g, bool ser, int64_t k, int64_t i) const
    {
        const double *p = r + ((size_t)k * sh.n_samples + i) * 3;
        return ser ? tau_rec<kSer>(g, alpha[i], p) : tau_rec<kTauSqrt>(g, alpha[i], p);
    }

    __device__ __forceinline__ static uint32_t qwrap(uint32_t v) { return v >= kQCap ? v - kQCap : v; }

    // Add the lines of pixels 64 h + (bits of `mask`) to the trace and clear them: lane l of a pass
    // takes value l % 3N (component (l % 3N) / N, grid point l % N) of the (l / 3N)-th line.
    __device__ void flush_lines(uint64_t mask, int h)
    {
        constexpr int NL = WcLine<T>::N, V = 3 * NL;
        const int n = __popcll(mask);
        if (n == 0) return;
        if ((mask >> lane) & 1ull) fpix[lanes_below(mask)] = lane + 64 * h;
        __builtin_amdgcn_wave_barrier();
        for (int l = lane; l < n * V; l += 64) {
            const int jj = l / V, w = l - jj * V;
            const int p = fpix[jj];
            const int c = w / NL, o = w - c * NL;
            T *line = wc + p * WcLine<T>::P + w;
            const T v = *line;
            *line = (T)0;
            const int64_t u = (int64_t)wcb[p] * NL + o;
            if (v != (T)0 && u < sh.n_obs) atomic_add(E + ((size_t)(tile * kTilePix + p) * 3 + c) * sh.n_obs + u, v);
        }
        __builtin_amdgcn_wave_barrier();
    }

    // Evaluate the cnt oldest queued crossings (lane j takes entry j).
    __device__ void drain(uint32_t cnt)
    {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const bool act = (uint32_t)lane < cnt;
        const uint2 e = act ? q[qwrap(qh + (uint32_t)lane)] : make_uint2(1u, 0u);
        const int ml0 = (int)(e.y & (uint32_t)(kTilePix - 1));
        // the entry's pixel geometry from the lane that owns the pixel (all lanes take part)
        PixGeo g;
        {
            const int own = ml0 & 63, hh = ml0 >> 6;
            auto pick = [&](double v0, double v1) {
                const double a = __shfl(v0, own);
                const double b = kPPL > 1 ? __shfl(v1, own) : a;
                return hh ? b : a;
            };
            g.nx = pick(gl[0].nx, gl[kPPL - 1].nx);
            g.ny = pick(gl[0].ny, gl[kPPL - 1].ny);
            g.nz = pick(gl[0].nz, gl[kPPL - 1].nz);
            g.D = pick(gl[0].D, gl[kPPL - 1].D);
            g.invD = pick(gl[0].invD, gl[kPPL - 1].invD);
            g.ok = true;
        }
        // the entry's interval: arrival times, fields at both ends and grid points [u0, u1)
        double ta = 0.0;
        int u0 = 0, u1 = 0;
        T idt = (T)0, eax = (T)0, eay = (T)0, eaz = (T)0, ebx = (T)0, eby = (T)0, ebz = (T)0;
        constexpr int NL = WcLine<T>::N;
        if (act) {
            const uint32_t i = e.x, kl = e.y;
            const int64_t k = k0 + (int64_t)((kl & ~kSerBit) >> kPixBits);
            const int ml = ml0;
            const int64_t m = tile * kTilePix + ml;
            // both samples of the interval, each value loaded once (all loads issued first)
            const size_t sa = ((size_t)k * sh.n_samples + i - 1) * 3;
            const double *ra = r + sa, *ba = beta + sa, *da = beta_dot + sa;
            const double rax = ra[0], ray = ra[1], raz = ra[2], rbx = ra[3], rby = ra[4], rbz = ra[5];
            const double bax = ba[0], bay = ba[1], baz = ba[2], bbx = ba[3], bby = ba[4], bbz = ba[5];
            const double dax = da[0], day = da[1], daz = da[2], dbx = da[3], dby = da[4], dbz = da[5];
            const double ala = alpha[i - 1], alb = alpha[i];
            const double q = charge ? charge[k] : -kQe;
            const double *xm = x_det + 3 * m;
            // arrival times in the form and operation order of the scan (same bits)
            double tb;
            if (kl & kSerBit) {
                ta = arrival_tau<GEOM, kSer>(g, ala, rax, ray, raz, sq3(rax, ray, raz), sh.inv_cdt);
                tb = arrival_tau<GEOM, kSer>(g, alb, rbx, rby, rbz, sq3(rbx, rby, rbz), sh.inv_cdt);
            } else {
                ta = arrival_tau<GEOM, kTauSqrt>(g, ala, rax, ray, raz, sq3(rax, ray, raz), sh.inv_cdt);
                tb = arrival_tau<GEOM, kTauSqrt>(g, alb, rbx, rby, rbz, sq3(rbx, rby, rbz), sh.inv_cdt);
            }
            lw_field<T, GEOM>(g, xm, rax, ray, raz, bax, bay, baz, dax, day, daz, q, sh.fmask, eax, eay, eaz);
            lw_field<T, GEOM>(g, xm, rbx, rby, rbz, bbx, bby, bbz, dbx, dby, dbz, q, sh.fmask, ebx, eby, ebz);
            // grid indices fit in 32 bits (n_obs < 2^31, checked on the host)
            const double nob = (double)sh.n_obs;
            u0 = (int)fmin(fmax(floor(ta) + 1.0, 0.0), nob);
            u1 = (int)fmin(fmax(floor(tb) + 1.0, 0.0), nob);
            // interpolation weight w = (u - ta)/(tb - ta), in the precision of the trace
            idt = sizeof(T) == 4 ? (T)__builtin_amdgcn_rcpf((float)(tb - ta)) : (T)(1.0 / (tb - ta));
            if (u1 - u0 <= kLongRun) {
                const int seg = wcb[ml];
                for (int u = u0; u < u1; ++u) {
                    const T w = (T)((double)u - ta) * idt, w1 = (T)1 - w;
                    const T vx = w1 * eax + w * ebx, vy = w1 * eay + w * eby, vz = w1 * eaz + w * ebz;
                    if (u / NL == seg) {
                        T *line = wc + ml * WcLine<T>::P + (u % NL);
                        lds_add(line, vx);
                        lds_add(line + NL, vy);
                        lds_add(line + 2 * NL, vz);
                    } else {
                        T *Em = E + (size_t)m * 3 * sh.n_obs + u;
                        atomic_add(Em, vx);
                        atomic_add(Em + sh.n_obs, vy);
                        atomic_add(Em + 2 * sh.n_obs, vz);
                    }
                }
            }
            if (u1 > u0) atomicMax(want + ml, (uint32_t)(u1 / NL) + 1u);
        }
        // intervals holding many grid points (a grid much finer than the sample spacing): the
        // whole wavefront deposits them one at a time, 64 consecutive grid points per pass
        uint64_t longm = __ballot(act && u1 - u0 > kLongRun);
        while (longm) {
            const int src = (int)__builtin_ctzll(longm);
            longm &= longm - 1;
            const double sta = readlane_double(ta, src);
            const int su0 = __builtin_amdgcn_readlane(u0, src), su1 = __builtin_amdgcn_readlane(u1, src);
            const int sml = __builtin_amdgcn_readlane(ml0, src);
            const T sidt = readlane_t(idt, src);
            const T sax = readlane_t(eax, src), say = readlane_t(eay, src), saz = readlane_t(eaz, src);
            const T sbx = readlane_t(ebx, src), sby = readlane_t(eby, src), sbz = readlane_t(ebz, src);
            T *Em = E + (size_t)(tile * kTilePix + sml) * 3 * sh.n_obs;
            // 64-bit index: su1 may sit within 64 of the largest int (n_obs up to 2^31 - 1)
            for (int64_t u = (int64_t)su0 + lane; u < su1; u += 64) {
                const T w = (T)((double)u - sta) * sidt, w1 = (T)1 - w;
                atomic_add(Em + u, w1 * sax + w * sbx);
                atomic_add(Em + sh.n_obs + u, w1 * say + w * sby);
                atomic_add(Em + 2 * sh.n_obs + u, w1 * saz + w * sbz);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        // steer each pixel's line to the segment of its next grid point; flush lines that move
#pragma unroll
        for (int h = 0; h < kPPL; ++h) {
            const int p = lane + 64 * h;
            const uint32_t wnt = want[p];
            want[p] = kWantNone;
            const int cur = wcb[p];
            const int nxt = wnt == kWantNone ? cur : (int)(wnt - 1u);
            const bool move = nxt != cur && nxt * (int64_t)WcLine<T>::N < sh.n_obs;
            const uint64_t fm = __ballot(move && cur >= 0);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            flush_lines(fm, h);
            if (move) wcb[p] = nxt;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        qh = __builtin_amdgcn_readfirstlane(qwrap(qh + cnt));
        qn = __builtin_amdgcn_readfirstlane(qn - cnt);
    }

    // Append the lanes with `hit` set (callers drain before 2 x kTilePix more can arrive).
    __device__ __forceinline__ void push(bool hit, uint64_t mask, uint32_t i, uint32_t tag)
    {
        if (hit) q[qwrap(qh + qn + lanes_below(mask))] = make_uint2(i, tag);
        qn = __builtin_amdgcn_readfirstlane(qn + (uint32_t)__popcll(mask));  // wavefront-uniform
    }

    __device__ __forceinline__ void pump()
    {
        while (qn >= 64) drain(64);
    }

    // Fast path: tau strictly increasing, all samples usable.  Samples go through LDS in
    // chunks of 64 (lane j loads sample c0 + j with vector loads one chunk ahead); every lane
    // then reads the staged samples by broadcast, two per trip, each for its kPPL pixels.
    template <int FORM>
    __device__ void fast_particle(const PixGeo *g, const bool *lane_ok, const bool *pix_in, int64_t k,
                                  unsigned long long &c1, unsigned long long &c2, unsigned long long &c3)
    {
        const int64_t ns = sh.n_samples;
        const double nob = (double)sh.n_obs;
        const double *s0 = r + (size_t)k * ns * 3;
        const uint32_t tag0 = ((uint32_t)(k - k0) << kPixBits) | (uint32_t)lane | (FORM == kTauSqrt ? 0u : kSerBit);
        double pa, px, py, pz, prr;
        // unconditional (clamped) loads, so that they stay in flight until the next chunk
        auto fetch = [&](int64_t c0) {
            const int64_t idx = std::min<int64_t>(c0 + lane, ns - 1);
            const double *p = s0 + (size_t)idx * 3;
            pa = alpha[idx];
            px = p[0];
            py = p[1];
            pz = p[2];
            prr = GEOM == LW_GEOM_EXACT ? sq3(px, py, pz) : 0.0;
        };
        fetch(0);
        double tau[kPPL], tau0[kPPL], gnext[kPPL];
        for (int64_t c0 = 0; c0 < ns; c0 += 64) {
            double *st = stage + lane * kStage;
            st[0] = pa;
            st[1] = px;
            st[2] = py;
            st[3] = pz;
            st[4] = prr;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            fetch(c0 + 64);
            const int cnt = (int)std::min<int64_t>(64, ns - c0);
            int j = 0;
            if (c0 == 0) {
#pragma unroll
                for (int h = 0; h < kPPL; ++h) {
                    tau[h] = tau0[h] =
                        arrival_tau<GEOM, FORM>(g[h], stage[0], stage[1], stage[2], stage[3], stage[4], sh.inv_cdt);
                    gnext[h] = lane_ok[h] ? next_grid(tau[h], nob) : INFINITY;
                }
                j = 1;
            }
            // queue the crossings of the arrival times tv of sample jj
            auto hits = [&](int jj, const double *tv) {
#pragma unroll
                for (int h = 0; h < kPPL; ++h) {
                    const bool hit = tv[h] >= gnext[h];
                    const uint64_t mask = __ballot(hit);
                    if (mask) {
                        if (hit) {
                            const double f = floor(tv[h]) + 1.0;
                            gnext[h] = f >= nob ? INFINITY : f;
                        }
                        push(hit, mask, (uint32_t)(c0 + jj), tag0 + 64u * (uint32_t)h);
                    }
                }
            };
            auto step = [&](int jj, const double *e) {
#pragma unroll
                for (int h = 0; h < kPPL; ++h)
                    tau[h] = arrival_tau<GEOM, FORM>(g[h], e[0], e[1], e[2], e[3], e[4], sh.inv_cdt);
                hits(jj, tau);
            };
            for (; j + 1 < cnt; j += 2) {
                double v[2][5];
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int c = 0; c < 5; ++c) v[u][c] = stage[(j + u) * kStage + c];
                // every arrival time is evaluated; one test per pixel on the later sample of the
                // pair (arrival times increase) decides whether the crossing logic runs
                double t0v[kPPL], t1v[kPPL];
                bool any = false;
#pragma unroll
                for (int h = 0; h < kPPL; ++h) {
                    t0v[h] = arrival_tau<GEOM, FORM>(g[h], v[0][0], v[0][1], v[0][2], v[0][3], v[0][4], sh.inv_cdt);
                    t1v[h] = arrival_tau<GEOM, FORM>(g[h], v[1][0], v[1][1], v[1][2], v[1][3], v[1][4], sh.inv_cdt);
                    any |= (t0v[h] >= gnext[h]) | (t1v[h] >= gnext[h]);
                }
                if (__ballot(any)) {
                    hits(j, t0v);
                    hits(j + 1, t1v);
                    pump();
                }
#pragma unroll
                for (int h = 0; h < kPPL; ++h) tau[h] = t1v[h];
            }
            for (; j < cnt; ++j) {
                step(j, stage + j * kStage);
                pump();
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
#pragma unroll
        for (int h = 0; h < kPPL; ++h) {
            if (lane_ok[h]) {
                const int64_t inside = grid_count(tau[h], nob) - grid_count(tau0[h], nob);
                c3 += (unsigned long long)inside;
                c2 += (unsigned long long)((int64_t)(floor(tau[h]) - floor(tau0[h])) - inside);
            } else if (pix_in[h]) {
                c1 += (unsigned long long)(ns - 1);
            }
        }
    }

    // Culling (LW_CULL, fast-path particles only): arrival times are strictly increasing, so the
    // particle deposits into this wavefront's pixels only if some pixel has a window grid point
    // in (tau_first, tau_last].  If none has, the counters follow from the two end points and
    // the particle is skipped; the results are those of the full scan.
    template <int FORM>
    __device__ bool outside(const PixGeo *g, const bool *lane_ok, const bool *pix_in, int64_t k,
                            unsigned long long &c1, unsigned long long &c2)
    {
        const int64_t ns = sh.n_samples;
        const double nob = (double)sh.n_obs;
        const double *p0 = r + (size_t)k * ns * 3, *p1 = p0 + (size_t)(ns - 1) * 3;
        const double a0 = alpha[0], a1 = alpha[ns - 1];
        double tf[kPPL], tl[kPPL];
        bool in = false;
#pragma unroll
        for (int h = 0; h < kPPL; ++h) {
            tf[h] = arrival_tau<GEOM, FORM>(g[h], a0, p0[0], p0[1], p0[2], sq3(p0[0], p0[1], p0[2]), sh.inv_cdt);
            tl[h] = arrival_tau<GEOM, FORM>(g[h], a1, p1[0], p1[1], p1[2], sq3(p1[0], p1[1], p1[2]), sh.inv_cdt);
            in |= lane_ok[h] && grid_count(tl[h], nob) > grid_count(tf[h], nob);
        }
        if (__ballot(in)) return false;
#pragma unroll
        for (int h = 0; h < kPPL; ++h) {
            if (lane_ok[h])
                c2 += (unsigned long long)(int64_t)(floor(tl[h]) - floor(tf[h]));
            else if (pix_in[h])
                c1 += (unsigned long long)(ns - 1);
        }
        return true;
    }

    // Careful path: the skip rules of lw_deposit_td interval by interval.
    __device__ void careful_particle(const PixGeo &g, bool lane_ok, bool pix_in, int64_t m, int h, int64_t k,
                                     unsigned long long &c0, unsigned long long &c1, unsigned long long &c2,
                                     unsigned long long &c3)
    {
        const int64_t ns = sh.n_samples;
        const double nob = (double)sh.n_obs;
        const bool ser = series(k);
        const double q = charge ? charge[k] : -kQe;
        bool prev_ok = false;
        double tprev = 0.0;
        const uint32_t tag = ((uint32_t)(k - k0) << kPixBits) | (uint32_t)(lane + 64 * h) | (ser ? kSerBit : 0u);
        for (int64_t i = 0; i < ns; ++i) {
            const size_t s = (size_t)k * ns + i;
            bool ok = lane_ok && sample_usable(r + 3 * s, beta + 3 * s, beta_dot + 3 * s);
            double tau = NAN;
            if (ok) {
                tau = tau_any(g, ser, k, i);
                T ex, ey, ez;
                lw_field<T, GEOM>(g, x_det + 3 * m, r[3 * s], r[3 * s + 1], r[3 * s + 2], beta[3 * s],
                                  beta[3 * s + 1], beta[3 * s + 2], beta_dot[3 * s], beta_dot[3 * s + 1],
                                  beta_dot[3 * s + 2], q, sh.fmask, ex, ey, ez);
                ok = isfinite(tau) && isfinite((double)ex) && isfinite((double)ey) && isfinite((double)ez);
            }
            bool hit = false;
            if (i > 0 && pix_in) {
                if (!ok || !prev_ok) {
                    c1 += 1;
                } else if (!(tau > tprev)) {
                    c0 += 1;
                } else {
                    const int64_t fa = grid_count(tprev, nob), fb = grid_count(tau, nob);
                    c3 += (unsigned long long)(fb - fa);
                    c2 += (unsigned long long)((int64_t)(floor(tau) - floor(tprev)) - (fb - fa));
                    hit = fb > fa;
                }
            }
            const uint64_t mask = __ballot(hit);
            if (mask) {
                push(hit, mask, (uint32_t)i, tag);
                pump();
            }
            prev_ok = ok;
            tprev = tau;
        }
    }
};

template <typename T, int GEOM, bool CULL>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_deposit(const double *__restrict__ r, const double *__restrict__ beta,
                                                 const double *__restrict__ beta_dot,
                                                 const double *__restrict__ charge, const double *__restrict__ x_det,
                                                 const double *__restrict__ alpha,
                                                 const int *__restrict__ pflag,
                                                 const unsigned long long *__restrict__ rmax2, T *__restrict__ E,
                                                 unsigned long long *__restrict__ diag, DepShape sh)
{
    __shared__ uint2 q_all[kWavesPerBlock][kQCap];
    __shared__ T wc_all[kWavesPerBlock][kTilePix * WcLine<T>::P];
    __shared__ int wcb_all[kWavesPerBlock][kTilePix];
    __shared__ uint32_t want_all[kWavesPerBlock][kTilePix];
    __shared__ int fpix_all[kWavesPerBlock][64];
    __shared__ double stage_all[kWavesPerBlock][64 * kStage];
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
    const int64_t k0 = grp * sh.parts_per_group;
    const int64_t k1 = grp < sh.n_groups ? std::min(k0 + sh.parts_per_group, sh.n_particles) : k0;
    const bool wave_live = tile < sh.n_tiles;

    int64_t m[kPPL];
    bool pix_in[kPPL], lane_ok[kPPL];
    PixGeo g[kPPL];
    double id2 = 0.0;
#pragma unroll
    for (int h = 0; h < kPPL; ++h) {
        m[h] = tile * kTilePix + 64 * h + lane;
        pix_in[h] = wave_live && m[h] < sh.n_pix;
        g[h] = pix_geo(x_det, pix_in[h] ? m[h] : 0);
        lane_ok[h] = pix_in[h] && g[h].ok;
        if (lane_ok[h]) id2 = fmax(id2, g[h].invD * g[h].invD);
    }
    for (int off = 32; off > 0; off >>= 1) id2 = fmax(id2, __shfl_xor(id2, off));

    Wave<T, GEOM> w;
    w.r = r;
    w.beta = beta;
    w.beta_dot = beta_dot;
    w.charge = charge;
    w.x_det = x_det;
    w.alpha = alpha;
    w.rmax2 = rmax2;
    w.E = E;
    w.sh = sh;
    w.invD2max = uniform_double(id2);
    w.lane = lane;
    w.tile = tile;
    w.k0 = k0;
    w.q = q_all[wv];
    w.wc = wc_all[wv];
    w.wcb = wcb_all[wv];
    w.want = want_all[wv];
    w.fpix = fpix_all[wv];
    w.stage = stage_all[wv];
#pragma unroll
    for (int h = 0; h < kPPL; ++h) w.gl[h] = g[h];
    w.qh = 0;
    w.qn = 0;
    for (int j = lane; j < kTilePix * WcLine<T>::P; j += 64) w.wc[j] = (T)0;
    for (int p = lane; p < kTilePix; p += 64) {
        w.wcb[p] = -1;
        w.want[p] = kWantNone;
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();

    unsigned long long c0 = 0, c1 = 0, c2 = 0, c3 = 0;
    for (int64_t k = wave_live ? k0 : k1; k < k1; ++k) {
        if (pflag[k] == 0) {
            if (GEOM == LW_GEOM_EXACT && w.series(k)) {
                if (CULL && w.template outside<Wave<T, GEOM>::kSer>(g, lane_ok, pix_in, k, c1, c2)) continue;
                w.template fast_particle<Wave<T, GEOM>::kSer>(g, lane_ok, pix_in, k, c1, c2, c3);
            } else {
                if (CULL && w.template outside<kTauSqrt>(g, lane_ok, pix_in, k, c1, c2)) continue;
                w.template fast_particle<kTauSqrt>(g, lane_ok, pix_in, k, c1, c2, c3);
            }
        } else {
#pragma unroll
            for (int h = 0; h < kPPL; ++h) w.careful_particle(g[h], lane_ok[h], pix_in[h], m[h], h, k, c0, c1, c2, c3);
        }
    }
    while (w.qn > 0) w.drain(w.qn < 64 ? w.qn : 64);
#pragma unroll
    for (int h = 0; h < kPPL; ++h) w.flush_lines(__ballot(w.wcb[lane + 64 * h] >= 0), h);

    // counters: block reduction in LDS, then one global atomic per counter
    if (c0) atomicAdd(&red[0], c0);
    if (c1) atomicAdd(&red[1], c1);
    if (c2) atomicAdd(&red[2], c2);
    if (c3) atomicAdd(&red[3], c3);
    __syncthreads();
    if (diag && threadIdx.x < 4 && red[threadIdx.x]) atomicAdd(diag + threadIdx.x, red[threadIdx.x]);
}

}  // namespace

size_t deposit_ws_bytes(int64_t n_particles, int64_t n_samples)
{
    const size_t np = (size_t)std::max<int64_t>(n_particles, 1), ns = (size_t)std::max<int64_t>(n_samples, 1);
    return align_up(np * sizeof(int), 256) + align_up(np * sizeof(unsigned long long), 256) +
           align_up(ns * sizeof(double), 256);
}

lw_status launch_deposit(const lw_traj_t *t, const lw_grid_t *gr, int prec, int fmask, int geom, bool accumulate,
                         void *E, int64_t *diag, void *ws, size_t ws_bytes, hipStream_t s, int64_t sample0)
{
    const int64_t n_p = t->n_particles, ns = t->n_samples, n_pix = gr->n_pix, n_obs = gr->n_obs;
    const bool cull = (geom & LW_CULL) != 0;
    geom &= ~LW_CULL;
    const size_t trace_elems = (size_t)n_pix * 3 * (size_t)n_obs;
    const bool f64 = prec == LW_PREC_FP64;
    if (n_obs > 0x7fffffff) return fail(LW_E_SHAPE, "lw_deposit_td: n_obs must be below 2^31");
    DepShape sh;
    sh.n_particles = n_p;
    sh.n_samples = ns;
    sh.n_pix = n_pix;
    sh.n_obs = n_obs;
    sh.n_tiles = (n_pix + kTilePix - 1) / kTilePix;
    sh.n_tile_blocks = (sh.n_tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    int64_t groups = std::max<int64_t>(1, (kTargetWaves + std::max<int64_t>(sh.n_tiles, 1) - 1) /
                                              std::max<int64_t>(sh.n_tiles, 1));
    groups = std::max<int64_t>(1, std::min<int64_t>(groups, n_p));
    sh.parts_per_group = std::max<int64_t>(1, (n_p + groups - 1) / groups);
    sh.n_groups = (n_p + sh.parts_per_group - 1) / sh.parts_per_group;
    sh.fmask = fmask;
    const int64_t chunks = (ns + kPrepassChunk - 1) / kPrepassChunk;
    const int64_t blocks = (sh.n_groups + 7) / 8 * 8 * sh.n_tile_blocks;
    if (sh.parts_per_group >= (int64_t(1) << (31 - kPixBits)))
        return fail(LW_E_SHAPE, "lw_deposit_td: too many particles per pixel tile group");
    if (n_p > 0x7fffffff || chunks > 65535) return fail(LW_E_SHAPE, "lw_deposit_td: too many samples");
    if (blocks > 0x7fffffff) return fail(LW_E_SHAPE, "lw_deposit_td: problem too large for one launch");
    if (!accumulate) {
        if (trace_elems) {
            const int blocks = (int)std::min<size_t>((trace_elems + 255) / 256, 65536);
            if (f64)
                k_fill<double><<<blocks, 256, 0, s>>>((double *)E, (int64_t)trace_elems);
            else
                k_fill<float><<<blocks, 256, 0, s>>>((float *)E, (int64_t)trace_elems);
        }
        if (diag) k_fill<unsigned long long><<<1, 64, 0, s>>>((unsigned long long *)diag, 4);
    }
    if (n_p == 0 || n_pix == 0 || ns == 0) return check_launch("deposit fill");
    const DepWs w = carve(ws, n_p, ns);
    const double inv_cdt = 1.0 / (kC * gr->dt_obs);
    sh.inv_cdt = inv_cdt;
    const int fill_blocks = (int)std::min<int64_t>((n_p + 255) / 256, 65536);
    k_fill<int><<<fill_blocks, 256, 0, s>>>(w.pflag, n_p);
    k_fill<unsigned long long><<<fill_blocks, 256, 0, s>>>(w.rmax2, n_p);
    {
        k_prepass<<<dim3((unsigned)n_p, (unsigned)chunks), 256, 0, s>>>(
            t->r, t->beta, t->beta_dot, ns, sample0, t->t_start, t->dt, gr->t0, gr->dt_obs, inv_cdt, w.alpha, w.pflag,
            w.rmax2);
    }
    unsigned long long *dg = (unsigned long long *)diag;
    const dim3 grid((unsigned)blocks), block(kBlockThreads);
#define LW_DEPOSIT_LAUNCH(T, G, C)                                                                                  \
    k_deposit<T, G, C><<<grid, block, 0, s>>>(t->r, t->beta, t->beta_dot, t->charge, gr->x_det, w.alpha, w.pflag,    \
                                              w.rmax2, (T *)E, dg, sh)
    // culling is a separate instantiation: the full evaluation carries none of its code
    hipEvent_t t_start = timing_begin(LW_KERNEL_DEPOSIT, s);
    if (f64) {
        if (geom == LW_GEOM_EXACT) {
            if (cull) LW_DEPOSIT_LAUNCH(double, LW_GEOM_EXACT, true); else LW_DEPOSIT_LAUNCH(double, LW_GEOM_EXACT, false);
        } else {
            if (cull) LW_DEPOSIT_LAUNCH(double, LW_GEOM_FARFIELD, true); else LW_DEPOSIT_LAUNCH(double, LW_GEOM_FARFIELD, false);
        }
    } else {
        if (geom == LW_GEOM_EXACT) {
            if (cull) LW_DEPOSIT_LAUNCH(float, LW_GEOM_EXACT, true); else LW_DEPOSIT_LAUNCH(float, LW_GEOM_EXACT, false);
        } else {
            if (cull) LW_DEPOSIT_LAUNCH(float, LW_GEOM_FARFIELD, true); else LW_DEPOSIT_LAUNCH(float, LW_GEOM_FARFIELD, false);
        }
    }
#undef LW_DEPOSIT_LAUNCH
    timing_end(LW_KERNEL_DEPOSIT, t_start, s);
    return check_launch("lw_deposit_td");
}

}  // namespace lw
