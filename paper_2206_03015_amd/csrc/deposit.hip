// Time-domain deposit (Algorithm 2 with the piecewise-linear interpolation of
// Sec. "Interpolation"), forward pass.
//
// Work decomposition (one GPU's share of the paper's detector decomposition):
//   * a pre-pass writes, for every (particle, sample), a record: the sample's arrival base d
//     (the two large, cancelling terms of the arrival time, carried in double-double and
//     rounded once) and, for the exact geometry with the path term in series form, the
//     coefficients of the arrival time as a polynomial in the pixel variable b
//     (tau = sum_j c_j b^j, b = C((1 - n_z) z - n_x x - n_y y): one fused multiply-add per
//     degree and pixel, at a lower degree where kModeRecLow applies); it also flags particles
//     whose arrival times are provably increasing and finds each particle's max |r|^2; a pixel
//     table holds each pixel's constants;
//   * fast path (k_scan): a wavefront owns a tile of kTilePix pixels and a group of particles.
//     For each particle it walks the samples in chunks of 64 (lane j holds sample 63 q + j of
//     chunk q, so consecutive chunks share one sample and every interval has both ends in one
//     chunk), three chunks at a time, the first value of each record of the next three loaded
//     ahead.  The records sit in vector registers; for each pixel of the tile its next grid point
//     and its constants come from LDS, the same address in every lane (the constants from the
//     pixel table with scalar loads where each pixel takes its own arrival-time form), and every
//     lane forms the arrival time of its sample and compares it with that grid point.  If any
//     lane reaches it, the intervals of the chunk that hold window grid points follow from the two
//     ends' arrival times (the neighbouring lane's value) and are queued in LDS with both arrival
//     times;
//   * careful path (k_careful, particles the pre-pass could not clear): lanes own pixels; the
//     skip rules of lw_deposit_td are applied interval by interval, and crossings go to the same
//     queue;
//   * the queue is drained 64 entries at a time, one per lane (see Wave::drain): the field at the
//     interval's two ends and the interpolated values at its grid points, added to the trace with
//     global atomics.  An interval holding more than kLongRun grid points (an observer grid much
//     finer than the samples) is deposited by the whole wavefront, 64 grid points per pass.
// The field is therefore evaluated only at samples that the interpolation reads.  Every decision
// and weight uses one arrival-time value per (sample, pixel): both orientations evaluate it with
// the same operations (tau_eval).  With LW_CULL (a separate instantiation) a fast-path particle
// is skipped when its first and last arrival times at the wavefront's pixels bracket no window
// grid point.
//
// Arrival-time forms (exact geometry): the polynomial records hold the path term's series
// (first order with single-precision fields, third order with double ones; valid where
// |r|^2 <= 1e-8 |x_m|^2 over the whole trajectory) for pixels at the records' distance
// (|x_m| of the first pixel), evaluated to a lower degree where the terms above it are provably
// negligible for the particle and the wavefront's pixels (kModeRecLow); a wavefront whose pixels
// sit at another distance, or a particle outside the series bound, evaluates arrival_tau per
// pixel instead (series or square-root form), from the same d.
//
// Fast path condition (checked per particle by the pre-pass): every sample usable and
// every step shorter than c*dt by a margin well above the rounding of tau, which makes
// tau strictly increasing for every pixel (|x - r_i| - |x - r_{i-1}| >= -|r_i - r_{i-1}|).
#include "lw_internal.h"

#include <algorithm>
#include <cmath>

namespace lw {
namespace {

constexpr int kPPL = 2;                 // pixels per lane
constexpr int kTilePix = 64 * kPPL;     // pixels per wavefront
constexpr int kPixBits = 7;
static_assert((1 << kPixBits) == kTilePix, "tile of 128 pixels");
constexpr int kBlockThreads = 64;
// queue ring: up to 63 pending entries plus one push (at most 64 crossings: one sample's pixels
// of one half of the tile on the careful path, one chunk's intervals on the fast path)
constexpr uint32_t kQCap = 128;
// intervals with more grid points than this are deposited by the whole wavefront
constexpr int kLongRun = 8;
// wavefronts per launch to aim for (particle groups x pixel tiles): ~26 rounds of the 3072
// resident wavefronts (12 per CU), so that the last, partly filled round is a small share
constexpr int kTargetWaves = 98304;
// at most this many particles per group: the wavefronts of a group (one per pixel tile, started
// together on one XCD) read the same records, and stay close enough to share them in L2
constexpr int kMaxPartsPerGroup = 4;
constexpr int kPrepassChunk = 8192;
// pixel table: kPT doubles per pixel (o, px, py, ok, nx, ny, nz, D, invD, padding), at most
// kPixTabMax pixels per pass (its share of the workspace); larger grids take several passes
constexpr int kPT = 16;
constexpr int64_t kPixTabMax = 16384;
static_assert(kPixTabMax % kTilePix == 0, "whole tiles per pixel pass");

// scan modes: polynomial records (degree 3 or 5 in b, exact geometry), far field (tau = d + b),
// or arrival_tau per pixel in one of its forms
constexpr int kModeRec3 = 0, kModeRec5 = 1, kModeFar = 2, kModeSqrt = 3, kModeSeries = 4, kModeShort = 5;
// arrival_tau per pixel with the form of each pixel (series where rb2 |x_m|^-2 <= kSeriesBound)
constexpr int kModeMixed = 6;
// polynomial records evaluated to a lower degree (RecLayout::LOW: 2 of 3 with single-precision
// fields, 3 of 5 with double ones) where tail_negligible holds for the particle and the tile
constexpr int kModeRecLow = 7;

// Record of one sample (doubles), read by the scan with scalar loads:
//   far field:          d, x, y, z
//   exact, degree 3:    c_0, c_1, c_2, x, y, z, d, (pad)
//   exact, degree 5:    c_0, c_1, c_2, c_3, c_4, x, y, z, d, (pad)
// (the leading coefficient c_DEG is the same for every sample and is not stored)
template <int GEOM, bool F64>
struct RecLayout {
    static constexpr int DEG = GEOM == LW_GEOM_FARFIELD ? 0 : (F64 ? 5 : 3);
    static constexpr int LOW = GEOM == LW_GEOM_FARFIELD ? 0 : (F64 ? 3 : 2);  // degree of kModeRecLow
    static constexpr int X = GEOM == LW_GEOM_FARFIELD ? 1 : DEG;      // x, y, z at X, X + 1, X + 2
    static constexpr int D = GEOM == LW_GEOM_FARFIELD ? 0 : DEG + 3;  // d
    static constexpr int W = GEOM == LW_GEOM_FARFIELD ? 4 : DEG + 5;  // width
};
__host__ __device__ constexpr int rec_width(int geom, bool f64)
{
    return geom == LW_GEOM_FARFIELD ? RecLayout<LW_GEOM_FARFIELD, false>::W
                                    : (f64 ? RecLayout<LW_GEOM_EXACT, true>::W : RecLayout<LW_GEOM_EXACT, false>::W);
}

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

// |r|^2 with the operation order of the pre-pass
__device__ __forceinline__ double sq3(double x, double y, double z) { return fma(z, z, fma(y, y, x * x)); }

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

// The previous lane's value (lane l gets lane l - 1's; lane 0 gets 0): a DPP shift of the
// wavefront by one lane, no LDS round trip
__device__ __forceinline__ double lane_shift_up(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138 /* wave_shr:1 */, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double uniform_double(double v)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// The records are written by the pre-pass launch and only read while the deposit kernel runs, so
// the scan reads them through the constant address space: with a wavefront-uniform address in
// scalar registers these become scalar loads.
typedef const __attribute__((address_space(4))) double *cdptr;
__device__ __forceinline__ cdptr uniform_ptr(const double *p)
{
    const uint64_t b = (uint64_t)reinterpret_cast<uintptr_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return (cdptr)(((uint64_t)hi << 32) | lo);
}

// ---------------------------------------------------------------------------------------------
// Pixel table and the arrival time shared by both orientations of the scan

// rows [0, n_rows): the pixels [0, n_pix), then padding rows (all zero, not usable) up to the end
// of the last tile, whose arrival times stay finite
__global__ void k_pixtab(const double *__restrict__ x_det, int64_t n_pix, int64_t n_rows, double C,
                         double *__restrict__ pt)
{
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n_rows) return;
    double *o = pt + m * kPT;
    if (m >= n_pix) {
#pragma unroll
        for (int j = 0; j < kPT; ++j) o[j] = 0.0;
        return;
    }
    const PixC p = pix_const(x_det, m, C);
    o[0] = p.o;
    o[1] = p.px;
    o[2] = p.py;
    o[3] = p.g.ok ? 1.0 : 0.0;
    o[4] = p.g.nx;
    o[5] = p.g.ny;
    o[6] = p.g.nz;
    o[7] = p.g.D;
    o[8] = p.g.invD;
#pragma unroll
    for (int j = 9; j < kPT; ++j) o[j] = 0.0;
}

// a pixel's constants from its table row (per lane, or wavefront-uniform through scalar loads)
template <typename P>
__device__ __forceinline__ PixC pixc_row(P row)
{
    PixC p;
    p.o = row[0];
    p.px = row[1];
    p.py = row[2];
    p.g.ok = row[3] != 0.0;
    p.g.nx = row[4];
    p.g.ny = row[5];
    p.g.nz = row[6];
    p.g.D = row[7];
    p.g.invD = row[8];
    return p;
}

// The part of a record a scan mode reads: offset OFF and count N of doubles; X: offset of the
// position within them; LEAD: the value (c_0 or d) that carries the arrival time's constant term
// (-inf there makes the arrival time -inf: no crossing)
template <int GEOM, bool F64, int MODE>
struct ScanVals {
    using L = RecLayout<GEOM, F64>;
    static constexpr bool kRecMode = MODE == kModeRec3 || MODE == kModeRec5 || MODE == kModeRecLow;
    static constexpr int OFF = MODE == kModeMixed ? L::X : 0;
    static constexpr int N = (MODE == kModeFar || MODE == kModeMixed) ? 4 : L::DEG + 3;
    static constexpr int X = MODE == kModeFar ? 1 : (MODE == kModeMixed ? 0 : L::DEG);
    static constexpr int LEAD = MODE == kModeMixed ? 3 : 0;
};

// Arrival time of one (sample, pixel) in scan mode MODE from the record values v and the pixel
// constants P: far field tau = d + b; polynomial records tau = sum_j c_j b^j (c_DEG = cK; up to
// j = LOW in kModeRecLow); else
// arrival_tau in the pixel's form (series where rb2 |x_m|^-2 <= kSeriesBound).  Both orientations
// (lanes over pixels, v uniform; lanes over samples, P uniform) run these same operations, so a
// (sample, pixel) gets the same bits wherever it is evaluated.
template <int GEOM, bool F64, int MODE>
__device__ __forceinline__ double tau_eval(const PixC &P, const double *v, double cK, double rb2, double C)
{
    if constexpr (MODE == kModeFar) {
        return pix_b(P, v[1], v[2], v[3]) + v[0];
    } else if constexpr (MODE == kModeRec3 || MODE == kModeRec5 || MODE == kModeRecLow) {
        constexpr int DEG = RecLayout<GEOM, F64>::DEG, LOW = RecLayout<GEOM, F64>::LOW;
        const double b = pix_b(P, v[DEG], v[DEG + 1], v[DEG + 2]);
        double u;
        if constexpr (MODE == kModeRecLow) {
            u = fma(b, v[LOW], v[LOW - 1]);
#pragma unroll
            for (int j = LOW - 2; j >= 0; --j) u = fma(b, u, v[j]);
        } else {
            u = fma(b, cK, v[DEG - 1]);
#pragma unroll
            for (int j = DEG - 2; j >= 0; --j) u = fma(b, u, v[j]);
        }
        return u;
    } else {
        constexpr int FORM = F64 ? kTauSeries : kTauShort;
        const double x = v[0], y = v[1], z = v[2], rr = sq3(x, y, z);
        if (rb2 * (P.g.invD * P.g.invD) <= kSeriesBound) return arrival_tau<GEOM, FORM>(P, v[3], x, y, z, rr, C);
        return arrival_tau<GEOM, kTauSqrt>(P, v[3], x, y, z, rr, C);
    }
}

// tau_eval of NB records at one pixel: with polynomial records the operations of each record are
// tau_eval's, in its order, interleaved across the records, so that a wavefront has NB
// independent chains to issue from instead of one dependent chain at a time (same bits)
template <int GEOM, bool F64, int MODE, int NB, int N>
__device__ __forceinline__ void tau_eval_block(const PixC &P, const double (*R)[N], double cK, double rb2, double C,
                                               double *t)
{
    if constexpr (MODE == kModeRec3 || MODE == kModeRec5 || MODE == kModeRecLow) {
        constexpr int DEG = RecLayout<GEOM, F64>::DEG, LOW = RecLayout<GEOM, F64>::LOW;
        double b[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) b[c] = P.o * R[c][DEG + 2];
#pragma unroll
        for (int c = 0; c < NB; ++c) b[c] = fma(P.px, R[c][DEG], b[c]);
#pragma unroll
        for (int c = 0; c < NB; ++c) b[c] = fma(P.py, R[c][DEG + 1], b[c]);
        // the highest power: cK, or c_LOW in kModeRecLow
        constexpr int TOP = MODE == kModeRecLow ? LOW - 1 : DEG - 1;
#pragma unroll
        for (int c = 0; c < NB; ++c) t[c] = MODE == kModeRecLow ? fma(b[c], R[c][LOW], R[c][LOW > 0 ? LOW - 1 : 0])
                                                               : fma(b[c], cK, R[c][DEG - 1]);
#pragma unroll
        for (int j = TOP - 1; j >= 0; --j)
#pragma unroll
            for (int c = 0; c < NB; ++c) t[c] = fma(b[c], t[c], R[c][j]);
    } else {
#pragma unroll
        for (int c = 0; c < NB; ++c) t[c] = tau_eval<GEOM, F64, MODE>(P, R[c], cK, rb2, C);
    }
}

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct DepWs {
    double *pt;                 // [kPixTabMax][kPT] pixel table of the current pass
    int *pflag;                 // [n_p] 0 = fast path
    unsigned long long *rmax2;  // [n_p] bits of max_i |r_i|^2 (non-negative doubles order as integers)
    double *rec;                // [n_p][n_s][rec_width] records
};

constexpr size_t kPixTabBytes = (size_t)kPixTabMax * kPT * sizeof(double);

// pixel table, flags, bounds and records (one record more than the samples: padding)
size_t ws_bytes_for(int64_t n_p, int64_t ns, int rw)
{
    const size_t np = (size_t)std::max<int64_t>(n_p, 1), nsz = (size_t)std::max<int64_t>(ns, 1);
    return kPixTabBytes + align_up(np * sizeof(int), 256) + align_up(np * sizeof(unsigned long long), 256) +
           align_up((np * nsz + 1) * (size_t)rw * sizeof(double), 256);
}

DepWs carve(void *ws, int64_t n_p)
{
    DepWs w;
    char *p = (char *)ws;
    w.pt = (double *)p;
    p += kPixTabBytes;
    w.pflag = (int *)p;
    p += align_up((size_t)std::max<int64_t>(n_p, 1) * sizeof(int), 256);
    w.rmax2 = (unsigned long long *)p;
    p += align_up((size_t)std::max<int64_t>(n_p, 1) * sizeof(unsigned long long), 256);
    w.rec = (double *)p;
    return w;
}

// ---------------------------------------------------------------------------------------------
// pre-pass: one block per (particle, chunk of samples): records, per-particle max |r|^2 and the
// fast-path flag
template <int GEOM, int DEG>
__global__ __launch_bounds__(256) void k_prepass(const double *__restrict__ r, const double *__restrict__ beta,
                                                 const double *__restrict__ beta_dot,
                                                 const double *__restrict__ x_det, int64_t n_samples,
                                                 int64_t sample0, double t_start, double dt, double t0,
                                                 double dt_obs, double C, double *__restrict__ rec,
                                                 int *__restrict__ pflag, unsigned long long *__restrict__ rmax2)
{
    using L = RecLayout<GEOM, DEG == 5>;
    __shared__ unsigned long long s_max[4];
    __shared__ int s_bad[4];
    const int64_t k = blockIdx.x;
    const int64_t i_begin = (int64_t)blockIdx.y * kPrepassChunk;
    const int64_t i_end = std::min<int64_t>(i_begin + kPrepassChunk, n_samples);
    const double cdt_step = kC * dt;
    const double Dref = pix_geo(x_det, 0).D;  // the records' pixel distance
    double mx = 0.0;
    int bad = 0;
    for (int64_t i = i_begin + threadIdx.x; i < i_end; i += blockDim.x) {
        const int64_t s = k * n_samples + i;
        const double *ri = r + 3 * s, *bi = beta + 3 * s, *di = beta_dot + 3 * s;
        const double x = ri[0], y = ri[1], z = ri[2];
        // sample i of the arrays is sample sample0 + i of the trajectory (spans of a longer one)
        const double d = arrival_base(t_start, dt, (double)(sample0 + i), t0, dt_obs, z);
        double *o = rec + (size_t)s * L::W;
        o[L::D] = d;
        o[L::X] = x;
        o[L::X + 1] = y;
        o[L::X + 2] = z;
        if (GEOM == LW_GEOM_EXACT) {
            double c[DEG + 1];
            tau_poly<DEG>(d, x, y, z, C, Dref, c);
#pragma unroll
            for (int j = 0; j < DEG; ++j) o[j] = c[j];
            o[L::W - 1] = 0.0;
        }
        const double rr = sq3(x, y, z);
        bool b = !sample_usable(ri, bi, di);
        if (!b) {
            mx = fmax(mx, rr);
            if (i > 0) {
                const double dx = x - ri[-3], dy = y - ri[-2], dz = z - ri[-1];
                const double step = sqrt(dx * dx + dy * dy + dz * dz);
                // bound of the rounding of tau (its terms: d, b ~ C (|x| + |y| + 2|z|), the path term)
                const double scale = fabs(d) + 2.0 * (fabs(x) + fabs(y) + fabs(z)) * C + 1.0;
                const double margin = (cdt_step - step) * C;  // lower bound of tau_i - tau_{i-1}
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
    int64_t n_tiles, n_groups, parts_per_group;
    double C;  // 1/(c dt_obs)
    int fmask;
};

// Per-wavefront state of the careful path (k_careful): lanes own pixels (kPPL each); a particle's
// samples are taken one at a time, with the skip rules applied per interval; crossings are queued
// in LDS and drained 64 at a time, each lane adding one interval's grid points to the trace with
// global atomics (ACC: how a contribution is added to the trace).
template <typename T, int GEOM, int ACC = kAccFloat>
struct Wave {
    const double *__restrict__ r;
    const double *__restrict__ beta;
    const double *__restrict__ beta_dot;
    const double *__restrict__ charge;
    const double *__restrict__ x_det;
    const double *__restrict__ rec;
    const double *__restrict__ pt;  // pixel table of this pass
    T *__restrict__ E;
    DepShape sh;
    double cK;  // leading coefficient of the polynomial records
    double rb2; // the current particle's bound of |r|^2 over its whole trajectory
    int lane;
    int64_t tile, k0;
    uint2 *q;          // queue ring in LDS: {sample index, (particle - k0) << kPixBits | pixel in tile}
    double2 *qt;       // the entry's arrival times {tau_{i-1}, tau_i}
    PixC pc[kPPL];     // constants of this lane's pixels (lane + 64 h)
    uint32_t qh, qn;   // queue ring head and length
    DetAcc det;        // high words and row scales (ACC == kAccFixed)

    __device__ __forceinline__ static uint32_t qwrap(uint32_t v) { return v >= kQCap ? v - kQCap : v; }

    // contribution v to element j of the trace, in the order-independent modes (FP64 only)
    __device__ __forceinline__ void put_det(size_t j, size_t row, double v) const
    {
        unsigned long long *lo = (unsigned long long *)E + j;
        if (ACC == kAccMaxAbs) {
            atomicMax(lo, (unsigned long long)__double_as_longlong(fabs(v)));
        } else {
            // |v * scale| < 2^62 by the choice of scale, and any term below 2^63 is taken, so a
            // last-bit difference between the two passes' v cannot drop one (a NaN scale drops
            // all: the row is NaN in the result).  The sign-extended term is added to the 128-bit
            // sum as its low word and, with the carry out of the low word, its high word.
            const double t = v * det.scale[row];
            const long long n = fabs(t) < 0x1p63 ? (long long)__builtin_rint(t) : 0ll;
            if (n != 0) {
                const unsigned long long un = (unsigned long long)n;
                const unsigned long long old = atomicAdd(lo, un);
                const long long dh = (n < 0 ? -1ll : 0ll) + (old + un < old ? 1ll : 0ll);
                if (dh != 0) atomicAdd(det.hi + j, (unsigned long long)dh);
            }
        }
    }

    using Lay = RecLayout<GEOM, sizeof(T) == 8>;
    // the part of a record a scan mode reads: offset and count of doubles
    template <int MODE>
    static constexpr int scan_off()
    {
        return MODE == kModeMixed ? Lay::X : 0;
    }
    template <int MODE>
    static constexpr int scan_n()
    {
        return MODE == kModeFar || MODE == kModeMixed ? 4 : Lay::DEG + 3;
    }

    // Arrival time of pixel h from the scan values v of a sample's record (wavefront-uniform)
    template <int MODE>
    __device__ __forceinline__ double tau_of(int h, const double *v) const
    {
        return tau_eval<GEOM, sizeof(T) == 8, MODE>(pc[h], v, cK, rb2, sh.C);
    }

    // the scan values of sample i of particle k
    template <int MODE>
    __device__ __forceinline__ void load_scan(int64_t k, int64_t i, double *v) const
    {
        const double *src = rec + ((size_t)k * sh.n_samples + i) * Lay::W + scan_off<MODE>();
#pragma unroll
        for (int c = 0; c < scan_n<MODE>(); ++c) v[c] = src[c];
    }

    // Evaluate the cnt oldest queued crossings (lane j takes entry j).
    __device__ void drain(uint32_t cnt)
    {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        const bool act = (uint32_t)lane < cnt;
        const uint32_t slot = qwrap(qh + (uint32_t)lane);
        const uint2 e = act ? q[slot] : make_uint2(1u, 0u);
        const double2 tt = act ? qt[slot] : make_double2(0.0, 1.0);
        const int ml0 = (int)(e.y & (uint32_t)(kTilePix - 1));
        // far field: the entry's pixel direction from the pixel table
        PixGeo g;
        if (GEOM == LW_GEOM_FARFIELD) {
            g = pixc_row(pt + (size_t)(tile * kTilePix + ml0) * kPT).g;
        } else {
            g.nx = g.ny = 0.0;
            g.nz = g.D = g.invD = 1.0;
            g.ok = true;
        }
        // the entry's interval: fields at both ends and grid points [u0, u1)
        const double ta = tt.x, tb = tt.y;
        int u0 = 0, u1 = 0;
        T idt = (T)0, eax = (T)0, eay = (T)0, eaz = (T)0, ebx = (T)0, eby = (T)0, ebz = (T)0;
        if (act) {
            const uint32_t i = e.x, kl = e.y;
            const int64_t k = k0 + (int64_t)(kl >> kPixBits);
            const int ml = ml0;
            const int64_t m = tile * kTilePix + ml;
            // both samples of the interval, each value loaded once (all loads issued first)
            const size_t sa = ((size_t)k * sh.n_samples + i - 1) * 3;
            const double *ra = r + sa, *ba = beta + sa, *da = beta_dot + sa;
            const double rax = ra[0], ray = ra[1], raz = ra[2], rbx = ra[3], rby = ra[4], rbz = ra[5];
            const double bax = ba[0], bay = ba[1], baz = ba[2], bbx = ba[3], bby = ba[4], bbz = ba[5];
            const double dax = da[0], day = da[1], daz = da[2], dbx = da[3], dby = da[4], dbz = da[5];
            const double q = charge ? charge[k] : -kQe;
            const double *xm = x_det + 3 * m;
            lw_field<T, GEOM>(g, xm, rax, ray, raz, bax, bay, baz, dax, day, daz, q, sh.fmask, eax, eay, eaz);
            lw_field<T, GEOM>(g, xm, rbx, rby, rbz, bbx, bby, bbz, dbx, dby, dbz, q, sh.fmask, ebx, eby, ebz);
            // grid indices fit in 32 bits (n_obs < 2^31, checked on the host)
            const double nob = (double)sh.n_obs;
            u0 = (int)fmin(fmax(floor(ta) + 1.0, 0.0), nob);
            u1 = (int)fmin(fmax(floor(tb) + 1.0, 0.0), nob);
            // interpolation weight w = (u - ta)/(tb - ta), in the precision of the trace
            idt = sizeof(T) == 4 ? (T)__builtin_amdgcn_rcpf((float)(tb - ta)) : (T)(1.0 / (tb - ta));
            if (u1 - u0 <= kLongRun) {
                T *Em = E + (size_t)m * 3 * sh.n_obs;
                for (int u = u0; u < u1; ++u) {
                    const T w = (T)((double)u - ta) * idt, w1 = (T)1 - w;
                    if constexpr (ACC == kAccFloat) {
                        atomic_add(Em + u, w1 * eax + w * ebx);
                        atomic_add(Em + sh.n_obs + u, w1 * eay + w * eby);
                        atomic_add(Em + 2 * sh.n_obs + u, w1 * eaz + w * ebz);
                    } else {
                        const size_t row = (size_t)m * 3, j = row * sh.n_obs + u;
                        put_det(j, row, w1 * eax + w * ebx);
                        put_det(j + sh.n_obs, row + 1, w1 * eay + w * eby);
                        put_det(j + 2 * sh.n_obs, row + 2, w1 * eaz + w * ebz);
                    }
                }
            }
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
                if constexpr (ACC == kAccFloat) {
                    atomic_add(Em + u, w1 * sax + w * sbx);
                    atomic_add(Em + sh.n_obs + u, w1 * say + w * sby);
                    atomic_add(Em + 2 * sh.n_obs + u, w1 * saz + w * sbz);
                } else {
                    const size_t row = (size_t)(tile * kTilePix + sml) * 3, j = row * sh.n_obs + u;
                    put_det(j, row, w1 * sax + w * sbx);
                    put_det(j + sh.n_obs, row + 1, w1 * say + w * sby);
                    put_det(j + 2 * sh.n_obs, row + 2, w1 * saz + w * sbz);
                }
            }
        }
        // the entries are read: later pushes may take their slots
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        qh = __builtin_amdgcn_readfirstlane(qwrap(qh + cnt));
        qn = __builtin_amdgcn_readfirstlane(qn - cnt);
    }

    // Append the lanes with `hit` set (callers drain before kTilePix more can arrive).
    __device__ __forceinline__ void push(bool hit, uint64_t mask, uint32_t i, uint32_t tag, double ta, double tb)
    {
        if (hit) {
            const uint32_t slot = qwrap(qh + qn + lanes_below(mask));
            q[slot] = make_uint2(i, tag);
            qt[slot] = make_double2(ta, tb);
        }
        qn = __builtin_amdgcn_readfirstlane(qn + (uint32_t)__popcll(mask));  // wavefront-uniform
    }

    __device__ __forceinline__ void pump()
    {
        while (qn >= 64) drain(64);
    }

    // Careful path: the skip rules of lw_deposit_td interval by interval, pixel h of this lane,
    // with the arrival times of the fast path's MODE (the same values wherever a particle takes
    // the fast path in one span and the careful path in another).
    template <int MODE, int H>
    __device__ __forceinline__ void careful_particle(bool lane_ok, bool pix_in, int64_t m, int64_t k,
                                                     unsigned long long &c0, unsigned long long &c1,
                                                     unsigned long long &c2, unsigned long long &c3)
    {
        constexpr int NV = scan_n<MODE>();
        const int64_t ns = sh.n_samples;
        const double nob = (double)sh.n_obs;
        const double q = charge ? charge[k] : -kQe;
        bool prev_ok = false;
        double tprev = 0.0;
        const uint32_t tag = ((uint32_t)(k - k0) << kPixBits) | (uint32_t)(lane + 64 * H);
        for (int64_t i = 0; i < ns; ++i) {
            const size_t s = (size_t)k * ns + i;
            double v[NV];
            load_scan<MODE>(k, i, v);
            const double x = r[3 * s], y = r[3 * s + 1], z = r[3 * s + 2];
            bool ok = lane_ok && sample_usable(r + 3 * s, beta + 3 * s, beta_dot + 3 * s);
            const double tv = tau_of<MODE>(H, v);
            double tau = NAN;
            if (ok) {
                tau = tv;
                T ex, ey, ez;
                lw_field<T, GEOM>(pc[H].g, x_det + 3 * m, x, y, z, beta[3 * s], beta[3 * s + 1], beta[3 * s + 2],
                                  beta_dot[3 * s], beta_dot[3 * s + 1], beta_dot[3 * s + 2], q, sh.fmask, ex, ey, ez);
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
                push(hit, mask, (uint32_t)i, tag, tprev, tau);
                pump();
            }
            prev_ok = ok;
            tprev = tau;
        }
    }

    // One particle in scan mode MODE, both pixels of this lane
    template <int MODE>
    __device__ __forceinline__ void particle(const bool *lane_ok, const bool *pix_in, const int64_t *m, int64_t k,
                                             unsigned long long &c0, unsigned long long &c1, unsigned long long &c2,
                                             unsigned long long &c3)
    {
        static_assert(kPPL == 2, "careful path written for two pixels per lane");
        careful_particle<MODE, 0>(lane_ok[0], pix_in[0], m[0], k, c0, c1, c2, c3);
        careful_particle<MODE, 1>(lane_ok[1], pix_in[1], m[1], k, c0, c1, c2, c3);
    }
};

// careful path: the particles the pre-pass flagged (a wavefront whose group holds none exits)
template <typename T, int GEOM, int ACC>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_careful(
    const double *__restrict__ r, const double *__restrict__ beta, const double *__restrict__ beta_dot,
    const double *__restrict__ charge, const double *__restrict__ x_det, const double *__restrict__ rec,
    const double *__restrict__ pt, const int *__restrict__ pflag, const unsigned long long *__restrict__ rmax2,
    const double *__restrict__ rbound2, T *__restrict__ E, unsigned long long *__restrict__ diag, DepShape sh, DetAcc det)
{
    constexpr bool kF64 = sizeof(T) == 8;
    constexpr int kRec = kF64 ? kModeRec5 : kModeRec3;
    // block -> (particle group, tile) as in k_scan
    const int64_t b = blockIdx.x;
    const int64_t xcd = b & 7, slot = b >> 3;
    const int64_t grp = (slot / sh.n_tiles) * 8 + xcd;
    const int64_t tile = slot % sh.n_tiles;
    const int64_t k0 = grp * sh.parts_per_group;
    const int64_t k1 = grp < sh.n_groups ? std::min(k0 + sh.parts_per_group, sh.n_particles) : k0;
    {
        bool any = false;
        for (int64_t k = k0 + (threadIdx.x & 63); k < k1; k += 64) any |= pflag[k] != 0;
        if (__ballot(any) == 0) return;  // whole block (one wavefront)
    }
    __shared__ uint2 q_all[kQCap];
    __shared__ double2 qt_all[kQCap];
    __shared__ unsigned long long red[4];
    const int lane = threadIdx.x & 63;
    if (threadIdx.x < 4) red[threadIdx.x] = 0ull;
    __syncthreads();

    Wave<T, GEOM, ACC> w;
    int64_t m[kPPL];
    bool pix_in[kPPL], lane_ok[kPPL];
    double id2 = 0.0, s2 = 0.0;
    const double Dref = pix_geo(x_det, 0).D;  // the records' pixel distance
    bool far_off = false;                     // a pixel of this wavefront at another distance
#pragma unroll
    for (int h = 0; h < kPPL; ++h) {
        m[h] = tile * kTilePix + 64 * h + lane;
        pix_in[h] = m[h] < sh.n_pix;
        w.pc[h] = pixc_row(pt + (pix_in[h] ? m[h] : 0) * kPT);
        lane_ok[h] = pix_in[h] && w.pc[h].g.ok;
        if (lane_ok[h]) {
            id2 = fmax(id2, w.pc[h].g.invD * w.pc[h].g.invD);
            s2 = fmax(s2, 2.0 * (1.0 - w.pc[h].g.nz));
            far_off |= !(fabs(w.pc[h].g.D - Dref) <= kSameDistance * Dref);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        id2 = fmax(id2, __shfl_xor(id2, off));
        s2 = fmax(s2, __shfl_xor(s2, off));
    }
    const double invD2max = uniform_double(id2), s2max = uniform_double(s2);
    const bool rec_ok = GEOM == LW_GEOM_EXACT && __ballot(far_off) == 0;
    {
        double c[6];
        if (kF64)
            tau_poly<5>(0.0, 0.0, 0.0, 0.0, sh.C, Dref, c);
        else
            tau_poly<3>(0.0, 0.0, 0.0, 0.0, sh.C, Dref, c);
        w.cK = c[kF64 ? 5 : 3];
    }

    w.r = r;
    w.beta = beta;
    w.beta_dot = beta_dot;
    w.charge = charge;
    w.x_det = x_det;
    w.rec = rec;
    w.pt = pt;
    w.E = E;
    if constexpr (ACC != kAccFloat) w.det = det;
    w.sh = sh;
    w.lane = lane;
    w.tile = tile;
    w.k0 = k0;
    w.q = q_all;
    w.qt = qt_all;
    w.qh = 0;
    w.qn = 0;

    unsigned long long c0 = 0, c1 = 0, c2 = 0, c3 = 0;
    for (int64_t k = k0; k < k1; ++k) {
        if (pflag[k] == 0) continue;  // fast path: k_scan
        // series forms where |r|^2 <= 1e-8 |x_m|^2 over the whole trajectory (the max over the
        // whole trajectory when given, else over the samples of this call), decided per pixel
        w.rb2 = rbound2 ? rbound2[k] : __longlong_as_double((long long)rmax2[k]);
        const bool all_ser = GEOM == LW_GEOM_EXACT && w.rb2 * invD2max <= kSeriesBound;
        if (GEOM == LW_GEOM_FARFIELD)
            w.template particle<kModeFar>(lane_ok, pix_in, m, k, c0, c1, c2, c3);
        else if (all_ser && rec_ok) {
            if (tail_negligible<kF64>(w.rb2, s2max, sh.C, w.cK, Dref))
                w.template particle<kModeRecLow>(lane_ok, pix_in, m, k, c0, c1, c2, c3);
            else
                w.template particle<kRec>(lane_ok, pix_in, m, k, c0, c1, c2, c3);
        } else
            w.template particle<kModeMixed>(lane_ok, pix_in, m, k, c0, c1, c2, c3);
    }
    while (w.qn > 0) w.drain(w.qn < 64 ? w.qn : 64);

    // counters: block reduction in LDS, then one global atomic per counter
    if (c0) atomicAdd(&red[0], c0);
    if (c1) atomicAdd(&red[1], c1);
    if (c2) atomicAdd(&red[2], c2);
    if (c3) atomicAdd(&red[3], c3);
    __syncthreads();
    if (diag && threadIdx.x < 4 && red[threadIdx.x]) atomicAdd(diag + threadIdx.x, red[threadIdx.x]);
}

// ---------------------------------------------------------------------------------------------
// Fast path.  Lanes over samples: lane j of chunk q holds sample 63 q + j (chunks share their
// boundary sample, so interval (63 q + j - 1, 63 q + j] has both ends in chunk q for j >= 1).

template <typename T, int GEOM, int ACC = kAccFloat>
struct ScanWave {
    static constexpr bool F64 = sizeof(T) == 8;
    using Lay = RecLayout<GEOM, F64>;
    // chunks per block: three. With double-precision fields (degree-5 records) this leaves a few
    // values that live through the whole kernel in scratch (36 bytes, reloaded once per particle);
    // still faster than two chunks: 1124 against 1141 ms on 1e4 electrons of the precision workload
    static constexpr int NB = 3;
    Wave<T, GEOM, ACC> d;  // queue and drain (shared with the careful path)
    double *pcl;           // LDS: o, px, py, g of the tile's pixels, [kTilePix + 1][4] (one padding row);
                           // g: the pixel's next grid point above the arrival times scanned so far
    uint64_t okmask[kPPL]; // pixels 64 h + l of the tile that take part (in the pass, geometry ok)

    // Issue the loads of the records of chunks q .. q + NB - 1 (lane = sample) into R; valid[c]
    // is false for samples past the last one and chunks past the last one (q + c >= nq), whose
    // constant term the caller sets to -inf once the loads are in (mask_block), so that the loads
    // can stay in flight meanwhile.
    template <int MODE>
    __device__ __forceinline__ void load_block(const double *rk, int q, int nq, double (*R)[ScanVals<GEOM, F64, MODE>::N],
                                               bool *valid, bool use_first, const double (&first)[NB]) const
    {
        using SV = ScanVals<GEOM, F64, MODE>;
        const int ns = (int)d.sh.n_samples;
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const int s = 63 * (q + c) + d.lane;
            valid[c] = s < ns && q + c < nq;
            const double *src = rk + (size_t)(valid[c] ? s : ns - 1) * Lay::W;
            R[c][0] = use_first ? first[c] : src[0];
#pragma unroll
            for (int v = 1; v < SV::N; ++v) R[c][v] = src[v];
        }
    }
    // The first scan value of each record of chunks q .. q + NB - 1, loaded one block ahead: it
    // brings the records' cache lines in while the current block is scanned (the rest of each
    // record is loaded at the block's start, from the cache).
    template <int MODE>
    __device__ __forceinline__ void touch_block(const double *rk, int q, double (&first)[NB]) const
    {
        const int ns = (int)d.sh.n_samples;
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            const int s = std::min(63 * (q + c) + d.lane, ns - 1);
            first[c] = rk[(size_t)s * Lay::W];
        }
    }
    template <int MODE>
    __device__ __forceinline__ static void mask_block(double (*R)[ScanVals<GEOM, F64, MODE>::N], const bool *valid)
    {
#pragma unroll
        for (int c = 0; c < NB; ++c)
            if (!valid[c]) R[c][ScanVals<GEOM, F64, MODE>::LEAD] = -INFINITY;
    }

    // Crossings of pixel p (tile-local) in the chunks of a block that reached its next grid point:
    // the intervals that hold grid points of the window are queued with their two arrival times
    // (the field and the deposit follow in the drain, 64 intervals at a time).
    __device__ __forceinline__ void crossings(int64_t k, int q0, int nq, int p, const double *t)
    {
        const int ns = (int)d.sh.n_samples;
        const double nob2 = (double)d.sh.n_obs - 2.0;
        const uint32_t tag = ((uint32_t)(k - d.k0) << kPixBits) | (uint32_t)p;
#pragma unroll
        for (int c = 0; c < NB; ++c) {
            if (q0 + c >= nq) break;
            const int s = 63 * (q0 + c) + d.lane;
            const bool iv = d.lane >= 1 && s < ns;  // this lane ends an interval
            const double tb = t[c];
            const double ta = lane_shift_up(tb);
            // arrival times increase on the fast path: the interval holds grid points iff the
            // count of window grid points up to its end, clamp(floor(t) + 1, 0, n_obs), exceeds
            // that up to its start; with ta <= tb that is floor(tb) > floor(ta), floor(tb) >= 0
            // and floor(ta) <= n_obs - 2
            const double fb = floor(tb), fa = lane_shift_up(fb);
            const bool hit = iv && fb > fa && fb >= 0.0 && fa <= nob2;
            const uint64_t mask = __ballot(hit);
            if (mask) {
                d.push(hit, mask, (uint32_t)s, tag, ta, tb);
                d.pump();
            }
        }
    }

    // Scan of a fast-path particle over all its intervals (each pixel's next grid point is in pcl)
    template <int MODE>
    __device__ __forceinline__ void scan(int64_t k, const double *rk)
    {
        using SV = ScanVals<GEOM, F64, MODE>;
        constexpr int NV = SV::N;
        const int ns = (int)d.sh.n_samples;
        const int nq = (ns - 1 + 62) / 63;  // chunks (ns >= 2)
        const double nob = (double)d.sh.n_obs;
        double R[NB][NV], first[NB] = {};
        bool vr[NB];
        for (int q0 = 0; q0 < nq; q0 += NB) {
            // this block's records, all in before the pixel loop, so that no wait inside it also
            // waits for the drain's atomics; the next block's first values are loaded meanwhile
            // (a whole prefetched block would take registers that cost a wavefront per SIMD)
            load_block<MODE>(rk, q0, nq, R, vr, q0 > 0, first);
            mask_block<MODE>(R, vr);
            __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0)
            if (q0 + NB < nq) touch_block<MODE>(rk, q0 + NB, first);
            // the block's last sample: chunk c_last, lane l_last (uniform)
            const int s_last = std::min(63 * (q0 + NB), ns - 1);
            const int c_last = (s_last - 1) / 63 - q0;
            const int l_last = s_last - 63 * (q0 + c_last);
            // every pixel of the tile: one that takes no part (past the pass's last pixel, or its
            // geometry not usable) has next grid point +inf, so its arrival times never reach it
#pragma unroll
            for (int h = 0; h < kPPL; ++h) {
                cdptr row = uniform_ptr(d.pt + (size_t)(d.tile * kTilePix + 64 * h) * kPT);
                // o, px, py, g of the next pixel, read from LDS one iteration ahead (the same address
                // in every lane; one padding row past the tile's last pixel)
                double no = pcl[4 * (64 * h)], npx = pcl[4 * (64 * h) + 1], npy = pcl[4 * (64 * h) + 2],
                       ng = pcl[4 * (64 * h) + 3];
#pragma unroll 2
                for (int l = 0; l < 64; ++l, row += kPT) {
                    const int p = 64 * h + l;
                    PixC P;
                    const double g = ng;
                    if constexpr (MODE == kModeMixed) {
                        P = pixc_row(row);  // the whole geometry, scalar loads
                    } else {
                        P.o = no;
                        P.px = npx;
                        P.py = npy;
                        no = pcl[4 * (p + 1)];
                        npx = pcl[4 * (p + 1) + 1];
                        npy = pcl[4 * (p + 1) + 2];
                    }
                    ng = pcl[4 * (p + 1) + 3];
                    double t[NB];
                    tau_eval_block<GEOM, F64, MODE, NB>(P, R, d.cK, d.rb2, d.sh.C, t);
                    uint64_t any = 0;
#pragma unroll
                    for (int c = 0; c < NB; ++c) any |= __ballot(t[c] >= g);
                    if (__builtin_expect(any != 0, 0)) {  // rare: keep the scan's path straight
                        crossings(k, q0, nq, p, t);
                        double tl = t[0];
#pragma unroll
                        for (int c = 1; c < NB; ++c)
                            if (c_last == c) tl = t[c];
                        const double gn = next_grid(readlane_double(tl, l_last), nob);
                        if (d.lane == 0) pcl[4 * p + 3] = gn;
                    }
                }
            }
        }
    }

    // One fast-path particle: first and last arrival times per pixel (lanes over pixels), the
    // culling test (LW_CULL), the scan, and the counters, which follow from the two end points.
    template <int MODE, bool CULL>
    __device__ __forceinline__ void particle(int64_t k, const bool *pix_in, unsigned long long &c1,
                                             unsigned long long &c2, unsigned long long &c3)
    {
        using SV = ScanVals<GEOM, F64, MODE>;
        constexpr int NV = SV::N;
        const int ns = (int)d.sh.n_samples;
        const double nob = (double)d.sh.n_obs;
        const double *rk = d.rec + (size_t)k * d.sh.n_samples * Lay::W + SV::OFF;
        double tau0[kPPL], taul[kPPL];
        bool lane_ok[kPPL];
        {
            const cdptr a = uniform_ptr(rk), b = uniform_ptr(rk + (size_t)(ns - 1) * Lay::W);
            double v0[NV], v1[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                v0[v] = a[v];
                v1[v] = b[v];
            }
            // this lane's pixel constants, read again per particle (not held through the scan)
            const double *ptl = d.pt;
            asm volatile("" : "+s"(ptl));
#pragma unroll
            for (int h = 0; h < kPPL; ++h) {
                const PixC pc = pixc_row(ptl + (size_t)(d.tile * kTilePix + 64 * h + d.lane) * kPT);
                lane_ok[h] = (okmask[h] >> d.lane) & 1ull;
                tau0[h] = tau_eval<GEOM, F64, MODE>(pc, v0, d.cK, d.rb2, d.sh.C);
                taul[h] = tau_eval<GEOM, F64, MODE>(pc, v1, d.cK, d.rb2, d.sh.C);
            }
        }
        bool skip = false;
        if (CULL) {
            bool in = false;
#pragma unroll
            for (int h = 0; h < kPPL; ++h) in |= lane_ok[h] && grid_count(taul[h], nob) > grid_count(tau0[h], nob);
            skip = __ballot(in) == 0;
        }
        // the counters (taken before the scan, so that the end points are not held through it)
#pragma unroll
        for (int h = 0; h < kPPL; ++h) {
            if (lane_ok[h]) {
                const int64_t inside = grid_count(taul[h], nob) - grid_count(tau0[h], nob);
                c3 += (unsigned long long)inside;
                c2 += (unsigned long long)((int64_t)(floor(taul[h]) - floor(tau0[h])) - inside);
            } else if (pix_in[h]) {
                c1 += (unsigned long long)(ns - 1);
            }
        }
        if (!skip && ns >= 2) {
#pragma unroll
            for (int h = 0; h < kPPL; ++h) pcl[4 * (64 * h + d.lane) + 3] = lane_ok[h] ? next_grid(tau0[h], nob) : INFINITY;
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            scan<MODE>(k, rk);
        }
    }
};

template <typename T, int GEOM, bool CULL, int ACC>
__global__ __launch_bounds__(kBlockThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_scan(
    const double *__restrict__ r, const double *__restrict__ beta, const double *__restrict__ beta_dot,
    const double *__restrict__ charge, const double *__restrict__ x_det, const double *__restrict__ rec,
    const double *__restrict__ pt, const int *__restrict__ pflag, const unsigned long long *__restrict__ rmax2,
    const double *__restrict__ rbound2, T *__restrict__ E, unsigned long long *__restrict__ diag, DepShape sh, DetAcc det)
{
    constexpr bool kF64 = sizeof(T) == 8;
    constexpr int kRec = kF64 ? kModeRec5 : kModeRec3;
    __shared__ uint2 q_all[kQCap];
    __shared__ double2 qt_all[kQCap];
    __shared__ double pcl_all[4 * (kTilePix + 1)];
    __shared__ unsigned long long red[4];
    const int lane = threadIdx.x & 63;
    if (threadIdx.x < 4) red[threadIdx.x] = 0ull;
    __syncthreads();

    // block -> (particle group, tile); consecutive groups on one XCD share trajectory lines in L2
    const int64_t b = blockIdx.x;
    const int64_t xcd = b & 7, slot = b >> 3;
    const int64_t grp = (slot / sh.n_tiles) * 8 + xcd;
    const int64_t tile = slot % sh.n_tiles;
    const int64_t k0 = grp * sh.parts_per_group;
    const int64_t k1 = grp < sh.n_groups ? std::min(k0 + sh.parts_per_group, sh.n_particles) : k0;

    ScanWave<T, GEOM, ACC> w;
    Wave<T, GEOM, ACC> &d = w.d;
    bool pix_in[kPPL];
    double id2 = 0.0, s2 = 0.0;
    const double Dref = pix_geo(x_det, 0).D;  // the records' pixel distance
    bool far_off = false;                     // a pixel of this wavefront at another distance
#pragma unroll
    for (int h = 0; h < kPPL; ++h) {
        const int p = 64 * h + lane;
        const int64_t m = tile * kTilePix + p;
        pix_in[h] = m < sh.n_pix;
        // rows past the pass's last pixel are zero padding (not usable)
        const PixC pc = pixc_row(pt + m * kPT);
        const bool ok = pix_in[h] && pc.g.ok;
        w.okmask[h] = __ballot(ok);
        pcl_all[4 * p] = pc.o;
        pcl_all[4 * p + 1] = pc.px;
        pcl_all[4 * p + 2] = pc.py;
        pcl_all[4 * p + 3] = INFINITY;
        if (p < 4) pcl_all[4 * kTilePix + p] = p == 3 ? INFINITY : 0.0;
        if (ok) {
            id2 = fmax(id2, pc.g.invD * pc.g.invD);
            s2 = fmax(s2, 2.0 * (1.0 - pc.g.nz));
            far_off |= !(fabs(pc.g.D - Dref) <= kSameDistance * Dref);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        id2 = fmax(id2, __shfl_xor(id2, off));
        s2 = fmax(s2, __shfl_xor(s2, off));
    }
    const double invD2max = uniform_double(id2), s2max = uniform_double(s2);
    const bool rec_ok = GEOM == LW_GEOM_EXACT && __ballot(far_off) == 0;
    {
        double c[6];
        if (kF64)
            tau_poly<5>(0.0, 0.0, 0.0, 0.0, sh.C, Dref, c);
        else
            tau_poly<3>(0.0, 0.0, 0.0, 0.0, sh.C, Dref, c);
        d.cK = c[kF64 ? 5 : 3];
    }
    w.pcl = pcl_all;
    d.r = r;
    d.beta = beta;
    d.beta_dot = beta_dot;
    d.charge = charge;
    d.x_det = x_det;
    d.rec = rec;
    d.pt = pt;
    d.E = E;
    if constexpr (ACC != kAccFloat) d.det = det;
    d.sh = sh;
    d.lane = lane;
    d.tile = tile;
    d.k0 = k0;
    d.q = q_all;
    d.qt = qt_all;
    d.qh = 0;
    d.qn = 0;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();

    unsigned long long c1 = 0, c2 = 0, c3 = 0;
    for (int64_t k = k0; k < k1; ++k) {
        if (pflag[k] != 0) continue;  // careful path: k_careful
        // series forms where |r|^2 <= 1e-8 |x_m|^2 over the whole trajectory (the max over the
        // whole trajectory when given, else over the samples of this call), decided per pixel
        d.rb2 = rbound2 ? rbound2[k] : __longlong_as_double((long long)rmax2[k]);
        const bool all_ser = GEOM == LW_GEOM_EXACT && d.rb2 * invD2max <= kSeriesBound;
        if (GEOM == LW_GEOM_FARFIELD)
            w.template particle<kModeFar, CULL>(k, pix_in, c1, c2, c3);
        else if (all_ser && rec_ok) {
            if (tail_negligible<kF64>(d.rb2, s2max, sh.C, d.cK, Dref))
                w.template particle<kModeRecLow, CULL>(k, pix_in, c1, c2, c3);
            else
                w.template particle<kRec, CULL>(k, pix_in, c1, c2, c3);
        } else
            w.template particle<kModeMixed, CULL>(k, pix_in, c1, c2, c3);
    }
    while (d.qn > 0) d.drain(d.qn < 64 ? d.qn : 64);

    // counters: block reduction in LDS, then one global atomic per counter
    if (c1) atomicAdd(&red[1], c1);
    if (c2) atomicAdd(&red[2], c2);
    if (c3) atomicAdd(&red[3], c3);
    __syncthreads();
    if (diag && threadIdx.x < 4 && red[threadIdx.x]) atomicAdd(diag + threadIdx.x, red[threadIdx.x]);
}

// Row scales of the fixed-point pass from the first pass's max |v| per element (bits of a
// non-negative double): scale = 2^(62 - e) where max < 2^e, so every |v| * scale < 2^62.  A row
// that received nothing takes 1; a row with a non-finite contribution takes NaN and is NaN in the
// result.
__global__ __launch_bounds__(256) void k_det_scale(const unsigned long long *__restrict__ mx, int64_t n_rows,
                                                   int64_t n_obs, double *__restrict__ scale)
{
    __shared__ unsigned long long red[256];
    for (int64_t row = blockIdx.x; row < n_rows; row += gridDim.x) {
        const unsigned long long *p = mx + (size_t)row * (size_t)n_obs;
        unsigned long long v = 0;
        for (int64_t u = threadIdx.x; u < n_obs; u += 256) v = p[u] > v ? p[u] : v;
        red[threadIdx.x] = v;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h && red[threadIdx.x + h] > red[threadIdx.x]) red[threadIdx.x] = red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const double M = __longlong_as_double((long long)red[0]);
            double sc = 1.0;
            if (!isfinite(M)) {
                sc = NAN;
            } else if (M > 0.0) {
                int e;
                frexp(M, &e);
                sc = ldexp(1.0, 62 - e < 1023 ? 62 - e : 1023);
            }
            scale[row] = sc;
        }
        __syncthreads();
    }
}

// The 128-bit sums (low words in E, high words in hi) to doubles, in place, then divided by the
// row's power of two.  A sum that fits in 64 bits converts with one rounding; a larger one is
// hi 2^64 + lo through the fma, where the rounding of lo (at most 2^10) is at most half an ulp of
// the result (|result| >= 2^63): at most one ulp in all.
__global__ __launch_bounds__(256) void k_det_finish(double *__restrict__ E, const unsigned long long *__restrict__ hi,
                                                    const double *__restrict__ scale, int64_t n_rows, int64_t n_obs)
{
    const size_t n = (size_t)n_rows * (size_t)n_obs;
    for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < n; j += (size_t)gridDim.x * blockDim.x) {
        const double sc = scale[j / (size_t)n_obs];
        const unsigned long long lo = (unsigned long long)__double_as_longlong(E[j]);
        const long long h = (long long)hi[j], sl = (long long)lo;
        const double v = h == (sl < 0 ? -1ll : 0ll) ? (double)sl : fma((double)h, 0x1p64, (double)lo);
        E[j] = isnan(sc) ? NAN : v * (1.0 / sc);
    }
}

template <int GEOM>
void launch_prepass(bool f64, dim3 grid, hipStream_t s, const double *r, const double *b, const double *bd,
                    const double *x_det, int64_t ns, int64_t sample0, double t_start, double dt, double t0,
                    double dt_obs, double C, const DepWs &w)
{
    if (f64)
        k_prepass<GEOM, 5><<<grid, 256, 0, s>>>(r, b, bd, x_det, ns, sample0, t_start, dt, t0, dt_obs, C, w.rec,
                                               w.pflag, w.rmax2);
    else
        k_prepass<GEOM, 3><<<grid, 256, 0, s>>>(r, b, bd, x_det, ns, sample0, t_start, dt, t0, dt_obs, C, w.rec,
                                               w.pflag, w.rmax2);
}

}  // namespace

size_t det_acc_bytes(int64_t n_pix, int64_t n_obs)
{
    return align_up((size_t)n_pix * 3 * (size_t)n_obs * 8, 256) + align_up((size_t)n_pix * 3 * 8, 256);
}

// Two deposits with the same per-contribution values: the first finds max |v| per trace element,
// the second adds the contributions as 128-bit fixed-point integers scaled per row by the first's
// maximum; the integer sums do not depend on the order in which the atomics land.
lw_status launch_deposit_det(const lw_traj_t *t, const lw_grid_t *gr, int fmask, int geom, double *E, int64_t *diag,
                             void *acc, void *ws, size_t ws_bytes, hipStream_t s)
{
    const int64_t rows = gr->n_pix * 3, n_obs = gr->n_obs;
    const size_t n_el = (size_t)rows * (size_t)n_obs;
    double *scale = (double *)((char *)acc + align_up(n_el * 8, 256));
    const DetAcc det{(unsigned long long *)acc, scale};
    const bool boris = t->kind == LW_TRAJ_BORIS;
    auto pass = [&](int mode, int64_t *dg) {
        return boris ? launch_deposit_boris(t, gr, LW_PREC_FP64, fmask, geom, false, E, dg, ws, ws_bytes, s, mode, det)
                     : launch_deposit(t, gr, LW_PREC_FP64, fmask, geom, false, E, dg, ws, ws_bytes, s, 0, nullptr, mode,
                                      det);
    };
    if (n_el == 0) return pass(kAccFixed, diag);  // nothing to deposit: the diag reset only
    lw_status st = pass(kAccMaxAbs, nullptr);
    if (st != LW_OK) return st;
    k_det_scale<<<(unsigned)std::min<int64_t>(rows, 65536), 256, 0, s>>>((const unsigned long long *)E, rows, n_obs,
                                                                        scale);
    const unsigned blocks = (unsigned)std::min<size_t>((n_el + 255) / 256, 65536);
    k_fill<unsigned long long><<<blocks, 256, 0, s>>>(det.hi, (int64_t)n_el);
    if ((st = check_launch("lw_deposit_td_det")) != LW_OK) return st;
    if ((st = pass(kAccFixed, diag)) != LW_OK) return st;
    k_det_finish<<<blocks, 256, 0, s>>>(E, det.hi, scale, rows, n_obs);
    return check_launch("lw_deposit_td_det");
}

size_t deposit_ws_bytes(int64_t n_particles, int64_t n_samples, int prec)
{
    return ws_bytes_for(n_particles, n_samples, rec_width(LW_GEOM_EXACT, prec == LW_PREC_FP64));
}

lw_status launch_deposit(const lw_traj_t *t, const lw_grid_t *gr, int prec, int fmask, int geom, bool accumulate,
                         void *E, int64_t *diag, void *ws, size_t ws_bytes, hipStream_t s, int64_t sample0,
                         const double *rbound2, int acc_mode, DetAcc det)
{
    const int64_t n_p = t->n_particles, ns = t->n_samples, n_pix = gr->n_pix, n_obs = gr->n_obs;
    const bool cull = (geom & LW_CULL) != 0;
    geom &= ~LW_CULL;
    const size_t trace_elems = (size_t)n_pix * 3 * (size_t)n_obs;
    const bool f64 = prec == LW_PREC_FP64;
    if (acc_mode != kAccFloat && (!f64 || cull))
        return fail(LW_E_UNSUPPORTED, "lw_deposit_td_det: FP64 without culling only");
    if (n_obs > 0x7fffffff) return fail(LW_E_SHAPE, "lw_deposit_td: n_obs must be below 2^31");
    if (ns > 0x7fffffff) return fail(LW_E_SHAPE, "lw_deposit_td: too many samples");
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
    const int rw = rec_width(geom, f64);
    // particles per launch: all of them, or as many as the workspace holds records for
    int64_t chunk = n_p;
    while (chunk > 1 && ws_bytes_for(chunk, ns, rw) > ws_bytes) chunk = std::max<int64_t>(1, chunk / 2);
    if (ws_bytes_for(chunk, ns, rw) > ws_bytes)
        return fail(LW_E_WORKSPACE, "lw_deposit_td: workspace of %zu bytes holds no particle (%zu needed)", ws_bytes,
                    ws_bytes_for(1, ns, rw));
    const double C = 1.0 / (kC * gr->dt_obs);
    const int64_t n_chunks_s = (ns + kPrepassChunk - 1) / kPrepassChunk;
    if (n_chunks_s > 65535) return fail(LW_E_SHAPE, "lw_deposit_td: too many samples");
    // pixel passes of at most kPixTabMax pixels (the pixel table's share of the workspace); each
    // pass is a deposit of its own pixels (records take the pass's first pixel as reference)
    for (int64_t m0 = 0; m0 < n_pix; m0 += kPixTabMax) {
        const int64_t npx = std::min<int64_t>(kPixTabMax, n_pix - m0);
        const double *xd = gr->x_det + 3 * m0;
        void *Ep = f64 ? (void *)((double *)E + (size_t)m0 * 3 * (size_t)n_obs)
                       : (void *)((float *)E + (size_t)m0 * 3 * (size_t)n_obs);
        // the pass's rows of the order-independent accumulators
        const DetAcc dp{det.hi ? det.hi + (size_t)m0 * 3 * (size_t)n_obs : nullptr,
                        det.scale ? det.scale + (size_t)m0 * 3 : nullptr};
        for (int64_t p0 = 0; p0 < n_p; p0 += chunk) {
            const int64_t np = std::min<int64_t>(chunk, n_p - p0);
            DepShape sh;
            sh.n_particles = np;
            sh.n_samples = ns;
            sh.n_pix = npx;
            sh.n_obs = n_obs;
            sh.n_tiles = (npx + kTilePix - 1) / kTilePix;
            int64_t groups = std::max<int64_t>(1, (kTargetWaves + sh.n_tiles - 1) / sh.n_tiles);
            groups = std::max<int64_t>(groups, (np + kMaxPartsPerGroup - 1) / kMaxPartsPerGroup);
            groups = std::max<int64_t>(1, std::min<int64_t>(groups, np));
            sh.parts_per_group = std::max<int64_t>(1, (np + groups - 1) / groups);
            sh.n_groups = (np + sh.parts_per_group - 1) / sh.parts_per_group;
            sh.fmask = fmask;
            sh.C = C;
            const int64_t blocks = (sh.n_groups + 7) / 8 * 8 * sh.n_tiles;
            if (sh.parts_per_group >= (int64_t(1) << (32 - kPixBits)))
                return fail(LW_E_SHAPE, "lw_deposit_td: too many particles per pixel tile group");
            if (np > 0x7fffffff) return fail(LW_E_SHAPE, "lw_deposit_td: too many particles");
            if (blocks > 0x7fffffff) return fail(LW_E_SHAPE, "lw_deposit_td: problem too large for one launch");
            const DepWs w = carve(ws, np);
            if (p0 == 0) {
                const int64_t rows = sh.n_tiles * kTilePix;  // <= kPixTabMax
                k_pixtab<<<(unsigned)((rows + 255) / 256), 256, 0, s>>>(xd, npx, rows, C, w.pt);
            }
            const double *r = t->r + (size_t)p0 * ns * 3, *b = t->beta + (size_t)p0 * ns * 3,
                         *bd = t->beta_dot + (size_t)p0 * ns * 3;
            const double *charge = t->charge ? t->charge + p0 : nullptr;
            const double *rb2 = rbound2 ? rbound2 + p0 : nullptr;
            const int fill_blocks = (int)std::min<int64_t>((np + 255) / 256, 65536);
            k_fill<int><<<fill_blocks, 256, 0, s>>>(w.pflag, np);
            k_fill<unsigned long long><<<fill_blocks, 256, 0, s>>>(w.rmax2, np);
            const dim3 pgrid((unsigned)np, (unsigned)n_chunks_s);
            if (geom == LW_GEOM_EXACT)
                launch_prepass<LW_GEOM_EXACT>(f64, pgrid, s, r, b, bd, xd, ns, sample0, t->t_start, t->dt, gr->t0,
                                              gr->dt_obs, C, w);
            else
                launch_prepass<LW_GEOM_FARFIELD>(f64, pgrid, s, r, b, bd, xd, ns, sample0, t->t_start, t->dt, gr->t0,
                                                 gr->dt_obs, C, w);
            unsigned long long *dg = (unsigned long long *)diag;
            const dim3 grid((unsigned)blocks), block(kBlockThreads);
            if (acc_mode != kAccFloat) {
#define LW_DET_LAUNCH(G, A)                                                                                          \
    do {                                                                                                             \
        k_scan<double, G, false, A><<<grid, block, 0, s>>>(r, b, bd, charge, xd, w.rec, w.pt, w.pflag, w.rmax2, rb2,  \
                                                           (double *)Ep, dg, sh, dp);                                \
        k_careful<double, G, A><<<grid, block, 0, s>>>(r, b, bd, charge, xd, w.rec, w.pt, w.pflag, w.rmax2, rb2,      \
                                                       (double *)Ep, dg, sh, dp);                                    \
    } while (0)
                if (geom == LW_GEOM_EXACT) {
                    if (acc_mode == kAccMaxAbs) LW_DET_LAUNCH(LW_GEOM_EXACT, kAccMaxAbs); else LW_DET_LAUNCH(LW_GEOM_EXACT, kAccFixed);
                } else {
                    if (acc_mode == kAccMaxAbs) LW_DET_LAUNCH(LW_GEOM_FARFIELD, kAccMaxAbs); else LW_DET_LAUNCH(LW_GEOM_FARFIELD, kAccFixed);
                }
#undef LW_DET_LAUNCH
                const lw_status st = check_launch("lw_deposit_td_det");
                if (st != LW_OK) return st;
                continue;
            }
            // the fast path (timed as the deposit kernel), then the careful path; culling is a
            // separate instantiation of the fast path, so the full evaluation carries none of its code
#define LW_SCAN_LAUNCH(T, G, CU)                                                                                  \
    k_scan<T, G, CU, kAccFloat><<<grid, block, 0, s>>>(r, b, bd, charge, xd, w.rec, w.pt, w.pflag, w.rmax2, rb2,      \
                                                       (T *)Ep, dg, sh, DetAcc{nullptr, nullptr})
#define LW_CAREFUL_LAUNCH(T, G)                                                                                   \
    k_careful<T, G, kAccFloat><<<grid, block, 0, s>>>(r, b, bd, charge, xd, w.rec, w.pt, w.pflag, w.rmax2, rb2,       \
                                                      (T *)Ep, dg, sh, DetAcc{nullptr, nullptr})
            hipEvent_t ev = timing_begin(LW_KERNEL_DEPOSIT, s);
            if (f64) {
                if (geom == LW_GEOM_EXACT) {
                    if (cull) LW_SCAN_LAUNCH(double, LW_GEOM_EXACT, true); else LW_SCAN_LAUNCH(double, LW_GEOM_EXACT, false);
                } else {
                    if (cull) LW_SCAN_LAUNCH(double, LW_GEOM_FARFIELD, true); else LW_SCAN_LAUNCH(double, LW_GEOM_FARFIELD, false);
                }
            } else {
                if (geom == LW_GEOM_EXACT) {
                    if (cull) LW_SCAN_LAUNCH(float, LW_GEOM_EXACT, true); else LW_SCAN_LAUNCH(float, LW_GEOM_EXACT, false);
                } else {
                    if (cull) LW_SCAN_LAUNCH(float, LW_GEOM_FARFIELD, true); else LW_SCAN_LAUNCH(float, LW_GEOM_FARFIELD, false);
                }
            }
            timing_end(LW_KERNEL_DEPOSIT, ev, s);
            if (f64) {
                if (geom == LW_GEOM_EXACT) LW_CAREFUL_LAUNCH(double, LW_GEOM_EXACT); else LW_CAREFUL_LAUNCH(double, LW_GEOM_FARFIELD);
            } else {
                if (geom == LW_GEOM_EXACT) LW_CAREFUL_LAUNCH(float, LW_GEOM_EXACT); else LW_CAREFUL_LAUNCH(float, LW_GEOM_FARFIELD);
            }
#undef LW_SCAN_LAUNCH
#undef LW_CAREFUL_LAUNCH
            const lw_status st = check_launch("lw_deposit_td");
            if (st != LW_OK) return st;
        }
    }
    return LW_OK;
}

}  // namespace lw
