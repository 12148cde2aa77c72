// |E(w)|^2 of every pixel trace on the FFT bins (Eq. efield_xfrom, rectangle rule).
//
// Packing: the three real components of a pixel pair (m, m+1) go into three complex
// sequences of length N:
//   Z0 = Ex_m + i Ey_m,   Z1 = Ex_{m+1} + i Ey_{m+1},   Z2 = Ez_m + i Ez_{m+1}.
// For real a, b with Z = a + i b:  A_j = (Z_j + conj Z_{N-j})/2,  B_j = (Z_j - conj Z_{N-j})/(2i),
// so |A_j|^2 + |B_j|^2 = (|Z_j|^2 + |Z_{N-j}|^2)/2.  Each pixel needs 1.5 complex transforms.
//
// Four-step transform, N = N1 * N2, n = N2 n1 + n2, k = k1 + N1 k2:
//   pass A ("columns"): Y[k1][n2] = W_N^{n2 k1} sum_{n1} x[N2 n1 + n2] W_N1^{n1 k1}
//   pass B ("rows"):    X[k1 + N1 k2] = sum_{n2} Y[k1][n2] W_N2^{n2 k2}
// Pass B handles rows k1 and N1 - k1 together, which hold X_j and X_{N-j}, and writes
// S_j for j <= N/2 directly.
//
// Forward path: rows are L = 4096 points (FP32) or 2048 (FP64), so N1 = N / L is small (64 for
// N = 2^18) and pass A reads C = 4096/N1 (2048/N1) adjacent columns: rows of 256 bytes.
// Sub-transforms are Stockham passes of radix 16 (FP32) or 8 (FP64), each butterfly held by one
// thread in registers between two barriers of an LDS exchange; the first pass takes the loaded
// registers and the last leaves its outputs in registers (k_fwd_cols_fast, k_fwd_rows_fast, all
// shapes fixed at compile time).  The trace scale dt_obs / sqrt(2 pi) rides on pass A's twiddles.
// Pass B writes the spectrum at a stride of N1 elements; all its blocks of one pixel pair run on
// one XCD so that those partial lines merge in its L2.  For N <= L one kernel reads the traces
// (k_fwd_row_direct), and columns longer than 256 points take the runtime-shaped k_fwd_cols.
//
// Adjoint path: N1 = 2^ceil(lg/2), N2 = 2^floor(lg/2), radix-4 Stockham passes between two
// LDS buffers.
#include "lw_internal.h"

#include <algorithm>
#include <cmath>
#include <mutex>

// Scratch of lw_spectrum_fft_noalloc: a fixed device array that every GPU the library runs on
// holds from the load of the code object until the process ends.  In host code the name is
// only a stand-in for the symbol; its device address (one per GPU) comes from
// hipGetSymbolAddress and is the only form in which host code uses it.
constexpr size_t kNoallocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace lw {
namespace {

template <typename T>
struct C2;
template <>
struct C2<float> {
    using type = float2;
};
template <>
struct C2<double> {
    using type = double2;
};

template <typename T2>
__device__ __forceinline__ T2 cmul(T2 a, T2 b)
{
    T2 r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}

__device__ __forceinline__ double2 unit_phasor(double minus_two_frac)  // exp(i pi * arg)
{
    double s, c;
    sincospi(minus_two_frac, &s, &c);
    return make_double2(c, s);
}
__device__ __forceinline__ float2 unit_phasor_f(float arg)
{
    float s, c;
    sincospif(arg, &s, &c);
    return make_float2(c, s);
}

template <typename T2>
__device__ __forceinline__ T2 twiddle(int64_t q, int64_t L);  // exp(-2 pi i q / L), 0 <= q < L
template <>
__device__ __forceinline__ double2 twiddle<double2>(int64_t q, int64_t L)
{
    return unit_phasor(-2.0 * (double)q / (double)L);
}
template <>
__device__ __forceinline__ float2 twiddle<float2>(int64_t q, int64_t L)
{
    // reduce to (-1, 1] before the float call so that the argument is exact
    int64_t qq = q * 2;
    if (qq > L) qq -= 2 * L;
    return unit_phasor_f(-(float)((double)qq / (double)L));
}

template <int R, typename T2>
__device__ __forceinline__ void dft(T2 *v)
{
    if (R == 2) {
        T2 a = v[0], b = v[1];
        v[0].x = a.x + b.x;
        v[0].y = a.y + b.y;
        v[1].x = a.x - b.x;
        v[1].y = a.y - b.y;
    } else {
        T2 a0, a1, a2, a3;
        a0.x = v[0].x + v[2].x;
        a0.y = v[0].y + v[2].y;
        a1.x = v[0].x - v[2].x;
        a1.y = v[0].y - v[2].y;
        a2.x = v[1].x + v[3].x;
        a2.y = v[1].y + v[3].y;
        // (v1 - v3) * (-i)
        a3.x = v[1].y - v[3].y;
        a3.y = -(v[1].x - v[3].x);
        v[0].x = a0.x + a2.x;
        v[0].y = a0.y + a2.y;
        v[2].x = a0.x - a2.x;
        v[2].y = a0.y - a2.y;
        v[1].x = a1.x + a3.x;
        v[1].y = a1.y + a3.y;
        v[3].x = a1.x - a3.x;
        v[3].y = a1.y - a3.y;
    }
}

// One Stockham pass of radix R over nseq sequences of length L = 2^lg (sequence s at in + s*stride).
template <int R, typename T2>
__device__ __forceinline__ void stage(const T2 *in, T2 *out, int lg, int Ns, int nseq, int stride, const T2 *tw,
                                      int tid, int nthr)
{
    const int L = 1 << lg;
    const int nb = L / R;
    const int lgnb = lg - (R == 4 ? 2 : 1);
    const int twstep = L / (Ns * R);
    for (int b = tid; b < nseq * nb; b += nthr) {
        const int s = b >> lgnb, j = b & (nb - 1);
        const T2 *src = in + s * stride;
        T2 v[R];
        const int k = j & (Ns - 1);
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = src[j + r * nb];
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[r * k * twstep]);
        dft<R>(v);
        const int d = (j - k) * R + k;
        T2 *dst = out + s * stride;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[d + r * Ns] = v[r];
    }
}

// Forward DFT (exp(-i)) of nseq sequences in LDS; returns the buffer that holds the result.
template <typename T2>
__device__ T2 *lds_fft(T2 *a, T2 *b, int lg, int nseq, int stride, const T2 *tw, int tid, int nthr)
{
    int Ns = 1;
    if (lg & 1) {
        stage<2>(a, b, lg, Ns, nseq, stride, tw, tid, nthr);
        T2 *t = a;
        a = b;
        b = t;
        Ns = 2;
        __syncthreads();
    }
    while (Ns < (1 << lg)) {
        stage<4>(a, b, lg, Ns, nseq, stride, tw, tid, nthr);
        T2 *t = a;
        a = b;
        b = t;
        Ns *= 4;
        __syncthreads();
    }
    return a;
}

struct FftShape {
    int64_t n_pix, pair0;
    int lg1, lg2, C;
};

template <typename T>
__device__ __forceinline__ void pair_pointers(const T *E, int64_t n_pix, int64_t p, int t, int64_t N, const T *&re,
                                              const T *&im)
{
    const int64_t m = 2 * p, m1 = 2 * p + 1;
    const bool has1 = m1 < n_pix;
    if (t == 0) {
        re = E + (m * 3 + 0) * N;
        im = E + (m * 3 + 1) * N;
    } else if (t == 1) {
        re = has1 ? E + (m1 * 3 + 0) * N : nullptr;
        im = has1 ? E + (m1 * 3 + 1) * N : nullptr;
    } else {
        re = E + (m * 3 + 2) * N;
        im = has1 ? E + (m1 * 3 + 2) * N : nullptr;
    }
}

// ---------------------------------------------------------------------------------------------
// Forward path (register-staged Stockham passes in one LDS buffer)

template <typename T>
struct FwdCfg;
template <>
struct FwdCfg<float> {
    static constexpr int kLgRow = 12;  // rows of up to 4096 points
    static constexpr int kET = 16;     // elements per thread
    static constexpr int kLgRadix = 4;
    static constexpr int kPadShift = 4;  // one pad element per 16 (128 bytes)
};
template <>
struct FwdCfg<double> {
    static constexpr int kLgRow = 11;
    static constexpr int kET = 8;
    static constexpr int kLgRadix = 3;
    static constexpr int kPadShift = 3;
};
constexpr int kThrA = 256, kThrB = 512;

template <typename T2>
__device__ __forceinline__ T2 cadd(T2 a, T2 b)
{
    a.x += b.x;
    a.y += b.y;
    return a;
}
template <typename T2>
__device__ __forceinline__ T2 csub(T2 a, T2 b)
{
    a.x -= b.x;
    a.y -= b.y;
    return a;
}
template <typename T2>
__device__ __forceinline__ T2 mul_mi(T2 a)  // a * (-i)
{
    T2 r;
    r.x = a.y;
    r.y = -a.x;
    return r;
}

// a * W_16^M, W_16 = exp(-2 pi i / 16), 0 <= M < 16, exact special cases
template <int M, typename T2>
__device__ __forceinline__ T2 w16mul(T2 a)
{
    using T = decltype(a.x);
    constexpr double c1 = 0.92387953251128675613, s1 = 0.38268343236508977173, h = 0.70710678118654752440;
    constexpr int m = M & 15;
    if constexpr (m == 0) {
        return a;
    } else if constexpr (m == 4) {
        return mul_mi(a);
    } else if constexpr (m == 8) {
        a.x = -a.x;
        a.y = -a.y;
        return a;
    } else if constexpr (m == 12) {
        T2 r;
        r.x = -a.y;
        r.y = a.x;
        return r;
    } else {
        constexpr double cs[16] = {1, c1, h, s1, 0, -s1, -h, -c1, -1, -c1, -h, -s1, 0, s1, h, c1};
        constexpr double sn[16] = {0, s1, h, c1, 1, c1, h, s1, 0, -s1, -h, -c1, -1, -c1, -h, -s1};
        const T wr = (T)cs[m], wi = (T)(-sn[m]);  // exp(-2 pi i m/16)
        T2 r;
        r.x = a.x * wr - a.y * wi;
        r.y = a.x * wi + a.y * wr;
        return r;
    }
}

template <typename T2>
__device__ __forceinline__ void dft4v(T2 &v0, T2 &v1, T2 &v2, T2 &v3)
{
    const T2 a0 = cadd(v0, v2), a1 = csub(v0, v2), a2 = cadd(v1, v3), a3 = mul_mi(csub(v1, v3));
    v0 = cadd(a0, a2);
    v2 = csub(a0, a2);
    v1 = cadd(a1, a3);
    v3 = csub(a1, a3);
}

// in-place DFT of R points, natural order in and out: X[k] = sum_r v[r] exp(-2 pi i r k / R)
template <int R, typename T2>
__device__ __forceinline__ void dftR(T2 *v)
{
    if constexpr (R == 2) {
        const T2 a = v[0];
        v[0] = cadd(a, v[1]);
        v[1] = csub(a, v[1]);
    } else if constexpr (R == 4) {
        dft4v(v[0], v[1], v[2], v[3]);
    } else if constexpr (R == 8) {
        // inner 4-point DFTs over v[2b + a], twiddle W_8^{a k1}, outer 2-point over a
        dft4v(v[0], v[2], v[4], v[6]);
        dft4v(v[1], v[3], v[5], v[7]);
        v[3] = w16mul<2>(v[3]);
        v[5] = w16mul<4>(v[5]);
        v[7] = w16mul<6>(v[7]);
        T2 x[8];
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            x[k1] = cadd(v[2 * k1], v[2 * k1 + 1]);
            x[k1 + 4] = csub(v[2 * k1], v[2 * k1 + 1]);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = x[q];
    } else {
        static_assert(R == 16, "radix 2, 4, 8 or 16");
        // inner 4-point DFTs over v[4b + a] (result k1 at v[4 k1 + a]), twiddle W_16^{a k1},
        // outer 4-point DFTs over a, X[k1 + 4 k2]
        dft4v(v[0], v[4], v[8], v[12]);
        dft4v(v[1], v[5], v[9], v[13]);
        dft4v(v[2], v[6], v[10], v[14]);
        dft4v(v[3], v[7], v[11], v[15]);
        v[5] = w16mul<1>(v[5]);
        v[6] = w16mul<2>(v[6]);
        v[7] = w16mul<3>(v[7]);
        v[9] = w16mul<2>(v[9]);
        v[10] = w16mul<4>(v[10]);
        v[11] = w16mul<6>(v[11]);
        v[13] = w16mul<3>(v[13]);
        v[14] = w16mul<6>(v[14]);
        v[15] = w16mul<9>(v[15]);
        T2 x[16];
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            T2 a0 = v[4 * k1], a1 = v[4 * k1 + 1], a2 = v[4 * k1 + 2], a3 = v[4 * k1 + 3];
            dft4v(a0, a1, a2, a3);
            x[k1] = a0;
            x[k1 + 4] = a1;
            x[k1 + 8] = a2;
            x[k1 + 12] = a3;
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = x[q];
    }
}

// W_4096^Q for 0 <= Q < 4096 from the two tables (tlo[b] = W_4096^b, thi[a] = W_64^a)
template <typename T2>
__device__ __forceinline__ T2 tw4096(int Q, const T2 *tlo, const T2 *thi)
{
    return cmul(thi[Q >> 6], tlo[Q & 63]);
}

template <typename T2>
__device__ __forceinline__ void build_tables(T2 *tlo, T2 *thi, int tid)
{
    if (tid < 64)
        tlo[tid] = twiddle<T2>(tid, 4096);
    else if (tid < 128)
        thi[tid - 64] = twiddle<T2>(tid - 64, 64);
}

// Column layout (pass A): element e of sequence s at e * C + s; consecutive butterflies
// take consecutive sequences.
struct LayCols {
    int lgC;
    __device__ __forceinline__ int addr(int s, int e) const { return (e << lgC) + s; }
    __device__ __forceinline__ void split(int b, int lgNb, int &s, int &j) const
    {
        s = b & ((1 << lgC) - 1);
        j = b >> lgC;
    }
};
// Row layout (pass B): element e of sequence s at s * L + e with one pad element every
// 2^PS; consecutive butterflies take consecutive positions of one sequence.
template <int PS>
struct LayRows {
    int lgL;
    __device__ __forceinline__ int addr(int s, int e) const
    {
        const int a = (s << lgL) + e;
        return a + (a >> PS);
    }
    __device__ __forceinline__ void split(int b, int lgNb, int &s, int &j) const
    {
        j = b & ((1 << lgNb) - 1);
        s = b >> lgNb;
    }
};

// One radix-R Stockham pass over nseq sequences of 2^lgL points, Ns = 2^lgNs: butterfly j
// reads e = j + r L/R, multiplies by W_{Ns R}^{r k} (k = j mod Ns), transforms, and writes
// (j - k) R + k + r Ns.  Each thread holds ET/R butterflies between the two barriers.
template <int R, int ET, typename T2, typename Lay>
__device__ __forceinline__ void stockham_pass(T2 *buf, const Lay &lay, int lgL, int lgNs, int nseq, const T2 *tlo,
                                              const T2 *thi, int tid, int nthr)
{
    constexpr int NB = ET / R;
    constexpr int lgR = R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4;
    const int lgNb = lgL - lgR;
    const int total = nseq << lgNb;
    T2 v[NB][R];
    int sj[NB][2];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int b = tid + i * nthr;
        int sq = -1, j = 0;
        if (b < total) lay.split(b, lgNb, sq, j);
        sj[i][0] = sq;
        sj[i][1] = j;
        if (sq >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[i][r] = buf[lay.addr(sq, j + (r << lgNb))];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const int sq = sj[i][0], j = sj[i][1];
        if (sq < 0) continue;
        const int k = j & ((1 << lgNs) - 1);
        if (lgNs > 0) {
            // W_{Ns R}^{r k} = W_4096^{r k 4096/(Ns R)}; powers 1, 2, 4, 8 from the tables,
            // the others as one product of two of them
            const int sh = 12 - lgNs - lgR;
            T2 w[R];
            w[1] = tw4096((k << sh) & 4095, tlo, thi);
            if constexpr (R >= 4) {
                w[2] = tw4096((2 * k << sh) & 4095, tlo, thi);
                w[3] = cmul(w[1], w[2]);
            }
            if constexpr (R >= 8) {
                w[4] = tw4096((4 * k << sh) & 4095, tlo, thi);
                w[5] = cmul(w[1], w[4]);
                w[6] = cmul(w[2], w[4]);
                w[7] = cmul(w[3], w[4]);
            }
            if constexpr (R >= 16) {
                w[8] = tw4096((8 * k << sh) & 4095, tlo, thi);
#pragma unroll
                for (int r = 9; r < 16; ++r) w[r] = cmul(w[r - 8], w[8]);
            }
#pragma unroll
            for (int r = 1; r < R; ++r) v[i][r] = cmul(v[i][r], w[r]);
        }
        dftR<R>(v[i]);
        const int d = ((j - k) << lgR) + k;
#pragma unroll
        for (int r = 0; r < R; ++r) buf[lay.addr(sq, d + (r << lgNs))] = v[i][r];
    }
    __syncthreads();
}

// Forward DFT in place of nseq sequences of 2^lgL points (2^lgL <= 4096): the remainder
// radix first (no twiddles), then radix 2^LGR passes.
template <int ET, int LGR, typename T2, typename Lay>
__device__ __forceinline__ void fft_inplace(T2 *buf, const Lay &lay, int lgL, int nseq, const T2 *tlo, const T2 *thi, int tid,
                            int nthr)
{
    int lgNs = 0;
    const int rem = lgL % LGR;
    if (rem == 1) {
        stockham_pass<2, ET>(buf, lay, lgL, lgNs, nseq, tlo, thi, tid, nthr);
        lgNs = 1;
    } else if (rem == 2) {
        stockham_pass<4, ET>(buf, lay, lgL, lgNs, nseq, tlo, thi, tid, nthr);
        lgNs = 2;
    } else if (rem == 3) {
        stockham_pass<8, ET>(buf, lay, lgL, lgNs, nseq, tlo, thi, tid, nthr);
        lgNs = 3;
    }
    while (lgNs < lgL) {
        stockham_pass<(1 << LGR), ET>(buf, lay, lgL, lgNs, nseq, tlo, thi, tid, nthr);
        lgNs += LGR;
    }
}

struct FwdShape {
    int64_t n_pix, pair0, nbatch;
    int lg, lg1, lg2, lgC;
};

// pass A: C adjacent columns of one packed transform of one pixel pair per block
template <typename T>
__global__ __launch_bounds__(kThrA) void k_fwd_cols(const T *__restrict__ E, typename C2<T>::type *__restrict__ Y,
                                                    FwdShape sh, T sc)
{
    using T2 = typename C2<T>::type;
    using Cfg = FwdCfg<T>;
    constexpr int EL = Cfg::kET * kThrA;  // C * N1
    __shared__ T2 buf[EL];
    __shared__ T2 tlo[64], thi[64];
    const int tid = threadIdx.x;
    const int lgC = sh.lgC, C = 1 << lgC;
    const int64_t N = (int64_t)1 << sh.lg;
    const int t = blockIdx.y;
    const int64_t pl = blockIdx.z, p = sh.pair0 + pl;
    const T *re, *im;
    pair_pointers(E, sh.n_pix, p, t, N, re, im);
    if (!re) return;  // transform of a missing pixel: pass B skips it too
    const int c0 = blockIdx.x * C;
    build_tables(tlo, thi, tid);
#pragma unroll
    for (int i = 0; i < Cfg::kET; ++i) {
        const int idx = tid + i * kThrA;
        const int n1 = idx >> lgC, c = idx & (C - 1);
        const int64_t n = ((int64_t)n1 << sh.lg2) + c0 + c;
        T2 v;
        v.x = re[n];
        v.y = im ? im[n] : (T)0;
        buf[idx] = v;
    }
    __syncthreads();
    const LayCols lay{lgC};
    fft_inplace<Cfg::kET, Cfg::kLgRadix>(buf, lay, sh.lg1, C, tlo, thi, tid, kThrA);
    T2 *Yt = Y + (pl * 3 + t) * N;
    const double inv_n = ldexp(1.0, -sh.lg);
#pragma unroll
    for (int i = 0; i < Cfg::kET; ++i) {
        const int idx = tid + i * kThrA;
        const int k1 = idx >> lgC, c = idx & (C - 1);
        const int64_t n2 = c0 + c;
        // W_N^{n2 k1}: argument reduced to (-1, 1] half-turns, exact in the working type
        int64_t q2 = 2 * ((n2 * k1) & (N - 1));
        if (q2 > N) q2 -= 2 * N;
        T2 w;
        if constexpr (sizeof(T) == 4) {
            w = unit_phasor_f(-(float)q2 * (float)inv_n);
        } else {
            w = unit_phasor(-(double)q2 * inv_n);
        }
        w.x *= sc;
        w.y *= sc;
        Yt[((int64_t)k1 << sh.lg2) + n2] = cmul(buf[idx], w);
    }
}

// N <= L: the three packed transforms of one pixel pair per block straight from the traces
// (one row, N1 = 1), then S
template <typename T>
__global__ __launch_bounds__(kThrB) void k_fwd_row_direct(const T *__restrict__ E, T *__restrict__ S, FwdShape sh,
                                                          T sc)
{
    using T2 = typename C2<T>::type;
    using Cfg = FwdCfg<T>;
    constexpr int PS = Cfg::kPadShift;
    constexpr int EL = 1 << Cfg::kLgRow;
    constexpr int LPT = EL / kThrB;  // loaded elements per thread
    constexpr int QPT = LPT / 2;     // outputs per thread (+1 for j = N/2)
    __shared__ T2 buf[EL + (EL >> PS)];
    __shared__ T2 tlo[64], thi[64];
    const int tid = threadIdx.x;
    const int lg = sh.lg;
    const int64_t N = (int64_t)1 << lg, half = N / 2;
    const int64_t p = sh.pair0 + blockIdx.y;
    const int64_t m = 2 * p, m1 = 2 * p + 1;
    const bool has1 = m1 < sh.n_pix;
    const LayRows<PS> lay{lg};
    build_tables(tlo, thi, tid);
    // outputs k < N/2, plus k = N/2 taken by thread 0 as output QPT
    const int nout = 1 << (lg - 1);
    const bool extra = tid == 0;
    T accm[QPT + 1], acc1[QPT + 1];
#pragma unroll
    for (int i = 0; i <= QPT; ++i) accm[i] = acc1[i] = (T)0;
    for (int t = 0; t < 3; ++t) {
        if (t == 1 && !has1) continue;
        __syncthreads();
        // the lane index as an opaque value per transform: keeps the compiler from holding
        // every per-lane address of the loop body in registers across the three transforms
        int ltid = tid;
        asm volatile("" : "+v"(ltid));
        const T *re, *im;
        pair_pointers(E, sh.n_pix, p, t, N, re, im);
#pragma unroll
        for (int i = 0; i < LPT; ++i) {
            const int q = ltid + i * kThrB;
            if (q >= N) continue;
            T2 v;
            v.x = re[q] * sc;
            v.y = im ? im[q] * sc : (T)0;
            buf[lay.addr(0, q)] = v;
        }
        __syncthreads();
        fft_inplace<Cfg::kET, Cfg::kLgRadix>(buf, lay, lg, 1, tlo, thi, ltid, kThrB);
#pragma unroll
        for (int i = 0; i <= QPT; ++i) {
            int k;
            if (i < QPT) {
                k = ltid + i * kThrB;
                if (k >= nout) continue;
            } else {
                if (!extra) continue;
                k = (int)half;
            }
            // X_{N-k} at (N - k) mod N
            const T2 zj = buf[lay.addr(0, k)], zm = buf[lay.addr(0, (int)((N - k) & (N - 1)))];
            if (t < 2) {
                const T v = (zj.x * zj.x + zj.y * zj.y + zm.x * zm.x + zm.y * zm.y) * (T)0.5;
                if (t == 0)
                    accm[i] += v;
                else
                    acc1[i] += v;
            } else {
                const T ax = (zj.x + zm.x) * (T)0.5, ay = (zj.y - zm.y) * (T)0.5;
                const T bx = (zj.x - zm.x) * (T)0.5, by = (zj.y + zm.y) * (T)0.5;
                accm[i] += ax * ax + ay * ay;
                acc1[i] += bx * bx + by * by;
            }
        }
    }
    const int64_t ldS = half + 1;
#pragma unroll
    for (int i = 0; i <= QPT; ++i) {
        int k;
        if (i < QPT) {
            k = tid + i * kThrB;
            if (k >= nout) continue;
        } else {
            if (!extra) continue;
            k = (int)half;
        }
        S[m * ldS + k] = accm[i];
        if (has1) S[m1 * ldS + k] = acc1[i];
    }
}

// ---------------------------------------------------------------------------------------------
// Forward path for N > L (L = 2^kLgL row points), every index fixed at compile time.
//
// Pass A (k_fwd_cols_fast<T, LG1>): thread (column c, group g < TPC = N1/ET) loads the ET
// column elements g + TPC m.  The first radix pass works on those registers, the middle passes
// go through LDS, and the last pass (radix ET, Ns = TPC) leaves the outputs k1 = g + TPC r in
// registers, where sc W_N^{n2 k1} = sc W_N^{n2 g} (W_N^{n2 TPC})^r is applied before the store.
//
// Pass B (k_fwd_rows_fast<T>): a block of 256 threads per row pair (k1, N1 - k1) of a pixel
// pair; the rows of the three packed transforms pass through one LDS row buffer in turn, the
// next row's loads in flight meanwhile.  Thread u loads elements u + 256 m (m < R) of a row;
// passes: radix R (Ns = 1), the remainder radix 2^(lg L mod lg R) if any, radix R up to the
// last one (Ns = L/R = 256), which yields outputs u + 256 m of row k1 and rho + 256 m of row
// N1 - k1 with rho = 255 - u: the partners N2 - 1 - e of its own outputs e, so X_{N-j} of each
// S_j it writes is in its registers.  Row 0 pairs with itself at (N2 - e) mod N2 (rho = -u mod
// 256, and for u = 0 a last pass that yields the outputs rotated by one), row N1/2 with itself
// at N2 - 1 - e.
//
// LDS addresses are one base per pass and thread plus compile-time offsets: the row buffer has
// one pad element per R elements (R = its period), and every stride a pass steps by is a
// multiple of R or stays inside one period.
template <typename T>
struct FastCfg;
// kRowWaves: waves per SIMD pass B is compiled for (its registers: a row of the prefetch, one
// row's outputs held while the partner row runs, and the accumulators of 2 R + 2 outputs).
// Measured alternatives on 16384 traces of 2^18 points: FP32 radix 8 with 512 threads, 36.8
// against 36.0 ms (more passes and LDS traffic for the doubled occupancy); a block of two
// 256-thread halves, one row each, swapping partner outputs through LDS, 34.8 ms in FP32 but
// 19.1 against 16.8 ms on 4096 FP64 traces (its two FP64 row buffers leave one block per CU).
template <>
struct FastCfg<float> {
    static constexpr int kLgL = 12, kLgR = 4, kRowThreads = 1 << (kLgL - kLgR), kRowWaves = 2;
};
template <>
struct FastCfg<double> {
    static constexpr int kLgL = 11, kLgR = 3, kRowThreads = 1 << (kLgL - kLgR), kRowWaves = 2;
};
// L / R = 256 threads in both: one radix-R butterfly each per row in the first and last passes.
// In-pass twiddle bases W_{Ns Rp}^k (k < Ns) are entries q < L/Rp of a table of W_L^q.
// Pass B's table covers its smallest radix (the remainder pass), pass A's radix ET.
template <typename T>
constexpr int tab_entries_rows()
{
    constexpr int rem = FastCfg<T>::kLgL % FastCfg<T>::kLgR;
    return 1 << (FastCfg<T>::kLgL - (rem ? rem : FastCfg<T>::kLgR));
}
template <typename T>
constexpr int tab_entries_cols()
{
    return 1 << (FastCfg<T>::kLgL - FwdCfg<T>::kLgRadix);
}

template <int PS>
struct AtRow {  // element e of the row buffer, one pad element every 2^PS
    __device__ __forceinline__ int operator()(int e) const { return e + (e >> PS); }
    static constexpr int far(int d) { return d + (d >> PS); }  // offset of +d, d a multiple of 2^PS
    static constexpr int near(int d) { return d; }             // offset of +d inside one period
};
template <int LGC>
struct AtCol {  // element e of column c among 2^LGC interleaved columns
    int c;
    __device__ __forceinline__ int operator()(int e) const { return (e << LGC) + c; }
    static constexpr int far(int d) { return d << LGC; }
    static constexpr int near(int d) { return d << LGC; }
};

// Twiddle table slot of entry q (one pad slot per 16 entries: the strided reads tab[16 k] of a
// middle pass fall in distinct banks)
__device__ __forceinline__ int tabi(int q) { return q + (q >> 4); }
constexpr int tab_slots(int entries) { return entries + entries / 16; }

// w[r] = w1^r for 1 <= r < RP, each a product chain of depth at most lg RP
template <int RP, typename T2>
__device__ __forceinline__ void powers(T2 w1, T2 *w)
{
    w[1] = w1;
#pragma unroll
    for (int r = 2; r < RP; ++r) {
        const int hb = 1 << (31 - __builtin_clz(r));
        w[r] = hb == r ? cmul(w[r / 2], w[r / 2]) : cmul(w[hb], w[r - hb]);
    }
}

// v[r] *= w1^r for 1 <= r < RP: w1^r = w1^(4 b) w1^a (r = 4 b + a) from w1, w1^2, w1^3 and a
// running w1^(4 b), product chains of depth <= 5 with 10 registers of powers live
template <int RP, typename T2>
__device__ __forceinline__ void twiddle_apply(T2 *v, T2 w1)
{
    v[1] = cmul(v[1], w1);
    if constexpr (RP > 2) {
        const T2 w2 = cmul(w1, w1), w3 = cmul(w2, w1);
        v[2] = cmul(v[2], w2);
        v[3] = cmul(v[3], w3);
        if constexpr (RP > 4) {
            const T2 w4 = cmul(w2, w2);
            T2 h = w4;
#pragma unroll
            for (int b = 1; b < RP / 4; ++b) {
                if (b == 2) h = cmul(w4, w4);
                if (b > 2) h = cmul(h, w4);
                v[4 * b] = cmul(v[4 * b], h);
                v[4 * b + 1] = cmul(v[4 * b + 1], cmul(h, w1));
                v[4 * b + 2] = cmul(v[4 * b + 2], cmul(h, w2));
                v[4 * b + 3] = cmul(v[4 * b + 3], cmul(h, w3));
            }
        }
    }
}

// First Stockham pass (Ns = 1, no twiddles) from registers: the thread's butterflies are
// j = j0 + JS s (s < NB), and X[s + NB r] holds element j + r (sequence length / RP).
// The RP outputs of a butterfly are adjacent (inside one pad period of the row layout).
template <int RP, int NB, int JS, typename T2, typename At>
__device__ __forceinline__ void first_pass(const T2 *X, T2 *buf, const At &at, int j0)
{
    T2 *pw = buf + at(j0 * RP);
#pragma unroll
    for (int s = 0; s < NB; ++s) {
        T2 v[RP];
#pragma unroll
        for (int r = 0; r < RP; ++r) v[r] = X[s + NB * r];
        dftR<RP>(v);
#pragma unroll
        for (int r = 0; r < RP; ++r) pw[At::far(JS * s * RP) + At::near(r)] = v[r];
    }
}

// One middle Stockham pass of radix RP = 2^LGRP at Ns = 2^LGNS over 2^LGN points: butterfly j
// reads e = j + r 2^LGN/RP, multiplies by W_{Ns RP}^{r k} (k = j mod Ns; W^k = tab entry
// k 2^(LGTAB - LGNS - LGRP)), transforms and writes (j - k) RP + k + r Ns.  The thread takes
// butterflies j0 + JS s, s < NB (JS a multiple of Ns).
template <int LGRP, int LGN, int LGNS, int NB, int JS, int LGTAB, typename T2, typename At>
__device__ __forceinline__ void mid_pass(T2 *buf, const At &at, int j0, const T2 *tab)
{
    constexpr int RP = 1 << LGRP, M = (1 << LGN) / RP, NS = 1 << LGNS;
    T2 v[NB][RP];
    const T2 *pr = buf + at(j0);
#pragma unroll
    for (int s = 0; s < NB; ++s)
#pragma unroll
        for (int r = 0; r < RP; ++r) v[s][r] = pr[At::far(JS * s + r * M)];
    __syncthreads();
    const int k = j0 & (NS - 1);
    T2 w1;
    if constexpr (LGNS > 0) w1 = tab[tabi(k << (LGTAB - LGNS - LGRP))];
    T2 *pw = buf + at((j0 - k) * RP + k);
#pragma unroll
    for (int s = 0; s < NB; ++s) {
        if constexpr (LGNS > 0) twiddle_apply<RP>(v[s], w1);
        dftR<RP>(v[s]);
#pragma unroll
        for (int r = 0; r < RP; ++r) pw[At::far(JS * s * RP + r * NS)] = v[s][r];
    }
    __syncthreads();
}

// Middle passes of radix 2^LGRP from Ns = 2^LGNS up to (not including) 2^LGEND, one butterfly
// j per thread.
template <int LGRP, int LGN, int LGNS, int LGEND, int LGTAB, typename T2, typename At>
__device__ __forceinline__ void mid_passes(T2 *buf, const At &at, int j, const T2 *tab)
{
    if constexpr (LGNS < LGEND) {
        mid_pass<LGRP, LGN, LGNS, 1, 1, LGTAB>(buf, at, j, tab);
        mid_passes<LGRP, LGN, LGNS + LGRP, LGEND, LGTAB>(buf, at, j, tab);
    }
}

// Last Stockham pass (Ns = 2^LGN / RP butterflies, k = j) into registers: out[r] = X[j + Ns r]
// with w1 = W_{2^LGN}^j.  (w1 = W_{2^LGN}^j W_RP instead gives out[r] = X[j + Ns ((r + 1) mod RP)].)
template <int LGRP, int LGN, typename T2, typename At>
__device__ __forceinline__ void last_pass_w(const T2 *buf, const At &at, int j, T2 w1, T2 *out)
{
    constexpr int RP = 1 << LGRP, NS = (1 << LGN) / RP;
    const T2 *pr = buf + at(j);
#pragma unroll
    for (int r = 0; r < RP; ++r) out[r] = pr[At::far(r * NS)];
    twiddle_apply<RP>(out, w1);
    dftR<RP>(out);
}
template <int LGRP, int LGN, int LGTAB, typename T2, typename At>
__device__ __forceinline__ void last_pass(const T2 *buf, const At &at, int j, const T2 *tab, T2 *out)
{
    constexpr int RP = 1 << LGRP, NS = (1 << LGN) / RP;
    if constexpr (NS > 1) {
        last_pass_w<LGRP, LGN>(buf, at, j, tab[tabi(j << (LGTAB - LGN))], out);
    } else {
        const T2 *pr = buf + at(j);
#pragma unroll
        for (int r = 0; r < RP; ++r) out[r] = pr[At::far(r * NS)];
        dftR<RP>(out);
    }
}

// exp(-2 pi i q / N) for 0 <= q (reduced mod N = 2^lg), argument exact in the working type
template <typename T2>
__device__ __forceinline__ T2 phasor_mod(int64_t q, int64_t N, double inv_n);
template <>
__device__ __forceinline__ float2 phasor_mod<float2>(int64_t q, int64_t N, double inv_n)
{
    int64_t q2 = 2 * (q & (N - 1));
    if (q2 > N) q2 -= 2 * N;
    return unit_phasor_f(-(float)q2 * (float)inv_n);
}
template <>
__device__ __forceinline__ double2 phasor_mod<double2>(int64_t q, int64_t N, double inv_n)
{
    int64_t q2 = 2 * (q & (N - 1));
    if (q2 > N) q2 -= 2 * N;
    return unit_phasor(-(double)q2 * inv_n);
}

// pass A: C = 2^LGC adjacent columns (of N1 = 2^LG1 points) of one packed transform of one pixel
// pair per block
template <typename T, int LG1>
__global__ __launch_bounds__(256) void k_fwd_cols_fast(const T *__restrict__ E, typename C2<T>::type *__restrict__ Y,
                                                       FwdShape sh, T sc)
{
    using T2 = typename C2<T>::type;
    constexpr int LGET = FwdCfg<T>::kLgRadix, ET = 1 << LGET;  // elements per thread
    constexpr int LGTAB = FastCfg<T>::kLgL;
    constexpr int LGC = 8 + LGET - LG1, C = 1 << LGC, TPC = 1 << (LG1 - LGET);
    static_assert(LG1 >= LGET && LGC >= 0, "columns of ET to 256 ET points");
    constexpr int LGR0 = LG1 % LGET ? LG1 % LGET : LGET, NB0 = ET >> LGR0;
    constexpr bool kLds = LG1 > LGET;
    __shared__ T2 buf[kLds ? (C << LG1) : 1];
    __shared__ T2 tab[tab_slots(tab_entries_cols<T>())];
    const int tid = threadIdx.x, c = tid & (C - 1), g = tid >> LGC;
    const int t = blockIdx.y;
    const int64_t pl = blockIdx.z, p = sh.pair0 + pl;
    const int64_t N = (int64_t)1 << sh.lg;
    const T *re, *im;
    pair_pointers(E, sh.n_pix, p, t, N, re, im);
    if (!re) return;  // transform of a missing pixel: pass B skips it too
    const int n2 = blockIdx.x * C + c;
    if constexpr (kLds) {
        for (int q = tid; q < tab_entries_cols<T>(); q += 256) tab[tabi(q)] = twiddle<T2>(q, 1 << LGTAB);
    }
    T2 X[ET];
#pragma unroll
    for (int m = 0; m < ET; ++m) {
        const int n = ((g + TPC * m) << sh.lg2) + n2;
        X[m].x = re[n];
        X[m].y = im ? im[n] : (T)0;
    }
    T2 O[ET];
    if constexpr (!kLds) {
#pragma unroll
        for (int r = 0; r < ET; ++r) O[r] = X[r];
        dftR<ET>(O);
    } else {
        const AtCol<LGC> at{c};
        first_pass<1 << LGR0, NB0, TPC>(X, buf, at, g);
        __syncthreads();
        mid_passes<LGET, LG1, LGR0, LG1 - LGET, LGTAB>(buf, at, g, tab);
        last_pass<LGET, LG1, LGTAB>(buf, at, g, tab, O);
    }
    // sc W_N^{n2 k1} for k1 = g + TPC r: bw (W_N^{n2 TPC})^r, the power a product chain of depth
    // <= LGET, bw = sc W_N^{n2 g} (the trace scale sc rides on the twiddle)
    const double inv_n = ldexp(1.0, -sh.lg);
    T2 bw = phasor_mod<T2>((int64_t)n2 * g, N, inv_n);
    bw.x *= sc;
    bw.y *= sc;
    T2 sp[ET];
    powers<ET>(phasor_mod<T2>((int64_t)n2 * TPC, N, inv_n), sp);
    T2 *Yt = Y + (pl * 3 + t) * N;
    Yt[(g << sh.lg2) + n2] = cmul(O[0], bw);
#pragma unroll
    for (int r = 1; r < ET; ++r) Yt[((g + TPC * r) << sh.lg2) + n2] = cmul(O[r], cmul(bw, sp[r]));
}

// Elements u + NT m (m < R) of a row of L complex values, by buffer loads: a scalar resource for
// the row, one lane offset, and the NT m steps as scalar offsets
template <int R, int NT, typename T2>
__device__ __forceinline__ void load_row_lanes(T2 *X, const T2 *row, int u)
{
    constexpr int L = R * NT;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc((void *)row, (short)0, (int)(L * sizeof(T2)), 0x00020000);
#pragma unroll
    for (int m = 0; m < R; ++m) {
        if constexpr (sizeof(T2) == 8)
            X[m] = __builtin_bit_cast(T2, __builtin_amdgcn_raw_buffer_load_b64(rs, u * 8, m * NT * 8, 0));
        else
            X[m] = __builtin_bit_cast(T2, __builtin_amdgcn_raw_buffer_load_b128(rs, u * 16, m * NT * 16, 0));
    }
}

// pass B: row pair (k1, N1 - k1) of the three packed transforms of one pixel pair per block, then S
template <typename T>
__global__ __launch_bounds__(FastCfg<T>::kRowThreads) __attribute__((amdgpu_waves_per_eu(FastCfg<T>::kRowWaves))) void k_fwd_rows_fast(
    const typename C2<T>::type *__restrict__ Y, T *__restrict__ S, FwdShape sh, T scale)
{
    using T2 = typename C2<T>::type;
    using Cfg = FastCfg<T>;
    constexpr int LGL = Cfg::kLgL, L = 1 << LGL, LGR = Cfg::kLgR, R = 1 << LGR, H = R / 2;
    constexpr int REM = LGL % LGR;  // remainder pass radix 2^REM (none if 0)
    constexpr int NT = L / R;  // threads: one butterfly each in the first and last passes
    static_assert(NT == Cfg::kRowThreads, "block size");
    __shared__ T2 buf[L + L / R];
    __shared__ T2 tab[tab_slots(tab_entries_rows<T>())];
    const int tid = threadIdx.x;
    const int N1 = 1 << sh.lg1;
    const int64_t N = (int64_t)1 << sh.lg, ldS = N / 2 + 1;
    // block -> (row pair, pixel pair): all row-pair blocks of one pixel pair run on one XCD
    // (blocks go to the 8 XCDs round robin), so the partial lines of its spectrum, written at a
    // stride of N1 elements, merge in that XCD's L2
    const int64_t b = blockIdx.x, xcd = b & 7, slot = b >> 3;
    const int nrp = N1 / 2 + 1;
    const int rp = (int)(slot % nrp);
    const int64_t pl = (slot / nrp) * 8 + xcd;
    if (pl >= sh.nbatch) return;  // padding block (whole block)
    const int64_t p = sh.pair0 + pl, m0 = 2 * p, m1 = m0 + 1;
    const bool has1 = m1 < sh.n_pix;
    const int ka = rp, kb = (N1 - rp) & (N1 - 1);
    const bool two = ka != kb, row0 = ka == 0;
    const int rho = row0 ? ((NT - tid) & (NT - 1)) : NT - 1 - tid;
    for (int q = tid; q < tab_entries_rows<T>(); q += NT) tab[tabi(q)] = twiddle<T2>(q, L);
    __syncthreads();
    const T2 wa = tab[tabi(tid)], wb = row0 && tid == 0 ? twiddle<T2>(1, R) : tab[tabi(rho)];
    const AtRow<LGR> at;
    // accm/acc1: [0, H) outputs tid + NT q of row ka, [H] j = N/2 (row 0, thread 0),
    // (H, 2H] outputs rho + NT q of row kb; pixel m0 / m1
    T accm[R + 1], acc1[R + 1];
#pragma unroll
    for (int q = 0; q <= R; ++q) accm[q] = acc1[q] = (T)0;
    // rows in order: (t, ka) and, with two rows, (t, kb) for t = 0, 1 (second pixel only), 2;
    // each row's loads are issued while the previous row runs through the buffer
    const int nt = has1 ? 3 : 2;
    auto row_ptr = [&](int tt, bool second) {  // the row (uniform), indexed by 32-bit offsets
        const int t = (!has1 && tt == 1) ? 2 : tt;
        return Y + (pl * 3 + t) * N + (int64_t)(second ? kb : ka) * L;
    };
    T2 X[R];
    auto load_row = [&](const T2 *src) { load_row_lanes<R, NT>(X, src, tid); };
    auto row_passes = [&](const T2 *next) {  // next: the row to load meanwhile, or null
        __syncthreads();  // the previous row's last pass has read the buffer
        first_pass<R, 1, 1>(X, buf, at, tid);
        if (next) load_row(next);
        __syncthreads();
        if constexpr (REM > 0) mid_pass<REM, LGL, LGR, (L >> REM) / NT, NT, LGL>(buf, at, tid, tab);
        mid_passes<LGR, LGL, LGR + REM, LGL - LGR, LGL>(buf, at, tid, tab);
    };
    load_row(row_ptr(0, false));
    for (int tt = 0; tt < nt; ++tt) {
        const int t = (!has1 && tt == 1) ? 2 : tt;
        const T2 *after = tt + 1 < nt ? row_ptr(tt + 1, false) : nullptr;
        T2 A[R], B[R];
        row_passes(two ? row_ptr(tt, true) : after);
        last_pass_w<LGR, LGL>(buf, at, tid, wa, A);
        if (two) row_passes(after);
        // row 0's thread 0 pairs element NT q with NT (R - q) mod L: B[i] = X[NT ((i + 1) mod R)]
        last_pass_w<LGR, LGL>(buf, at, rho, wb, B);
        // t < 2: S += (|Z_j|^2 + |Z_{N-j}|^2) / 2 for pixel m0 (t = 0) or m1 (t = 1); t = 2 (Ez of
        // both): |A_j|^2 and |B_j|^2 of the two real parts, (s +- c) / 4 with s = |Z_j|^2 +
        // |Z_{N-j}|^2, c = 2 Re(Z_j Z_{N-j}); all four times larger here (scale = 1/4; pass A has
        // applied the trace scale)
        const T fs0 = t == 0 ? (T)2 : t == 2 ? (T)1 : (T)0, fs1 = t == 1 ? (T)2 : t == 2 ? (T)1 : (T)0;
        const T fc = t == 2 ? (T)1 : (T)0;
#pragma unroll
        for (int q = 0; q <= R; ++q) {
            // q <= H: output tid + NT q of row ka, partner B[R-1-q]; q > H: output
            // rho + NT (q-H-1) of row kb, partner A[R-1-(q-H-1)]
            const T2 zj = q <= H ? A[q] : B[q - H - 1];
            const T2 zm = q <= H ? B[R - 1 - q] : A[R - 1 - (q - H - 1)];
            const T sq = zj.x * zj.x + zj.y * zj.y + zm.x * zm.x + zm.y * zm.y;
            const T c = (T)2 * fc * (zj.x * zm.x - zj.y * zm.y);
            accm[q] += fs0 * sq + c;
            acc1[q] += fs1 * sq - c;
        }
    }
    T *S0 = S + m0 * ldS, *S1 = S + m1 * ldS;
#pragma unroll
    for (int q = 0; q < H; ++q) {
        const int j = ka + ((tid + NT * q) << sh.lg1);
        S0[j] = accm[q] * scale;
        if (has1) S1[j] = acc1[q] * scale;
    }
    if (row0 && tid == 0) {
        S0[N / 2] = accm[H] * scale;
        if (has1) S1[N / 2] = acc1[H] * scale;
    }
    if (two) {
#pragma unroll
        for (int q = 0; q < H; ++q) {
            const int j = kb + ((rho + NT * q) << sh.lg1);
            S0[j] = accm[H + 1 + q] * scale;
            if (has1) S1[j] = acc1[H + 1 + q] * scale;
        }
    }
}

// Adjoint path, pass A: C adjacent columns of one transform of one pixel pair per block
template <typename T>
__global__ __launch_bounds__(256) void k_fft_cols(const T *__restrict__ E, typename C2<T>::type *__restrict__ Y,
                                                  FftShape sh)
{
    using T2 = typename C2<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T2 *smem = reinterpret_cast<T2 *>(smem_raw);
    const int N1 = 1 << sh.lg1, N2 = 1 << sh.lg2;
    const int64_t N = (int64_t)N1 * N2;
    const int t = blockIdx.y;
    const int64_t pl = blockIdx.z, p = sh.pair0 + pl;
    const T *re, *im;
    pair_pointers(E, sh.n_pix, p, t, N, re, im);
    if (!re) return;  // transform of a missing pixel: pass B skips it too
    const int C = sh.C, c0 = blockIdx.x * C;
    T2 *bufA = smem, *bufB = smem + C * N1, *tw = smem + 2 * C * N1;
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int q = tid; q < N1; q += nthr) tw[q] = twiddle<T2>(q, N1);
    for (int idx = tid; idx < N1 * C; idx += nthr) {
        const int n1 = idx / C, cc = idx - n1 * C;
        const int64_t n = (int64_t)n1 * N2 + c0 + cc;
        T2 v;
        v.x = re[n];
        v.y = im ? im[n] : (T)0;
        bufA[cc * N1 + n1] = v;
    }
    __syncthreads();
    T2 *res = lds_fft(bufA, bufB, sh.lg1, C, N1, tw, tid, nthr);
    T2 *Yt = Y + (pl * 3 + t) * N;
    for (int idx = tid; idx < N1 * C; idx += nthr) {
        const int k1 = idx / C, cc = idx - k1 * C;
        const int n2 = c0 + cc;
        const int64_t q = ((int64_t)n2 * k1) & (N - 1);
        Yt[(int64_t)k1 * N2 + n2] = cmul(res[cc * N1 + k1], twiddle<T2>(q, N));
    }
}

// ---------------------------------------------------------------------------------------------
// Adjoint.  With F_c = DFT(E_c) and S_j = (dt^2/2pi) sum_c |F_c[j]|^2 (j <= N/2):
//   dE_c[u] = (dt^2/pi) Re sum_{j<=N/2} dS_j F_c[j] e^{+2 pi i j u/N}
//           = (dt^2/pi) IDFT(G_c)[u],   G_c[j] = h_j dS_{min(j,N-j)} F_c[j],  h_0 = h_{N/2} = 1, else 1/2,
// an IDFT whose output is real.  In the packed transforms Z = a + i b this gives
//   Z0, Z1:  G = h dS_{j*} Z[j]
//   Z2:      G = (h/2) [(dS_m + dS_m+1) Z2[j] + (dS_m - dS_m+1) conj Z2[N-j]]
// and the real / imaginary parts of IDFT(G) are the two packed components.
// The inverse four-step runs rows then columns, each as conj(DFT(conj(.))).

// pass B': forward row transforms, multiply, inverse row transforms, inverse twiddle; in place
template <typename T>
__global__ __launch_bounds__(256) void k_fft_rows_bwd(typename C2<T>::type *__restrict__ Y, const T *__restrict__ dS,
                                                      FftShape sh)
{
    using T2 = typename C2<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T2 *smem = reinterpret_cast<T2 *>(smem_raw);
    const int N1 = 1 << sh.lg1, N2 = 1 << sh.lg2;
    const int64_t N = (int64_t)N1 * N2, half = N / 2;
    const int rp = blockIdx.x;
    const int64_t pl = blockIdx.y, p = sh.pair0 + pl;
    const int64_t m = 2 * p, m1 = 2 * p + 1;
    const bool has1 = m1 < sh.n_pix;
    const int ka = rp, kb = (N1 - rp) & (N1 - 1);
    const int nrows = ka == kb ? 1 : 2;
    T2 *bufA = smem, *bufB = smem + 2 * N2, *tw = smem + 4 * N2;
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int q = tid; q < N2; q += nthr) tw[q] = twiddle<T2>(q, N2);
    const int64_t ldS = half + 1;
    const T *dSm = dS + m * ldS, *dSm1 = has1 ? dS + m1 * ldS : nullptr;
    for (int t = 0; t < 3; ++t) {
        if (t == 1 && !has1) continue;
        T2 *Yt = Y + (pl * 3 + t) * N;
        __syncthreads();
        for (int idx = tid; idx < nrows * N2; idx += nthr) {
            const int row = idx >> sh.lg2, k2 = idx & (N2 - 1);
            bufA[row * N2 + k2] = Yt[(int64_t)(row ? kb : ka) * N2 + k2];
        }
        __syncthreads();
        T2 *res = lds_fft(bufA, bufB, sh.lg2, nrows, N2, tw, tid, nthr);
        T2 *oth = res == bufA ? bufB : bufA;
        for (int q = tid; q < nrows * N2; q += nthr) {
            const int row = q >> sh.lg2, k2 = q & (N2 - 1);
            const int kr = row ? kb : ka;
            const int64_t j = kr + (int64_t)N1 * k2;
            const int64_t jm = (N - j) & (N - 1);
            const int64_t js = j < jm ? j : jm;
            const T h = (j == 0 || j == half) ? (T)1 : (T)0.5;
            const T2 z = res[q];
            T2 g;
            if (t < 2) {
                const T d = h * (t == 0 ? dSm[js] : dSm1[js]);
                g.x = d * z.x;
                g.y = d * z.y;
            } else {
                int mrow, mk2;
                if (kr == 0) {
                    mrow = row;
                    mk2 = (N2 - k2) & (N2 - 1);
                } else {
                    mrow = (N1 - kr == ka) ? 0 : 1;
                    mk2 = N2 - 1 - k2;
                }
                const T2 zm = res[mrow * N2 + mk2];
                const T a = dSm[js], b = has1 ? dSm1[js] : (T)0;
                const T sp = (T)0.5 * h * (a + b), sm = (T)0.5 * h * (a - b);
                // sp z + sm conj(zm)
                g.x = sp * z.x + sm * zm.x;
                g.y = sp * z.y - sm * zm.y;
            }
            g.y = -g.y;  // conj before the forward transform
            oth[q] = g;
        }
        __syncthreads();
        T2 *res2 = lds_fft(oth, res, sh.lg2, nrows, N2, tw, tid, nthr);
        for (int q = tid; q < nrows * N2; q += nthr) {
            const int row = q >> sh.lg2, n2 = q & (N2 - 1);
            const int kr = row ? kb : ka;
            T2 v = res2[q];
            v.y = -v.y;  // conj after: inverse row transform
            // inverse twiddle exp(+2 pi i n2 kr / N) = conj(exp(-2 pi i n2 kr / N))
            T2 w = twiddle<T2>(((int64_t)n2 * kr) & (N - 1), N);
            w.y = -w.y;
            Yt[(int64_t)kr * N2 + n2] = cmul(v, w);
        }
    }
}

// pass C: inverse column transforms; real / imaginary parts are the two packed components of dE
template <typename T>
__global__ __launch_bounds__(256) void k_fft_cols_inv(const typename C2<T>::type *__restrict__ Y, T *__restrict__ dE,
                                                      FftShape sh, T scale)
{
    using T2 = typename C2<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T2 *smem = reinterpret_cast<T2 *>(smem_raw);
    const int N1 = 1 << sh.lg1, N2 = 1 << sh.lg2;
    const int64_t N = (int64_t)N1 * N2;
    const int t = blockIdx.y;
    const int64_t pl = blockIdx.z, p = sh.pair0 + pl;
    const int64_t m = 2 * p, m1 = 2 * p + 1;
    const bool has1 = m1 < sh.n_pix;
    if (t == 1 && !has1) return;
    T *re, *im;
    if (t == 0) {
        re = dE + (m * 3 + 0) * N;
        im = dE + (m * 3 + 1) * N;
    } else if (t == 1) {
        re = dE + (m1 * 3 + 0) * N;
        im = dE + (m1 * 3 + 1) * N;
    } else {
        re = dE + (m * 3 + 2) * N;
        im = has1 ? dE + (m1 * 3 + 2) * N : nullptr;
    }
    const int C = sh.C, c0 = blockIdx.x * C;
    T2 *bufA = smem, *bufB = smem + C * N1, *tw = smem + 2 * C * N1;
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int q = tid; q < N1; q += nthr) tw[q] = twiddle<T2>(q, N1);
    const T2 *Yt = Y + (pl * 3 + t) * N;
    for (int idx = tid; idx < N1 * C; idx += nthr) {
        const int k1 = idx / C, cc = idx - k1 * C;
        T2 v = Yt[(int64_t)k1 * N2 + c0 + cc];
        v.y = -v.y;
        bufA[cc * N1 + k1] = v;
    }
    __syncthreads();
    T2 *res = lds_fft(bufA, bufB, sh.lg1, C, N1, tw, tid, nthr);
    for (int idx = tid; idx < N1 * C; idx += nthr) {
        const int n1 = idx / C, cc = idx - n1 * C;
        const T2 v = res[cc * N1 + n1];
        const int64_t n = (int64_t)n1 * N2 + c0 + cc;
        re[n] = scale * v.x;
        if (im) im[n] = -scale * v.y;
    }
}

int ilog2(int64_t v)
{
    int l = 0;
    while ((int64_t(1) << l) < v) ++l;
    return l;
}

template <typename T>
size_t per_pair_bytes(int64_t n_obs)
{
    return (size_t)3 * (size_t)n_obs * sizeof(typename C2<T>::type);
}

constexpr int64_t kMaxGridYZ = 65535;

// columns of up to 2^kFastColsMaxLg1 points take the compile-time pass A; longer ones leave it
// fewer than 16 adjacent columns per block, where it measured slower than k_fwd_cols (FP64,
// 2^20 points: 113.6 against 109.5 ms for 4096 traces)
constexpr int kFastColsMaxLg1 = 8;
template <typename T>
using ColsKernel = void (*)(const T *, typename C2<T>::type *, FwdShape, T);
template <typename T, int LG1>
ColsKernel<T> pick_cols_fast(int lg1)
{
    if constexpr (LG1 > kFastColsMaxLg1)
        return nullptr;
    else
        return lg1 == LG1 ? k_fwd_cols_fast<T, LG1> : pick_cols_fast<T, LG1 + 1>(lg1);
}

template <typename T>
lw_status run_fft(const T *E, int64_t n_pix, int64_t n_obs, double dt_obs, T *S, void *ws, size_t ws_bytes,
                  hipStream_t s)
{
    using T2 = typename C2<T>::type;
    using Cfg = FwdCfg<T>;
    FwdShape sh;
    sh.n_pix = n_pix;
    sh.nbatch = 0;
    sh.lg = ilog2(n_obs);
    sh.lg2 = std::min(sh.lg, Cfg::kLgRow);
    sh.lg1 = sh.lg - sh.lg2;
    const int lgEL = ilog2(Cfg::kET * kThrA);
    if (sh.lg1 > lgEL) return fail(LW_E_SHAPE, "lw_spectrum_fft: n_obs too large");
    sh.lgC = lgEL - sh.lg1;  // C * N1 = elements per block of pass A
    const T sc = (T)(dt_obs / sqrt(2.0 * kPi));
    const int64_t pairs = (n_pix + 1) / 2;
    if (sh.lg1 == 0) {
        for (int64_t p0 = 0; p0 < pairs; p0 += kMaxGridYZ) {
            sh.pair0 = p0;
            const int64_t nb = std::min(kMaxGridYZ, pairs - p0);
            k_fwd_row_direct<T><<<dim3(1, (unsigned)nb, 1), kThrB, 0, s>>>(E, S, sh, sc);
        }
        return check_launch("lw_spectrum_fft");
    }
    const int64_t batch = std::min<int64_t>({pairs, (int64_t)(ws_bytes / per_pair_bytes<T>(n_obs)), kMaxGridYZ});
    T2 *Y = (T2 *)ws;
    // N > L: the compile-time passes (pass A for columns of ET to 2^kFastColsMaxLg1 points)
    const ColsKernel<T> cols = pick_cols_fast<T, Cfg::kLgRadix>(sh.lg1);
    const int lgC_fast = 8 + Cfg::kLgRadix - sh.lg1;
    const unsigned gx_a = (unsigned)(1u << (sh.lg2 - (cols ? lgC_fast : sh.lgC))), gx_b = (unsigned)((1 << sh.lg1) / 2 + 1);
    for (int64_t p0 = 0; p0 < pairs; p0 += batch) {
        const int64_t nb = std::min(batch, pairs - p0);
        sh.pair0 = p0;
        if (cols)
            cols<<<dim3(gx_a, 3, (unsigned)nb), 256, 0, s>>>(E, Y, sh, sc);
        else
            k_fwd_cols<T><<<dim3(gx_a, 3, (unsigned)nb), kThrA, 0, s>>>(E, Y, sh, sc);
        sh.nbatch = nb;
        k_fwd_rows_fast<T><<<dim3((unsigned)((nb + 7) / 8 * 8 * gx_b), 1, 1), FastCfg<T>::kRowThreads, 0, s>>>(
            Y, S, sh, (T)0.25);
    }
    return check_launch("lw_spectrum_fft");
}

template <typename T>
lw_status run_fft_bwd(const T *E, const T *dS, int64_t n_pix, int64_t n_obs, double dt_obs, T *dE, void *ws,
                      size_t ws_bytes, hipStream_t s)
{
    using T2 = typename C2<T>::type;
    const int lg = ilog2(n_obs);
    FftShape sh;
    sh.n_pix = n_pix;
    sh.lg2 = lg / 2;
    sh.lg1 = lg - sh.lg2;
    const int N1 = 1 << sh.lg1, N2 = 1 << sh.lg2;
    if (2 * N2 > 16 * 256) return fail(LW_E_SHAPE, "lw_spectrum_fft_bwd: n_obs too large");
    const size_t lds_budget = 64 * 1024;
    int C = 1;
    while (C * 2 <= N2 && (size_t)(2 * (C * 2) * N1 + N1) * sizeof(T2) <= lds_budget && C * 2 <= 16) C *= 2;
    sh.C = C;
    const size_t smemA = (size_t)(2 * C * N1 + N1) * sizeof(T2);
    const size_t smemB = (size_t)(5 * N2) * sizeof(T2);
    const void *kerA[2] = {(const void *)k_fft_cols<T>, (const void *)k_fft_cols_inv<T>};
    for (const void *kk : kerA)
        if (smemA > 64 * 1024 &&
            hipFuncSetAttribute(kk, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smemA) != hipSuccess)
            return fail(LW_E_UNSUPPORTED, "lw_spectrum_fft_bwd: LDS request of %zu bytes refused", smemA);
    if (smemB > 64 * 1024 && hipFuncSetAttribute((const void *)k_fft_rows_bwd<T>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)smemB) != hipSuccess)
        return fail(LW_E_UNSUPPORTED, "lw_spectrum_fft_bwd: LDS request of %zu bytes refused", smemB);
    const int64_t pairs = (n_pix + 1) / 2;
    const int64_t batch = std::min<int64_t>({pairs, (int64_t)(ws_bytes / per_pair_bytes<T>(n_obs)), kMaxGridYZ});
    T2 *Y = (T2 *)ws;
    const T scale = (T)(dt_obs * dt_obs / kPi);
    for (int64_t p0 = 0; p0 < pairs; p0 += batch) {
        const int64_t nb = std::min(batch, pairs - p0);
        sh.pair0 = p0;
        k_fft_cols<T><<<dim3(N2 / C, 3, (unsigned)nb), 256, smemA, s>>>(E, Y, sh);
        k_fft_rows_bwd<T><<<dim3(N1 / 2 + 1, (unsigned)nb, 1), 256, smemB, s>>>(Y, dS, sh);
        k_fft_cols_inv<T><<<dim3(N2 / C, 3, (unsigned)nb), 256, smemA, s>>>(Y, dE, sh, scale);
    }
    return check_launch("lw_spectrum_fft_bwd");
}

}  // namespace

size_t fft_ws_bytes(int64_t n_pix, int64_t n_obs, int prec)
{
    const size_t per = prec == LW_PREC_FP64 ? per_pair_bytes<double>(n_obs) : per_pair_bytes<float>(n_obs);
    const int64_t pairs = std::max<int64_t>((n_pix + 1) / 2, 1);
    // up to 1 GiB of intermediate: larger batches fill the GPU better (measured on the bunch
    // workload: 18.1 ms at 12 GiB, 19.0 ms at 768 MiB, 20.5 ms at 192 MiB in FP32); the
    // intermediate need not stay in the last-level cache
    int64_t want = std::max<int64_t>(1, (int64_t)((size_t(1) << 30) / per));
    want = std::min(want, pairs);
    return per * (size_t)want;
}

lw_status launch_fft(const void *E, int64_t n_pix, int64_t n_obs, double dt_obs, int prec, void *S, void *ws,
                     size_t ws_bytes, hipStream_t s)
{
    if (n_pix == 0) return LW_OK;
    const size_t per = prec == LW_PREC_FP64 ? per_pair_bytes<double>(n_obs) : per_pair_bytes<float>(n_obs);
    if (!ws || ws_bytes < per)
        return fail(LW_E_WORKSPACE, "lw_spectrum_fft: workspace of %zu bytes < %zu needed for one pixel pair",
                    ws_bytes, per);
    if (prec == LW_PREC_FP64)
        return run_fft<double>((const double *)E, n_pix, n_obs, dt_obs, (double *)S, ws, ws_bytes, s);
    return run_fft<float>((const float *)E, n_pix, n_obs, dt_obs, (float *)S, ws, ws_bytes, s);
}

}  // namespace lw

namespace lw {
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mx;
void *g_scratch_ptr[kMaxDevices] = {};  // device address of `scratch` per GPU, once looked up

// the current device's address of `scratch` (looked up once per device, with it current)
lw_status noalloc_scratch(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail(LW_E_HIP, "lw_spectrum_fft_noalloc: no current device (or device index >= %d)", kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mx);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(LW_E_HIP, "lw_spectrum_fft_noalloc: hipGetSymbolAddress(scratch) failed on device %d: %s",
                        dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LW_OK;
}
}  // namespace

size_t fft_noalloc_scratch_bytes() { return kNoallocScratchBytes; }

lw_status launch_fft_noalloc(const void *E, int64_t n_pix, int64_t n_obs, double dt_obs, int prec, void *S,
                             hipStream_t s)
{
    if (n_pix == 0) return LW_OK;
    const size_t per = prec == LW_PREC_FP64 ? per_pair_bytes<double>(n_obs) : per_pair_bytes<float>(n_obs);
    if (per > kNoallocScratchBytes)
        return fail(LW_E_WORKSPACE,
                    "lw_spectrum_fft_noalloc: one pixel pair of n_obs = %lld needs %zu bytes of scratch, more than "
                    "the %zu-byte static scratch (use lw_spectrum_fft with a workspace)",
                    (long long)n_obs, per, kNoallocScratchBytes);
    void *ptr = nullptr;
    const lw_status st = noalloc_scratch(&ptr);
    if (st != LW_OK) return st;
    return launch_fft(E, n_pix, n_obs, dt_obs, prec, S, ptr, kNoallocScratchBytes, s);
}

lw_status launch_fft_bwd(const void *E, const void *dS, int64_t n_pix, int64_t n_obs, double dt_obs, int prec,
                         void *dE, void *ws, size_t ws_bytes, hipStream_t s)
{
    if (n_pix == 0) return LW_OK;
    const size_t per = prec == LW_PREC_FP64 ? per_pair_bytes<double>(n_obs) : per_pair_bytes<float>(n_obs);
    if (!ws || ws_bytes < per)
        return fail(LW_E_WORKSPACE, "lw_spectrum_fft_bwd: workspace of %zu bytes < %zu needed for one pixel pair",
                    ws_bytes, per);
    if (prec == LW_PREC_FP64)
        return run_fft_bwd<double>((const double *)E, (const double *)dS, n_pix, n_obs, dt_obs, (double *)dE, ws,
                                   ws_bytes, s);
    return run_fft_bwd<float>((const float *)E, (const float *)dS, n_pix, n_obs, dt_obs, (float *)dE, ws, ws_bytes,
                              s);
}
}  // namespace lw
