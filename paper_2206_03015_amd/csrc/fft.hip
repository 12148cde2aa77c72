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
// S_j for j <= N/2 directly.  Sub-transforms are radix-4 (+ one radix-2) Stockham
// autosort passes in LDS with a per-block W_L^q table.
#include "lw_internal.h"

#include <algorithm>
#include <cmath>

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

// pass A: C adjacent columns of one transform of one pixel pair per block
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

// pass B: rows k1 and N1-k1 of the three transforms of one pixel pair per block, then S
template <typename T>
__global__ __launch_bounds__(256) void k_fft_rows(const typename C2<T>::type *__restrict__ Y, T *__restrict__ S,
                                                  FftShape sh, T sc)
{
    using T2 = typename C2<T>::type;
    constexpr int kMaxQ = 16;  // 2*N2 <= kMaxQ * 256
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
    T accm[kMaxQ], acc1[kMaxQ];
#pragma unroll
    for (int i = 0; i < kMaxQ; ++i) accm[i] = acc1[i] = (T)0;
    for (int t = 0; t < 3; ++t) {
        if (t == 1 && !has1) continue;
        const T2 *Yt = Y + (pl * 3 + t) * N;
        __syncthreads();
        for (int idx = tid; idx < nrows * N2; idx += nthr) {
            const int row = idx >> sh.lg2, k2 = idx & (N2 - 1);
            const int kr = row ? kb : ka;
            T2 v = Yt[(int64_t)kr * N2 + k2];
            v.x *= sc;
            v.y *= sc;
            bufA[row * N2 + k2] = v;
        }
        __syncthreads();
        const T2 *res = lds_fft(bufA, bufB, sh.lg2, nrows, N2, tw, tid, nthr);
#pragma unroll
        for (int i = 0; i < kMaxQ; ++i) {
            const int q = tid + i * nthr;
            if (q >= nrows * N2) continue;
            const int row = q >> sh.lg2, k2 = q & (N2 - 1);
            const int kr = row ? kb : ka;
            const int64_t j = kr + (int64_t)N1 * k2;
            if (j > half) continue;
            int mrow, mk2;
            if (kr == 0) {
                mrow = row;
                mk2 = (N2 - k2) & (N2 - 1);
            } else {
                const int mk1 = N1 - kr;
                mrow = (mk1 == ka) ? 0 : 1;
                mk2 = N2 - 1 - k2;
            }
            const T2 zj = res[row * N2 + k2], zm = res[mrow * N2 + mk2];
            if (t < 2) {
                T v = (zj.x * zj.x + zj.y * zj.y + zm.x * zm.x + zm.y * zm.y) * (T)0.5;
                if (t == 0)
                    accm[i] += v;
                else
                    acc1[i] += v;
            } else {
                // A = (zj + conj zm)/2 -> Ez_m ; B = (zj - conj zm)/(2i) -> Ez_{m+1}
                T ax = (zj.x + zm.x) * (T)0.5, ay = (zj.y - zm.y) * (T)0.5;
                T bx = (zj.x - zm.x) * (T)0.5, by = (zj.y + zm.y) * (T)0.5;
                accm[i] += ax * ax + ay * ay;
                acc1[i] += bx * bx + by * by;
            }
        }
    }
    const int64_t ldS = half + 1;
#pragma unroll
    for (int i = 0; i < kMaxQ; ++i) {
        const int q = tid + i * nthr;
        if (q >= nrows * N2) continue;
        const int row = q >> sh.lg2, k2 = q & (N2 - 1);
        const int kr = row ? kb : ka;
        const int64_t j = kr + (int64_t)N1 * k2;
        if (j > half) continue;
        S[m * ldS + j] = accm[i];
        if (has1) S[m1 * ldS + j] = acc1[i];
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

template <typename T>
lw_status run_fft(const T *E, int64_t n_pix, int64_t n_obs, double dt_obs, T *S, void *ws, size_t ws_bytes,
                  hipStream_t s)
{
    using T2 = typename C2<T>::type;
    const int lg = ilog2(n_obs);
    FftShape sh;
    sh.n_pix = n_pix;
    sh.lg2 = lg / 2;
    sh.lg1 = lg - sh.lg2;
    const int N1 = 1 << sh.lg1, N2 = 1 << sh.lg2;
    if (2 * N2 > 16 * 256) return fail(LW_E_SHAPE, "lw_spectrum_fft: n_obs too large");
    const size_t lds_budget = 64 * 1024;
    int C = 1;
    while (C * 2 <= N2 && (size_t)(2 * (C * 2) * N1 + N1) * sizeof(T2) <= lds_budget && C * 2 <= 16) C *= 2;
    sh.C = C;
    const size_t smemA = (size_t)(2 * C * N1 + N1) * sizeof(T2);
    const size_t smemB = (size_t)(5 * N2) * sizeof(T2);
    if (smemA > 64 * 1024) {
        if (hipFuncSetAttribute((const void *)k_fft_cols<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)smemA) != hipSuccess)
            return fail(LW_E_UNSUPPORTED, "lw_spectrum_fft: LDS request of %zu bytes refused", smemA);
    }
    if (smemB > 64 * 1024) {
        if (hipFuncSetAttribute((const void *)k_fft_rows<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)smemB) != hipSuccess)
            return fail(LW_E_UNSUPPORTED, "lw_spectrum_fft: LDS request of %zu bytes refused", smemB);
    }
    const int64_t pairs = (n_pix + 1) / 2;
    const int64_t batch = std::min<int64_t>(pairs, (int64_t)(ws_bytes / per_pair_bytes<T>(n_obs)));
    T2 *Y = (T2 *)ws;
    const T sc = (T)(dt_obs / sqrt(2.0 * kPi));
    for (int64_t p0 = 0; p0 < pairs; p0 += batch) {
        const int64_t nb = std::min(batch, pairs - p0);
        sh.pair0 = p0;
        k_fft_cols<T><<<dim3(N2 / C, 3, (unsigned)nb), 256, smemA, s>>>(E, Y, sh);
        k_fft_rows<T><<<dim3(N1 / 2 + 1, (unsigned)nb, 1), 256, smemB, s>>>(Y, S, sh, sc);
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
    const int64_t batch = std::min<int64_t>(pairs, (int64_t)(ws_bytes / per_pair_bytes<T>(n_obs)));
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
    // enough pairs per pass to fill the GPU; bounded so that the intermediate stays near the last-level cache
    int64_t want = std::max<int64_t>(1, (int64_t)((192u << 20) / per));
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
