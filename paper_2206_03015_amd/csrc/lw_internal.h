// Internal declarations of liblw.so (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lw.h"

namespace lw {

// CODATA 2018 (SI)
constexpr double kC = 299792458.0;
constexpr double kQe = 1.602176634e-19;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kMe = 9.1093837015e-31;
constexpr double kPi = 3.14159265358979323846;
constexpr double kCoulomb = 1.0 / (4.0 * kPi * kEps0);
constexpr double kInvC = 1.0 / kC;

// error reporting (thread-local message, see lw_last_error)
void set_error(const char *fmt, ...);
lw_status fail(lw_status st, const char *fmt, ...);
lw_status check_launch(const char *what);

inline bool aligned(const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) & (a - 1)) == 0; }

// kernel timing (lw_timing_enable): timing_begin returns an event recorded on s just before the
// launch (nullptr when timing is off); timing_end records the closing event after the launch
hipEvent_t timing_begin(int which, hipStream_t s);
void timing_end(int which, hipEvent_t start, hipStream_t s);

// ---------------------------------------------------------------------------------------------
// Pixel geometry, shared by the arrival-time and field evaluations.
// 1/sqrt(x) for positive normal x to double precision: the hardware estimate refined by two
// Newton steps y <- y (3 - x y^2)/2 (each squares the relative error).
// rsqrt_nr<1> (one step) is used where the result feeds single-precision fields only.
template <int STEPS>
__device__ __forceinline__ double rsqrt_nr(double x)
{
    double y = __builtin_amdgcn_rsq(x);
#pragma unroll
    for (int it = 0; it < STEPS; ++it) {
        const double e = fma(-x * y, y, 1.0);
        y = fma(0.5 * y, e, y);
    }
    return y;
}
__device__ __forceinline__ double rsqrt_fp64(double x) { return rsqrt_nr<2>(x); }

struct PixGeo {
    double nx, ny, nz;  // unit direction x_m / |x_m|
    double D, invD;     // |x_m|, 1/|x_m|
    bool ok;
};

__device__ __forceinline__ PixGeo pix_geo(const double *x_det, int64_t m)
{
    PixGeo g;
    double x = x_det[3 * m], y = x_det[3 * m + 1], z = x_det[3 * m + 2];
    double D = sqrt(x * x + y * y + z * z);
    g.ok = (D > 0.0) && isfinite(D);
    if (!g.ok) D = 1.0, x = 0.0, y = 0.0, z = 1.0;
    g.nx = x / D;
    g.ny = y / D;
    g.nz = z / D;
    g.D = D;
    g.invD = 1.0 / D;
    return g;
}

// ---------------------------------------------------------------------------------------------
// Arrival time in grid units, tau = (t_i + (|x_m - r_i| - |x_m|)/c - t0)/dt_obs (exact geometry,
// Eq. advanced_condition) or (t_i - n.r_i/c - t0)/dt_obs (far field, Eq. far_adv), split as
//   tau = d + b (+ corr),   d = (t_i - t0 - z_i/c)/dt_obs,   b = C ((1 - n_z) z - n_x x - n_y y),
// with C = 1/(c dt_obs) and corr = C |r_perp|^2/(|x - r| + |x| - s), s = n.r, r_perp = r - s n (the
// identity |x - r| - |x| = -s + |r_perp|^2/(|x - r| + |x| - s), free of cancellation).  d holds
// the two terms of size t_i/dt_obs (up to ~1e8 grid units) that cancel; it is formed once per
// sample with every step in double-double arithmetic and rounded once, so its error is that of
// one rounding of the (window-sized) result.  b is of the size of the transverse offsets and
// (1 - n_z) is formed without cancellation.

// s + e = a + b exactly (Knuth's two-sum)
__host__ __device__ __forceinline__ void two_sum(double a, double b, double &s, double &e)
{
    s = a + b;
    const double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// d of sample idx (t_idx = t_start + idx dt) at height z
__host__ __device__ __forceinline__ double arrival_base(double t_start, double dt, double idx, double t0, double dt_obs,
                                                        double z)
{
    const double p = idx * dt, pe = fma(idx, dt, -p);  // idx dt = p + pe
    double s, se, a, ae, n, ne;
    two_sum(t_start, p, s, se);  // t_idx = s + se + pe
    two_sum(s, -t0, a, ae);      // t_idx - t0 = a + alo
    const double alo = ae + (se + pe);
    const double q = z / kC;
    const double qr = fma(-q, kC, z) / kC;  // z/c = q + qr (the division's residual is exact)
    two_sum(a, -q, n, ne);                  // t_idx - t0 - z/c = n + nlo
    const double nlo = ne + (alo - qr);
    const double h = n / dt_obs;
    const double rem = fma(-h, dt_obs, n);
    return h + (rem + nlo) / dt_obs;
}

// Constants of one pixel: geometry and the coefficients of b.
struct PixC {
    PixGeo g;
    double o, px, py;  // C (1 - n_z), -C n_x, -C n_y
};

__device__ __forceinline__ PixC pix_const_of(const PixGeo &g, double C)
{
    PixC p;
    p.g = g;
    const double nx = p.g.nx, ny = p.g.ny, nz = p.g.nz;
    const double omz = nz > 0.0 ? (nx * nx + ny * ny) / (1.0 + nz) : 1.0 - nz;
    p.o = C * omz;
    p.px = -C * nx;
    p.py = -C * ny;
    return p;
}

__device__ __forceinline__ PixC pix_const(const double *x_det, int64_t m, double C)
{
    return pix_const_of(pix_geo(x_det, m), C);
}

__device__ __forceinline__ double pix_b(const PixC &p, double x, double y, double z)
{
    return fma(p.py, y, fma(p.px, x, p.o * z));
}

// The path correction corr (exact geometry) in one of three forms:
//   kTauSqrt    with its square root and divide;
//   kTauSeries  (valid when |r| <= 1e-4 |x|, checked by the caller) with x = s/|x| and
//               q = |r_perp|^2/(|x| - s)^2:  1/(|x| - s) = (1 + x + x^2 + x^3 + O(x^4))/|x|,
//               1/(|x - r| + |x| - s) = (1/(|x| - s)) (1/2 - q/8 + O(q^2)), |r_perp|^2 = |r|^2 - s^2;
//               truncation below 1e-16 relative under that bound;
//   kTauShort   the same expansion to first order, |r_perp|^2 (1 + x)/(2 |x|): it drops x^2 + q/4
//               <= 1.25e-8 of the correction under the bound (used with single-precision fields).
// Written with explicit fma so that every evaluation of the same (pixel, sample) gives the same bits.
constexpr int kTauSqrt = 0, kTauSeries = 1, kTauShort = 2;
// number of set bits of a wavefront mask below this lane
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// (|r|/|x|)^2 up to which the series forms of the exact-geometry arrival time are used
constexpr double kSeriesBound = 1e-8;
// pixels whose |x_m| is within this relative distance of the records' distance use the records
// (tau_poly at that distance)
constexpr double kSameDistance = 4.0 * 2.220446049250313e-16;
// The polynomial records (tau_poly) are evaluated to a lower degree -- 2 of 3 with
// single-precision fields, 3 of 5 with double ones -- where the terms left out stay within
// kTailBound grid units for the particle's whole trajectory and the pixels of a 128-pixel tile:
// 1e-7 (about the rounding of the single-precision interpolation weights), resp. 1e-12 (far
// below the rounding of a double arrival time of up to ~1e7 grid units).
template <bool F64>
constexpr double kTailBound = F64 ? 1e-12 : 1e-7;
// Whether that holds for a particle with |r|^2 <= rb2 over its trajectory and pixels with
// 2 (1 - n_z) <= s2 at the records' distance D: b = C (e_z - n) . r, so
// |b| <= C |e_z - n| |r| = C sqrt(2 (1 - n_z)) |r|.  Degree 3 (cK = K e): the cubic term K e b^3.
// Degree 5 (cK = 7 K e^3 / 4): |c_4| <= 1.3 K e^2 within the series range (|r| <= 1e-4 D;
// 1.251 K e^2 is its maximum there), and K e^2 = (4/7) cK C D, so
// |c_4 b^4 + cK b^5| <= cK b^4 (0.75 C D + |b|).
template <bool F64>
__device__ __forceinline__ bool tail_negligible(double rb2, double s2, double C, double cK, double D)
{
    const double bmax = C * sqrt(rb2 * s2);
    const double b3 = bmax * bmax * bmax;
    if constexpr (F64)
        return cK * b3 * bmax * (0.75 * C * D + bmax) <= kTailBound<true>;
    else
        return cK * b3 <= kTailBound<false>;
}
template <int GEOM, int FORM>
__device__ __forceinline__ double arrival_tau(const PixC &p, double d, double rx, double ry, double rz, double rr,
                                              double C)
{
    double tau = d + pix_b(p, rx, ry, rz);
    if (GEOM == LW_GEOM_EXACT) {
        const PixGeo &g = p.g;
        const double s = fma(g.nz, rz, fma(g.ny, ry, g.nx * rx));
        if (FORM == kTauShort) {
            const double p2 = fma(-s, s, rr);
            const double k1 = 0.5 * C * g.invD;  // loop invariants
            const double k2 = k1 * g.invD;
            tau = fma(p2, fma(s, k2, k1), tau);
        } else if (FORM == kTauSeries) {
            const double p2 = fma(-s, s, rr);
            const double x = s * g.invD;
            const double h = fma(x, fma(x, x + 1.0, 1.0), 1.0);
            const double y = g.invD * h;
            const double py = p2 * y;
            const double q = py * y;
            tau = fma(py, fma(q, -0.125 * C, 0.5 * C), tau);
        } else {
            const double px = fma(-s, g.nx, rx), py = fma(-s, g.ny, ry), pz = fma(-s, g.nz, rz);
            const double p2 = fma(pz, pz, fma(py, py, px * px));
            const double ds = g.D - s;
            const double R = sqrt(fma(ds, ds, p2));
            tau += p2 * C / (R + ds);
        }
    }
    return tau;
}

// The series forms as polynomials in b for pixels at one distance D (the scan's records):
// with s = z - b/C, |r_perp|^2 = (rho + 2 z' b - b^2)/C^2 (rho = C^2 (x^2 + y^2), z' = C z),
// x = s/D = u - e b (u = z/D, e = 1/(C D)) and K = e/2,
//   kTauShort:  corr = K P (1 + x)                                    (degree 3 in b)
//   kTauSeries: corr = K P [(1 + x + x^2 + x^3) - (P e^2/4)(1 + 3 x)]  (degree 5 in b)
// with P = rho + 2 z' b - b^2 (the same truncations as arrival_tau's series forms), and
// tau(b) = d + b + corr(b) = sum_j c[j] b^j.  The leading coefficient does not depend on the
// sample (K e, resp. 7 K e^3/4).
template <int DEG>
__host__ __device__ __forceinline__ void tau_poly(double d, double x, double y, double z, double C, double D,
                                                  double *c)
{
    const double zp = C * z, cx = C * x, cy = C * y;
    const double rho = fma(cy, cy, cx * cx);
    const double e = 1.0 / (C * D), K = 0.5 * e, u = z / D;
    const double P[3] = {rho, 2.0 * zp, -1.0};
    double T[4] = {0.0, 0.0, 0.0, 0.0};  // the bracket, a polynomial in b
    if (DEG == 3) {
        T[0] = 1.0 + u;
        T[1] = -e;
    } else {
        // S(x) = 1 + x + x^2 + x^3 with x = u - e b
        const double u2 = u * u, e2 = e * e;
        T[0] = 1.0 + u + u2 + u2 * u;
        T[1] = -e * (1.0 + 2.0 * u + 3.0 * u2);
        T[2] = e2 * (1.0 + 3.0 * u);
        T[3] = -e2 * e;
        // minus (e^2/4) P (1 + 3u - 3e b)
        const double f = 0.25 * e2, a0 = 1.0 + 3.0 * u, a1 = -3.0 * e;
        T[0] -= f * (P[0] * a0);
        T[1] -= f * (P[0] * a1 + P[1] * a0);
        T[2] -= f * (P[1] * a1 + P[2] * a0);
        T[3] -= f * (P[2] * a1);
    }
    for (int j = 0; j <= DEG; ++j) c[j] = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j + i <= DEG && j < 4; ++j) c[i + j] += K * (P[i] * T[j]);
    c[0] += d;
    c[1] += 1.0;
}

// Lienard-Wiechert field of one sample at one pixel.  Geometry (n, R, n - beta, kappa) in
// double; the field arithmetic in T.  kappa = 1 - n.b is formed as (1-b^2)/(1+|b|) + |b||n - b^|^2/2.
template <typename T, int GEOM>
__device__ __forceinline__ void lw_field(const PixGeo &g, const double *xm, double rx, double ry, double rz,
                                         double bx, double by, double bz, double ax, double ay, double az, double q,
                                         int fmask, T &Ex, T &Ey, T &Ez, double *kappa_out = nullptr)
{
    // single-precision fields need one Newton step of the reciprocal square roots (relative
    // error ~1e-13, far below float rounding of n - beta and kappa); double fields take two
    constexpr int kNR = sizeof(T) == 4 ? 1 : 2;
    double nx, ny, nz, iR;
    if (GEOM == LW_GEOM_EXACT) {
        double dx = xm[0] - rx, dy = xm[1] - ry, dz = xm[2] - rz;
        iR = rsqrt_nr<kNR>(dx * dx + dy * dy + dz * dz);
        nx = dx * iR;
        ny = dy * iR;
        nz = dz * iR;
    } else {
        nx = g.nx;
        ny = g.ny;
        nz = g.nz;
        iR = g.invD;
    }
    double b2 = bx * bx + by * by + bz * bz;
    double kappa = 1.0;
    if (b2 > 0.0) {
        // 1 - n.b = (1 - |b|) + |b| |n - b/|b||^2 / 2 for a unit n, with no cancellation of
        // the O(1/gamma^2) result against O(1) terms
        const double ib = rsqrt_nr<kNR>(b2), bn = b2 * ib;
        double dx = nx - bx * ib, dy = ny - by * ib, dz = nz - bz * ib;
        kappa = (1.0 - bn) + 0.5 * bn * (dx * dx + dy * dy + dz * dz);
    }
    if (kappa_out) *kappa_out = kappa;
    T pk;  // q/(4 pi eps0 kappa^3)
    if constexpr (sizeof(T) == 4) {
        // kappa is exact to double rounding here; its reciprocal in float: hardware estimate
        // and one Newton step (~1 ulp)
        const float kf = (float)kappa;
        float ikf = __builtin_amdgcn_rcpf(kf);
        ikf = fmaf(fmaf(-kf, ikf, 1.0f), ikf, ikf);
        pk = (float)(q * kCoulomb) * (ikf * ikf * ikf);
    } else {
        const double ik = 1.0 / kappa;
        pk = q * kCoulomb * ik * ik * ik;
    }
    T tnx = (T)nx, tny = (T)ny, tnz = (T)nz;
    // n - beta in double: n_z - beta_z ~ 1/(2 gamma^2) would lose most of its bits in float
    T mx = (T)(nx - bx), my = (T)(ny - by), mz = (T)(nz - bz);
    Ex = Ey = Ez = (T)0;
    if (fmask & LW_FIELD_VELOCITY) {
        T f = pk * (T)((1.0 - b2) * iR * iR);
        Ex += f * mx;
        Ey += f * my;
        Ez += f * mz;
    }
    if (fmask & LW_FIELD_ACCEL) {
        T tax = (T)ax, tay = (T)ay, taz = (T)az;
        // w = (n - b) x bd ; v = n x w
        T wx = my * taz - mz * tay, wy = mz * tax - mx * taz, wz = mx * tay - my * tax;
        T vx = tny * wz - tnz * wy, vy = tnz * wx - tnx * wz, vz = tnx * wy - tny * wx;
        T f = pk * (T)(iR * kInvC);
        Ex += f * vx;
        Ey += f * vy;
        Ez += f * vz;
    }
}

// Vector-Jacobian product of lw_field (double): given g = dJ/dE at one (sample, pixel), adds
// dJ/dr, dJ/dbeta, dJ/dbeta_dot to gr, gb, ga.  Reverse mode written from the field formula
// E = P [F_vel (1-b^2)(n-b)/(kappa^3 R^2) + F_acc n x ((n-b) x a)/(c kappa^3 R)], kappa = 1 - n.b,
// with n = (x - r)/R, R = |x - r| (exact geometry) or n, R fixed (far field).  g_kappa adds a
// gradient with respect to kappa itself (used where kappa multiplies E outside the field).
template <int GEOM>
__device__ __forceinline__ void lw_field_vjp(const PixGeo &g, const double *xm, const double *r, const double *b,
                                             const double *a, double q, int fmask, const double *gE, double *gr,
                                             double *gb, double *ga, double g_kappa = 0.0)
{
    double n[3], R;
    if (GEOM == LW_GEOM_EXACT) {
        const double d0 = xm[0] - r[0], d1 = xm[1] - r[1], d2 = xm[2] - r[2];
        R = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
        n[0] = d0 / R;
        n[1] = d1 / R;
        n[2] = d2 / R;
    } else {
        n[0] = g.nx;
        n[1] = g.ny;
        n[2] = g.nz;
        R = g.D;
    }
    const double b2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    const double bn = sqrt(b2);
    double kappa = 1.0;
    if (bn > 0.0) {
        const double ib = 1.0 / bn;
        const double e0 = n[0] - b[0] * ib, e1 = n[1] - b[1] * ib, e2 = n[2] - b[2] * ib;
        kappa = (1.0 - b2) / (1.0 + bn) + 0.5 * bn * (e0 * e0 + e1 * e1 + e2 * e2);
    }
    const double P = q * kCoulomb;
    const double k3 = kappa * kappa * kappa;
    const double nb[3] = {n[0] - b[0], n[1] - b[1], n[2] - b[2]};
    double gn[3] = {0, 0, 0}, gnb[3] = {0, 0, 0}, gk = g_kappa, gR = 0.0, gbb[3] = {0, 0, 0};
    if (fmask & LW_FIELD_ACCEL) {
        const double w[3] = {nb[1] * a[2] - nb[2] * a[1], nb[2] * a[0] - nb[0] * a[2], nb[0] * a[1] - nb[1] * a[0]};
        const double v[3] = {n[1] * w[2] - n[2] * w[1], n[2] * w[0] - n[0] * w[2], n[0] * w[1] - n[1] * w[0]};
        const double sa = P / (kC * k3 * R);
        const double gsa = gE[0] * v[0] + gE[1] * v[1] + gE[2] * v[2];
        const double gv[3] = {sa * gE[0], sa * gE[1], sa * gE[2]};
        // v = n x w : gn += w x gv ; gw = gv x n
        gn[0] += w[1] * gv[2] - w[2] * gv[1];
        gn[1] += w[2] * gv[0] - w[0] * gv[2];
        gn[2] += w[0] * gv[1] - w[1] * gv[0];
        const double gw[3] = {gv[1] * n[2] - gv[2] * n[1], gv[2] * n[0] - gv[0] * n[2], gv[0] * n[1] - gv[1] * n[0]};
        // w = nb x a : gnb += a x gw ; ga += gw x nb
        gnb[0] += a[1] * gw[2] - a[2] * gw[1];
        gnb[1] += a[2] * gw[0] - a[0] * gw[2];
        gnb[2] += a[0] * gw[1] - a[1] * gw[0];
        ga[0] += gw[1] * nb[2] - gw[2] * nb[1];
        ga[1] += gw[2] * nb[0] - gw[0] * nb[2];
        ga[2] += gw[0] * nb[1] - gw[1] * nb[0];
        gk += gsa * (-3.0 * sa / kappa);
        gR += gsa * (-sa / R);
    }
    if (fmask & LW_FIELD_VELOCITY) {
        const double sv = P * (1.0 - b2) / (k3 * R * R);
        const double gsv = gE[0] * nb[0] + gE[1] * nb[1] + gE[2] * nb[2];
        for (int c = 0; c < 3; ++c) gnb[c] += sv * gE[c];
        const double gb2 = gsv * (-P / (k3 * R * R));
        gk += gsv * (-3.0 * sv / kappa);
        gR += gsv * (-2.0 * sv / R);
        for (int c = 0; c < 3; ++c) gbb[c] += 2.0 * gb2 * b[c];
    }
    for (int c = 0; c < 3; ++c) {
        gn[c] += gnb[c] - gk * b[c];
        gbb[c] += -gnb[c] - gk * n[c];
        gb[c] += gbb[c];
    }
    if (GEOM == LW_GEOM_EXACT) {
        const double gnn = gn[0] * n[0] + gn[1] * n[1] + gn[2] * n[2];
        for (int c = 0; c < 3; ++c) gr[c] -= (gn[c] - gnn * n[c]) / R + gR * n[c];
    }
}

__device__ __forceinline__ bool sample_usable(const double *r, const double *b, const double *a)
{
    bool ok = true;
#pragma unroll
    for (int c = 0; c < 3; ++c) ok = ok && isfinite(r[c]) && isfinite(b[c]) && isfinite(a[c]);
    return ok && (b[0] * b[0] + b[1] * b[1] + b[2] * b[2] < 1.0);
}

__device__ __forceinline__ void atomic_add(float *p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(double *p, double v) { unsafeAtomicAdd(p, v); }

// How the deposit adds a contribution v to trace element j.  kAccFloat: a floating-point atomic
// add (the result depends on the order of arrival in its last bits).  The two modes of the
// order-independent FP64 deposit: kAccMaxAbs keeps max |v| per element (as the bits of a
// non-negative double, which order like unsigned integers); kAccFixed adds round(v * scale[row])
// to a 128-bit two's-complement fixed-point sum per element, low words in the trace, high words
// in DetAcc::hi.  Integer sums do not depend on the order of their terms.
enum { kAccFloat = 0, kAccMaxAbs = 1, kAccFixed = 2 };
struct DetAcc {
    unsigned long long *hi;  // [n_pix][3][n_obs] high words (kAccFixed)
    const double *scale;     // [n_pix][3] power of two per trace row (kAccFixed)
};

// host-side launch helpers (defined in the kernel files)
// sample0: index of the first sample of traj within a longer trajectory (its arrival times use
// t_start + (sample0 + i) dt); 0 for whole trajectories.  rbound2: per particle, max |r|^2 over
// the whole trajectory (nullptr: the max over the samples given), which decides the series forms
// of the arrival time per particle and pixel.
lw_status launch_deposit(const lw_traj_t *traj, const lw_grid_t *grid, int prec, int field_mask, int geom,
                         bool accumulate, void *E, int64_t *diag, void *ws, size_t ws_bytes, hipStream_t s,
                         int64_t sample0 = 0, const double *rbound2 = nullptr, int acc_mode = kAccFloat,
                         DetAcc det = DetAcc{nullptr, nullptr});
// lw_deposit_td_det: FP64 deposit whose result does not depend on the order of the contributions
// (acc: the high words and row scales, det_acc_bytes(n_pix, n_obs) bytes)
lw_status launch_deposit_det(const lw_traj_t *traj, const lw_grid_t *grid, int field_mask, int geom, double *E,
                             int64_t *diag, void *acc, void *ws, size_t ws_bytes, hipStream_t s);
size_t det_acc_bytes(int64_t n_pix, int64_t n_obs);
// workspace of a deposit launch that holds the records of all its particles (a smaller one makes
// it process the particles in chunks)
size_t deposit_ws_bytes(int64_t n_particles, int64_t n_samples, int prec);
lw_status launch_fft(const void *E, int64_t n_pix, int64_t n_obs, double dt_obs, int prec, void *S, void *ws,
                     size_t ws_bytes, hipStream_t s);
size_t fft_ws_bytes(int64_t n_pix, int64_t n_obs, int prec);
// lw_spectrum_fft with the library's static scratch array instead of a workspace
lw_status launch_fft_noalloc(const void *E, int64_t n_pix, int64_t n_obs, double dt_obs, int prec, void *S,
                             hipStream_t s);
size_t fft_noalloc_scratch_bytes();
lw_status launch_fft_bwd(const void *E, const void *dS, int64_t n_pix, int64_t n_obs, double dt_obs, int prec,
                         void *dE, void *ws, size_t ws_bytes, hipStream_t s);
lw_status launch_direct_fd(const lw_traj_t *traj, const lw_grid_t *grid, const double *omega, int64_t n_omega,
                           int prec, int field_mask, int geom, double *S, void *ws, size_t ws_bytes, hipStream_t s);
lw_status launch_direct_fd_bwd(const lw_traj_t *traj, const lw_grid_t *grid, const double *omega, int64_t n_omega,
                               int field_mask, int geom, const double *dS, double *d_r, double *d_beta,
                               double *d_beta_dot, void *ws, size_t ws_bytes, hipStream_t s);
size_t direct_fd_ws_bytes(int64_t n_pix, int64_t n_omega);
lw_status launch_boris(const lw_traj_t *traj, double *r, double *beta, double *beta_dot, hipStream_t s);
// max |r|^2 over every sample of each trajectory of traj (LW_TRAJ_BORIS), [n_particles]
lw_status launch_boris_rmax2(const lw_traj_t *traj, double *rmax2, hipStream_t s);
// samples s0 .. s0 + n_span - 1 of every particle of traj (LW_TRAJ_BORIS), starting from init
// (s0 = 0) or from the pusher state [n_particles][9] left by the span that ended at sample s0
lw_status launch_boris_span(const lw_traj_t *traj, int64_t s0, int64_t n_span, double *state, double *r,
                            double *beta, double *beta_dot, hipStream_t s);
lw_status launch_boris_bwd(const lw_traj_t *traj, const double *g_r, const double *g_beta,
                           const double *g_beta_dot, double *grad_init, double *grad_a0, hipStream_t s);
// the pusher's tangents over samples s0 .. s0 + n_span - 1 (gradients g_* [n_particles][n_span][3]),
// their state [n_particles][7][18] carried between spans; the first span (s0 = 0) writes
// grad_init, grad_a0, later ones add to them
lw_status launch_boris_bwd_span(const lw_traj_t *traj, int64_t s0, int64_t n_span, double *tstate,
                                const double *g_r, const double *g_beta, const double *g_beta_dot, double *grad_init,
                                double *grad_a0, hipStream_t s);
// adjoint of the deposit; rbound2 as for launch_deposit (nullptr: computed from the samples into
// ws, which then needs deposit_bwd_ws_bytes(n_particles) bytes)
lw_status launch_deposit_bwd(const lw_traj_t *traj, const lw_grid_t *grid, int field_mask, int geom, const double *dE,
                             double *d_r, double *d_beta, double *d_beta_dot, void *ws, size_t ws_bytes,
                             hipStream_t s, int64_t sample0 = 0, const double *rbound2 = nullptr);
size_t deposit_bwd_ws_bytes(int64_t n_particles);
// trajectories recomputed from LW_TRAJ_BORIS initial conditions (boris_stream.hip): the deposit
// and its adjoint push batches of particles over spans of samples.
struct BorisPlan {
    int64_t batch, span;  // particles per batch, samples per span (spans share their boundary sample)
};
// bwd: the adjoint's plan (sample arrays and their gradients, tangent states)
BorisPlan boris_plan_default(int64_t n_p, int64_t ns, int prec, bool bwd = false);
BorisPlan boris_plan_fit(int64_t n_p, int64_t ns, int64_t span_req, size_t ws_bytes, int prec, bool bwd = false);
size_t boris_plan_ws_bytes(const BorisPlan &p, int prec, bool bwd = false);
lw_status launch_deposit_boris(const lw_traj_t *t, const lw_grid_t *gr, int prec, int fmask, int geom,
                               bool accumulate, void *E, int64_t *diag, void *ws, size_t ws_bytes, hipStream_t s,
                               int acc_mode = kAccFloat, DetAcc det = DetAcc{nullptr, nullptr});
lw_status launch_deposit_bwd_boris(const lw_traj_t *t, const lw_grid_t *gr, int fmask, int geom, const double *dE,
                                   double *grad_init, double *grad_a0, void *ws, size_t ws_bytes, hipStream_t s);

}  // namespace lw
