/*
 * lw_oracle.c -- plain FP64 CPU oracle for the time-domain Lienard-Wiechert
 * spectrum method of Kan, Kaertner, Le Borne, Ruprecht and Zemke,
 * "Parallel computation of inverse Compton scattering radiation spectra based
 * on Lienard-Wiechert potentials" (arXiv:2206.03015).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header, table or constant
 * with the HIP library: every constant and formula below is written out here
 * from the paper (and the textbook relations it cites).
 *
 * Everything is IEEE double, no fast-math, loops in the obvious order.  The
 * only parallelism is an OpenMP loop over observers (the paper's detector
 * decomposition, Sec. "Parallelization"), which does not change any result:
 * each observer is computed by one thread in a fixed order.
 *
 * Parity status of each function (what pins it) is listed in oracle/__init__.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* CODATA 2018 exact / recommended values (SI). */
#define O_C 299792458.0
#define O_QE 1.602176634e-19
#define O_EPS0 8.8541878128e-12
#define O_ME 9.1093837015e-31
#define O_PI 3.14159265358979323846

#define O_FIELD_ACCEL 1
#define O_FIELD_VELOCITY 2
#define O_GEOM_EXACT 0
#define O_GEOM_FARFIELD 1

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* A sample is usable when all nine numbers are finite and |beta| < 1. */
static int sample_ok(const double *r, const double *b, const double *bd)
{
    for (int c = 0; c < 3; ++c)
        if (!isfinite(r[c]) || !isfinite(b[c]) || !isfinite(bd[c])) return 0;
    return dot3(b, b) < 1.0;
}

/*
 * Field of one charge sample seen by one observer.
 *
 * Observer at x (|x| = D, n_m = x/D).  Emission at time t from position r with
 * velocity beta = v/c and normalised acceleration beta_dot = a/c (1/s).
 *
 * Output tt: the advanced (arrival) time minus t minus D/c, i.e. the shift
 * that, added to the emission time t, gives the observer time measured from
 * D/c.
 *   - far field (Eq. far_adv, the approximation the paper uses throughout):
 *         tt = -n_m . r / c,   n = n_m,   R := D           (Eqs. far_efield, far_adv)
 *   - exact geometry (Eq. advanced_condition, t_a = t + |x - r|/c):
 *         tt = (R - D)/c with R = |x - r|, written through the exact identity
 *         R - D = -s + |r - s n_m|^2 / (R + D - s),  s = n_m . r,
 *         which has no cancellation; n = (x - r)/R.
 * Output E (V/m), Lienard-Wiechert field (Eq. lw_fields_retarded for the
 * acceleration part; the velocity part is the Coulomb-like term the paper
 * drops, Jackson Eq. 14.14):
 *     E = q/(4 pi eps0) [ F_vel (1-b^2)(n-b) / (kappa^3 R^2)
 *                        + F_acc n x ((n-b) x bd) / (c kappa^3 R) ]
 * with kappa = 1 - n.b formed as (1-b^2)/(1+|b|) + |b| |n - b/|b||^2 / 2,
 * an exact identity for unit n that avoids the cancellation of 1 - n.b near
 * |b| = 1.  kappa is returned too (the Jacobian dt_a/dt of Eq. const_phase_drop).
 */
static void eval_one(const double *x, const double *r, const double *b, const double *bd, double q, int fmask,
                     int geom, double *tt, double *E, double *kappa_out)
{
    double D = sqrt(dot3(x, x));
    double nm[3] = {x[0] / D, x[1] / D, x[2] / D};
    double s = dot3(nm, r);
    double n[3], R;
    if (geom == O_GEOM_FARFIELD) {
        n[0] = nm[0];
        n[1] = nm[1];
        n[2] = nm[2];
        R = D;
        *tt = -s / O_C;
    } else {
        double rp[3] = {r[0] - s * nm[0], r[1] - s * nm[1], r[2] - s * nm[2]};
        double dx[3] = {x[0] - r[0], x[1] - r[1], x[2] - r[2]};
        R = sqrt(dot3(dx, dx));
        n[0] = dx[0] / R;
        n[1] = dx[1] / R;
        n[2] = dx[2] / R;
        *tt = -s / O_C + dot3(rp, rp) / (O_C * (R + D - s));
    }
    double b2 = dot3(b, b);
    double bn = sqrt(b2);
    double kappa;
    if (bn > 0.0) {
        double d[3] = {n[0] - b[0] / bn, n[1] - b[1] / bn, n[2] - b[2] / bn};
        kappa = (1.0 - b2) / (1.0 + bn) + 0.5 * bn * dot3(d, d);
    } else {
        kappa = 1.0;
    }
    double pref = q / (4.0 * O_PI * O_EPS0);
    double k3 = kappa * kappa * kappa;
    E[0] = E[1] = E[2] = 0.0;
    double nb[3] = {n[0] - b[0], n[1] - b[1], n[2] - b[2]};
    if (fmask & O_FIELD_VELOCITY) {
        double f = pref * (1.0 - b2) / (k3 * R * R);
        for (int c = 0; c < 3; ++c) E[c] += f * nb[c];
    }
    if (fmask & O_FIELD_ACCEL) {
        double w[3], v[3];
        cross3(nb, bd, w);
        cross3(n, w, v);
        double f = pref / (O_C * k3 * R);
        for (int c = 0; c < 3; ++c) E[c] += f * v[c];
    }
    if (kappa_out) *kappa_out = kappa;
}

/*
 * Arrival time of sample i (emitted at t_i = t_start + i*dt from r) at observer x, in grid units
 * of the observer grid that starts at |x|/c + t0:
 *     exact (Eq. advanced_condition):  tau = (t_i + (|x - r| - |x|)/c - t0) / dt_obs
 *     far field (Eq. far_adv):         tau = (t_i - n_m.r/c - t0) / dt_obs
 * The definition is a real-number relation between the double inputs.  Its two large terms,
 * t_i/dt_obs and n_m.r/(c dt_obs), reach ~1e8 grid units at the largest workloads and cancel to
 * the size of the window, so one double rounding of them moves tau by ~1e-8 grid units, far
 * more than the 1e-10 spectral agreement asked of double-precision results.  The oracle
 * therefore forms this one expression in long double (x87, 64-bit significand: ~1e-11 grid
 * units), with |x - r| - |x| through the cancellation-free identity of eval_one.
 */
/* the arrival time minus |x|/c + t0, in seconds */
static long double arrival_time_ld(const double *x, const double *r, double t_start, double dt, int64_t i, double t0,
                                   int geom)
{
    const long double c = O_C;
    long double X[3] = {x[0], x[1], x[2]}, Rv[3] = {r[0], r[1], r[2]};
    long double D = sqrtl(X[0] * X[0] + X[1] * X[1] + X[2] * X[2]);
    long double n[3] = {X[0] / D, X[1] / D, X[2] / D};
    long double s = n[0] * Rv[0] + n[1] * Rv[1] + n[2] * Rv[2];
    long double shift;
    if (geom == O_GEOM_FARFIELD) {
        shift = -s / c;
    } else {
        long double rp[3] = {Rv[0] - s * n[0], Rv[1] - s * n[1], Rv[2] - s * n[2]};
        long double d[3] = {X[0] - Rv[0], X[1] - Rv[1], X[2] - Rv[2]};
        long double R = sqrtl(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        shift = (-s + (rp[0] * rp[0] + rp[1] * rp[1] + rp[2] * rp[2]) / (R + D - s)) / c;
    }
    long double ti = (long double)t_start + (long double)i * (long double)dt;
    return ti + shift - (long double)t0;
}

static double arrival_tau_ld(const double *x, const double *r, double t_start, double dt, int64_t i, double t0,
                             double dt_obs, int geom)
{
    return (double)(arrival_time_ld(x, r, t_start, dt, i, t0, geom) / (long double)dt_obs);
}

/* Exported arrival time of single samples (used by the precision pin): tau[j] for x[j], r[j], i[j]. */
void orc_arrival_tau(int64_t n, const double *x, const double *r, const int64_t *i, double t_start, double dt,
                     double t0, double dt_obs, int geom, double *tau)
{
    for (int64_t j = 0; j < n; ++j)
        tau[j] = arrival_tau_ld(x + 3 * j, r + 3 * j, t_start, dt, i[j], t0, dt_obs, geom);
}

/* Exported single-sample evaluation (used by the closed-form pins). */
void orc_eval(const double *x, const double *r, const double *b, const double *bd, double q, int fmask, int geom,
              double *tt, double *E, double *kappa)
{
    eval_one(x, r, b, bd, q, fmask, geom, tt, E, kappa);
}

/*
 * Time-domain deposit: Algorithm 2 ("Proposed Time-Domain Method") with the
 * paper's piecewise-linear interpolation (Sec. "Interpolation").
 *
 * Observer grid of pixel m: t_u = D_m/c + t0 + u*dt_obs, u = 0..n_obs-1.
 * Sample i of particle k is emitted at t_i = t_start + i*dt (multiplied, not
 * accumulated) and arrives at tau_i = (t_i + tt_i - t0)/dt_obs in grid units.
 *
 * Readings of the algorithm (the text's listing leaves these open):
 *   - the one-step buffer is primed by sample 0: the first interval is
 *     (tau_0, tau_1]; nothing is deposited before tau_0 or after tau_last;
 *   - the buffer update belongs to the per-particle body;
 *   - interval (tau_{i-1}, tau_i] is half-open; grid point u in it receives
 *     (1-w) E_{i-1} + w E_i with w = (u - tau_{i-1})/(tau_i - tau_{i-1});
 *   - an interval with tau_i <= tau_{i-1} is skipped and counted (diag[0]);
 *   - an interval touching an unusable sample (non-finite value, |beta| >= 1,
 *     or a non-finite tau) is skipped and counted (diag[1]);
 *   - grid points of deposited intervals that fall outside [0, n_obs) are
 *     dropped and counted (diag[2]); deposited grid points are counted in
 *     diag[3].
 * Loop order: observer, particle, step.  Contributions are additive, so the
 * order only changes rounding.
 *
 * r, beta, beta_dot: [n_p][n_samples][3].  charge: [n_p] or NULL (-e each).
 * E_tot: [n_pix][3][n_obs], overwritten.  diag: [4].
 */
/*
 * The interpolation step for one particle and one observer: the sample stream
 * tau[0..n-1] (grid units), E[0..n-1][3], ok[0..n-1] is deposited into
 * out[3][n_obs] following the readings above.  cnt[0..3] are incremented as
 * diag[0..3].
 */
static void deposit_stream(int64_t n, const double *tau, const double *E, const unsigned char *ok, int64_t n_obs,
                           double *out, int64_t *cnt)
{
    for (int64_t i = 1; i < n; ++i) {
        if (!ok[i] || !ok[i - 1]) {
            cnt[1] += 1;
            continue;
        }
        double tb = tau[i - 1], ta = tau[i];
        if (!(ta > tb)) {
            cnt[0] += 1;
            continue;
        }
        /* integers u with tb < u <= ta, i.e. floor(tb)+1 .. floor(ta) */
        double ulo = floor(tb) + 1.0, uhi = floor(ta);
        double lo = ulo < 0.0 ? 0.0 : ulo;
        double hi = uhi > (double)(n_obs - 1) ? (double)(n_obs - 1) : uhi;
        double inside = hi >= lo ? hi - lo + 1.0 : 0.0;
        cnt[2] += (int64_t)((uhi - ulo + 1.0) - inside);
        for (double uf = lo; uf <= hi; uf += 1.0) {
            int64_t u = (int64_t)uf;
            double w = (uf - tb) / (ta - tb);
            for (int c = 0; c < 3; ++c) out[(size_t)c * n_obs + u] += (1.0 - w) * E[3 * (i - 1) + c] + w * E[3 * i + c];
            cnt[3] += 1;
        }
    }
}

/* Exported interpolation step alone (tests feed it designed tau/E streams). */
int orc_interp_deposit(int64_t n, const double *tau, const double *E, const unsigned char *ok, int64_t n_obs,
                       double *out, int64_t *diag)
{
    if (n < 0 || n_obs < 1) return -1;
    int64_t cnt[4] = {0, 0, 0, 0};
    deposit_stream(n, tau, E, ok, n_obs, out, cnt);
    for (int j = 0; j < 4; ++j) diag[j] += cnt[j];
    return 0;
}

int orc_deposit_td(int64_t n_p, int64_t n_samples, double t_start, double dt, const double *r, const double *beta,
                   const double *beta_dot, const double *charge, int64_t n_pix, const double *x_det, double t0,
                   double dt_obs, int64_t n_obs, int fmask, int geom, double *E_tot, int64_t *diag)
{
    if (n_p < 0 || n_samples < 0 || n_pix < 0 || n_obs < 1 || !(dt_obs > 0.0)) return -1;
    memset(E_tot, 0, sizeof(double) * (size_t)(n_pix * 3 * n_obs));
    int64_t d0 = 0, d1 = 0, d2 = 0, d3 = 0;
    int fail = 0;
#pragma omp parallel reduction(+ : d0, d1, d2, d3, fail)
    {
        size_t ns = (size_t)(n_samples > 0 ? n_samples : 1);
        double *tau = (double *)malloc(ns * sizeof(double));
        double *Ea = (double *)malloc(ns * 3 * sizeof(double));
        unsigned char *ok = (unsigned char *)malloc(ns);
        if (!tau || !Ea || !ok) fail += 1;
#pragma omp for schedule(dynamic, 1)
        for (int64_t m = 0; m < n_pix; ++m) {
            if (!tau || !Ea || !ok) continue;
            const double *x = x_det + 3 * m;
            double *out = E_tot + (size_t)m * 3 * n_obs;
            int64_t cnt[4] = {0, 0, 0, 0};
            for (int64_t k = 0; k < n_p; ++k) {
                double q = charge ? charge[k] : -O_QE;
                /* evaluate: arrival time and field of every sample (Eqs. far_adv / advanced_condition, far_efield) */
                for (int64_t i = 0; i < n_samples; ++i) {
                    size_t s = (size_t)(k * n_samples + i) * 3;
                    ok[i] = (unsigned char)sample_ok(r + s, beta + s, beta_dot + s);
                    tau[i] = NAN;
                    if (!ok[i]) continue;
                    double tt;
                    eval_one(x, r + s, beta + s, beta_dot + s, q, fmask, geom, &tt, Ea + 3 * i, NULL);
                    tau[i] = arrival_tau_ld(x, r + s, t_start, dt, i, t0, dt_obs, geom);
                    ok[i] = (unsigned char)(isfinite(tau[i]) && isfinite(Ea[3 * i]) && isfinite(Ea[3 * i + 1]) &&
                                            isfinite(Ea[3 * i + 2]));
                }
                /* interpolate onto the uniform observer grid and superimpose */
                deposit_stream(n_samples, tau, Ea, ok, n_obs, out, cnt);
            }
            d0 += cnt[0];
            d1 += cnt[1];
            d2 += cnt[2];
            d3 += cnt[3];
        }
        free(tau);
        free(Ea);
        free(ok);
    }
    if (fail) return -2;
    if (diag) {
        diag[0] = d0;
        diag[1] = d1;
        diag[2] = d2;
        diag[3] = d3;
    }
    return 0;
}

/*
 * Per-sample arrival times and fields, for tests: tau[n_pix][n_p][n_samples]
 * (grid units) and E[n_pix][n_p][n_samples][3].  Unusable samples give NaN.
 */
int orc_eval_samples(int64_t n_p, int64_t n_samples, double t_start, double dt, const double *r, const double *beta,
                     const double *beta_dot, const double *charge, int64_t n_pix, const double *x_det, double t0,
                     double dt_obs, int fmask, int geom, double *tau, double *E, double *kappa)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t m = 0; m < n_pix; ++m) {
        for (int64_t k = 0; k < n_p; ++k) {
            double q = charge ? charge[k] : -O_QE;
            for (int64_t i = 0; i < n_samples; ++i) {
                size_t s = (size_t)(k * n_samples + i);
                size_t o = (size_t)((m * n_p + k) * n_samples + i);
                if (!sample_ok(r + 3 * s, beta + 3 * s, beta_dot + 3 * s)) {
                    tau[o] = NAN;
                    E[3 * o] = E[3 * o + 1] = E[3 * o + 2] = NAN;
                    if (kappa) kappa[o] = NAN;
                    continue;
                }
                double tt, kap;
                eval_one(x_det + 3 * m, r + 3 * s, beta + 3 * s, beta_dot + 3 * s, q, fmask, geom, &tt, E + 3 * o,
                         &kap);
                tau[o] = arrival_tau_ld(x_det + 3 * m, r + 3 * s, t_start, dt, i, t0, dt_obs, geom);
                if (kappa) kappa[o] = kap;
            }
        }
    }
    return 0;
}

/*
 * Direct frequency-domain sum (Eq. inty_dft with the abbreviations of
 * Eq. freq:far_field_freq, Algorithm 1), generalised to the exact geometry and
 * the velocity term by using the integrand E(t_a) dt_a/dt = E kappa:
 *
 *   F_c(w) = (dt / sqrt(2 pi)) sum_k sum_{i=0}^{N_s} E_{k,i,c} kappa_{k,i}
 *                                       exp(+j w (t_i + tt_{k,i} - t0))
 *   S(w)   = sum_c |F_c(w)|^2
 *
 * All n_samples = N_s + 1 samples enter with weight dt (the rectangle rule of
 * Eq. inty_dft, whose index runs from 0; the later abbreviations start at 1).
 * In the far field with the acceleration term only, E kappa equals
 * q A_k / (4 pi eps0 c D) with A_k of Eq. const_phase_drop, so that
 * 2 eps0 c D^2 S(w) is exactly the right-hand side of Eq. inty_dft (the
 * spectral-angular intensity).  Unusable samples are skipped.  The phase origin t0 only
 * multiplies each F_c(w) by a unit phasor.
 * S: [n_pix][n_omega].
 */
int orc_direct_fd(int64_t n_p, int64_t n_samples, double t_start, double dt, const double *r, const double *beta,
                  const double *beta_dot, const double *charge, int64_t n_pix, const double *x_det, double t0,
                  const double *omega, int64_t n_omega, int fmask, int geom, double *S)
{
    double *acc_all = (double *)calloc((size_t)n_pix * (size_t)n_omega * 6, sizeof(double));
    if (!acc_all) return -2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t m = 0; m < n_pix; ++m) {
        double *acc = acc_all + (size_t)m * n_omega * 6;
        for (int64_t k = 0; k < n_p; ++k) {
            double q = charge ? charge[k] : -O_QE;
            for (int64_t i = 0; i < n_samples; ++i) {
                size_t s = (size_t)(k * n_samples + i);
                if (!sample_ok(r + 3 * s, beta + 3 * s, beta_dot + 3 * s)) continue;
                double tt, Ev[3], kap;
                eval_one(x_det + 3 * m, r + 3 * s, beta + 3 * s, beta_dot + 3 * s, q, fmask, geom, &tt, Ev, &kap);
                /* arrival time relative to t0 (s), in the extended precision of arrival_tau_ld, and
                   the phase reduced to one revolution before its cosine and sine */
                long double ta = arrival_time_ld(x_det + 3 * m, r + 3 * s, t_start, dt, i, t0, geom);
                for (int64_t w = 0; w < n_omega; ++w) {
                    long double cyc = (long double)omega[w] * ta / (2.0L * 3.14159265358979323846264338327950288L);
                    cyc -= floorl(cyc);
                    double ph = (double)(cyc * 2.0L * 3.14159265358979323846264338327950288L);
                    double cs = cos(ph), sn = sin(ph);
                    for (int c = 0; c < 3; ++c) {
                        acc[6 * w + 2 * c] += Ev[c] * kap * cs;
                        acc[6 * w + 2 * c + 1] += Ev[c] * kap * sn;
                    }
                }
            }
        }
        double f = dt * dt / (2.0 * O_PI);
        for (int64_t w = 0; w < n_omega; ++w) {
            double sum = 0.0;
            for (int c = 0; c < 6; ++c) sum += acc[6 * w + c] * acc[6 * w + c];
            S[m * n_omega + w] = f * sum;
        }
    }
    free(acc_all);
    return 0;
}

/*
 * Laser field used to drive the trajectories.  The paper only says "sinusoidal
 * plane wave" and integrates the equations of motion with the Boris method;
 * the pulse model below is this code's reading (counter-propagating along -z,
 * x-polarised, sin^2 envelope of n_cycles periods centred on phase 0, optional
 * zeroth-order Gaussian transverse profile of waist w0; w0 <= 0 = plane wave).
 * It is written through the normalised vector potential
 *     a_x(phi) = a0 g(phi) sin(phi),  g = cos^2(phi/(2 n_cycles)) for |phi| < pi n_cycles,
 *     phi = omega_L (t + z/c),
 * so that E_x = -E0 T(rho) d(g sin)/dphi, B_y = -E_x/c, E0 = a0 m_e c omega_L / e,
 * T = exp(-(x^2+y^2)/w0^2).  For the plane wave this makes the analytic
 * trajectory (oracle/trajectory.py) an exact solution of the same equations.
 */
typedef struct {
    double a0, lambda, w0, n_cycles;
} orc_laser;

static void laser_eb(const orc_laser *L, const double *x, double t, double *E, double *B)
{
    E[0] = E[1] = E[2] = B[0] = B[1] = B[2] = 0.0;
    double wl = 2.0 * O_PI * O_C / L->lambda;
    double phi = wl * (t + x[2] / O_C);
    double nc = L->n_cycles;
    if (!(fabs(phi) < O_PI * nc)) return;
    double h = phi / (2.0 * nc);
    double g = cos(h) * cos(h);
    double gp = -sin(phi / nc) / (2.0 * nc);
    double sp = gp * sin(phi) + g * cos(phi);
    double T = 1.0;
    if (L->w0 > 0.0) T = exp(-(x[0] * x[0] + x[1] * x[1]) / (L->w0 * L->w0));
    double E0 = L->a0 * O_ME * O_C * wl / O_QE;
    E[0] = -E0 * T * sp;
    B[1] = -E[0] / O_C;
}

/* One Boris velocity update of u = gamma*beta over time h (charge q, mass m). */
static void boris_kick(double *u, const double *E, const double *B, double q, double m, double h)
{
    double a = q * h / (2.0 * m * O_C);
    double um[3] = {u[0] + a * E[0], u[1] + a * E[1], u[2] + a * E[2]};
    double gm = sqrt(1.0 + dot3(um, um));
    double tv[3] = {q * h * B[0] / (2.0 * m * gm), q * h * B[1] / (2.0 * m * gm), q * h * B[2] / (2.0 * m * gm)};
    double t2 = dot3(tv, tv);
    double sv[3] = {2.0 * tv[0] / (1.0 + t2), 2.0 * tv[1] / (1.0 + t2), 2.0 * tv[2] / (1.0 + t2)};
    double c1[3], up[3], c2[3];
    cross3(um, tv, c1);
    for (int c = 0; c < 3; ++c) up[c] = um[c] + c1[c];
    cross3(up, sv, c2);
    for (int c = 0; c < 3; ++c) u[c] = um[c] + c2[c] + a * E[c];
}

/* normalised acceleration d(beta)/dt for charge q, mass m at velocity b in fields E, B:
 * dbeta/dt = q/(gamma m c) [E + c b x B - b (b.E)] */
static void beta_dot_of(const double *b, const double *E, const double *B, double q, double m, double *bd)
{
    double g = 1.0 / sqrt(1.0 - dot3(b, b));
    double bxB[3];
    cross3(b, B, bxB);
    double be = dot3(b, E);
    double f = q / (g * m * O_C);
    for (int c = 0; c < 3; ++c) bd[c] = f * (E[c] + O_C * bxB[c] - b[c] * be);
}

/*
 * FP64 Boris pusher (the trajectory integrator the paper names; its details
 * are the textbook leap-frog form).  Positions live on t_i = t_start + i dt,
 * momenta u = gamma beta on half steps:
 *   u_{1/2}   = Boris kick of u_0 over dt/2 with the fields at (r_0, t_0)
 *   r_{i+1}   = r_i + c u_{i+1/2}/gamma_{i+1/2} dt
 *   u_{i+3/2} = Boris kick of u_{i+1/2} over dt with the fields at (r_{i+1}, t_{i+1})
 * Sample values: beta_0 from u_0; for i >= 1, beta_i from u_i = (u_{i-1/2} + u_{i+1/2})/2;
 * beta_dot_i from the Lorentz force at (r_i, t_i) with beta_i.
 * init: [n_p][6] = x, y, z (m), ux, uy, uz at t_start.  Electrons (q = -e, m_e).
 */
int orc_boris(int64_t n_p, int64_t n_samples, double t_start, double dt, const double *init, double a0, double lambda,
              double w0, double n_cycles, double *r, double *beta, double *beta_dot)
{
    orc_laser L = {a0, lambda, w0, n_cycles};
    const double q = -O_QE, m = O_ME;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < n_p; ++k) {
        double x[3] = {init[6 * k], init[6 * k + 1], init[6 * k + 2]};
        double us[3] = {init[6 * k + 3], init[6 * k + 4], init[6 * k + 5]}; /* u at the sample time */
        double uh[3] = {us[0], us[1], us[2]};                               /* u half a step later */
        double E[3], B[3];
        laser_eb(&L, x, t_start, E, B);
        boris_kick(uh, E, B, q, m, 0.5 * dt);
        for (int64_t i = 0; i < n_samples; ++i) {
            double ti = t_start + (double)i * dt;
            size_t o = (size_t)(k * n_samples + i) * 3;
            double g = sqrt(1.0 + dot3(us, us));
            double b[3] = {us[0] / g, us[1] / g, us[2] / g};
            laser_eb(&L, x, ti, E, B);
            for (int c = 0; c < 3; ++c) {
                r[o + c] = x[c];
                beta[o + c] = b[c];
            }
            beta_dot_of(b, E, B, q, m, beta_dot + o);
            if (i + 1 == n_samples) break;
            double gh = sqrt(1.0 + dot3(uh, uh));
            for (int c = 0; c < 3; ++c) x[c] += O_C * uh[c] / gh * dt;
            double un[3] = {uh[0], uh[1], uh[2]};
            laser_eb(&L, x, t_start + (double)(i + 1) * dt, E, B);
            boris_kick(un, E, B, q, m, dt);
            for (int c = 0; c < 3; ++c) {
                us[c] = 0.5 * (uh[c] + un[c]);
                uh[c] = un[c];
            }
        }
    }
    return 0;
}

/* Laser fields at given points, for tests: E, B [n][3]. */
void orc_laser_fields(int64_t n, const double *x, const double *t, double a0, double lambda, double w0,
                      double n_cycles, double *E, double *B)
{
    orc_laser L = {a0, lambda, w0, n_cycles};
    for (int64_t j = 0; j < n; ++j) laser_eb(&L, x + 3 * j, t[j], E + 3 * j, B + 3 * j);
}
