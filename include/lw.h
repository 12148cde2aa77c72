/*
 * lw.h -- C ABI of liblw.so: time-domain Lienard-Wiechert radiation spectra
 * on AMD Instinct MI355X (gfx950).
 *
 * Method: Kan, Kaertner, Le Borne, Ruprecht, Zemke, "Parallel computation of
 * inverse Compton scattering radiation spectra based on Lienard-Wiechert
 * potentials", arXiv:2206.03015.  Equation labels below are the paper's.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array pointer is a DEVICE pointer (hipMalloc'd or from a framework
 *    allocator) owned by the caller; the library never frees caller memory and
 *    never keeps a pointer past the call.  The lw_traj_t / lw_grid_t structs
 *    themselves are HOST memory, read during the call only.
 *  - Every call validates its arguments on the host, then enqueues kernels on
 *    `stream` and returns without synchronising.  A non-zero status means that
 *    nothing was enqueued, except LW_E_HIP (a HIP launch failed; the stream may
 *    hold part of the work).  No C++ exception crosses the ABI.
 *  - lw_last_error() returns a thread-local description of the last failure.
 *  - Device pointers must be 8-byte aligned (16-byte for E/S/dE/dS).
 *  - Units are SI throughout (m, s, V/m).  beta = v/c, beta_dot = dbeta/dt (1/s).
 *  - Calls that share output buffers must not run concurrently.
 *
 * Observer grid (Sec. "Time-Domain Method", Eqs. tu_min, tu_max): pixel m at
 * x_m receives samples at t_u = |x_m|/c + t0 + u*dt_obs, u = 0..n_obs-1.  t0 is
 * measured from |x_m|/c so that no call ever forms 3.3 ns - 3.3 ns differences.
 */
#ifndef LW_H
#define LW_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LW_OK = 0,
    LW_E_ARG = -1,         /* NULL pointer or value out of range             */
    LW_E_SHAPE = -2,       /* inconsistent or unsupported sizes              */
    LW_E_ALIGN = -3,       /* misaligned device pointer                      */
    LW_E_WORKSPACE = -4,   /* workspace too small (see lw_workspace_bytes)   */
    LW_E_HIP = -5,         /* a HIP runtime call failed                      */
    LW_E_UNSUPPORTED = -6  /* combination not implemented                    */
} lw_status;

/* precision: LW_PREC_FP64 = everything in double; LW_PREC_MIXED = arrival
 * times (tau) in double, fields, trace, FFT and spectrum in float. */
#define LW_PREC_FP64 0
#define LW_PREC_MIXED 1

/* field terms (bit mask): the paper keeps the acceleration ("radiation")
 * term of Eq. lw_fields_retarded and drops the velocity term. */
#define LW_FIELD_ACCEL 1
#define LW_FIELD_VELOCITY 2

/* geometry: exact = Eq. advanced_condition with n = (x - r)/|x - r|;
 * far field = Eqs. far_efield, far_adv (n = x/|x| fixed, |x - r| ~ |x| - n.r). */
#define LW_GEOM_EXACT 0
#define LW_GEOM_FARFIELD 1

/* flag OR-ed into the geometry argument of lw_deposit_td: add into E (and
 * diag) instead of overwriting them (for particle-chunked calls). */
#define LW_ACCUMULATE (1 << 8)

/* flag OR-ed into the geometry argument of lw_deposit_td: skip every particle whose
 * arrival times at a wavefront's pixels hold no observer grid point (tested on the
 * first and last sample where the arrival times are provably increasing; particles
 * that take the careful path are never skipped).  E and diag are exactly those of the
 * full evaluation; only the work changes.  Not set in the headline measurement. */
#define LW_CULL (1 << 9)

/* trajectory source */
#define LW_TRAJ_SAMPLES 0 /* stored samples r, beta, beta_dot                  */
#define LW_TRAJ_BORIS 1   /* FP64 Boris push from init + laser (lw_trajectory_boris) */

/* Laser pulse driving the electrons (the paper's "sinusoidal plane wave";
 * the pulse shape is this library's reading): propagation along -z,
 * x-polarised, normalised vector potential a_x = a0 g(phi) sin(phi) with
 * phi = (2 pi c/lambda)(t + z/c), g = cos^2(phi/(2 n_cycles)) for
 * |phi| < pi n_cycles (else 0), times exp(-(x^2+y^2)/w0^2) when w0 > 0.
 * E_x = -E0 d(a_x/a0)/dphi, B_y = -E_x/c, E0 = a0 m_e c (2 pi c/lambda)/e. */
typedef struct {
    double a0;
    double lambda;   /* m                            */
    double w0;       /* m; <= 0 means plane wave     */
    double n_cycles; /* number of optical periods    */
} lw_laser_t;

/* Particle trajectories.  Samples i = 0..n_samples-1 are taken at
 * t_i = t_start + i*dt (computed, never accumulated). */
typedef struct {
    int32_t kind;          /* LW_TRAJ_SAMPLES or LW_TRAJ_BORIS                          */
    int32_t span;          /* 0, or >= 2: samples per pushed span of an LW_TRAJ_BORIS     */
                           /* deposit or its adjoint (0: chosen from the workspace);     */
                           /* 0 elsewhere                                                */
    int64_t n_particles;   /* >= 0                                                       */
    int64_t n_samples;     /* >= 1  (= N_s + 1 in the paper's notation)                  */
    double t_start, dt;    /* s; dt > 0                                                  */
    const double *r;        /* [n_particles][n_samples][3] m       (SAMPLES)               */
    const double *beta;     /* [n_particles][n_samples][3]         (SAMPLES)               */
    const double *beta_dot; /* [n_particles][n_samples][3] 1/s     (SAMPLES)               */
    const double *init;     /* [n_particles][6] x,y,z (m), u = gamma*beta (BORIS)          */
    lw_laser_t laser;       /* (BORIS)                                                     */
    const double *charge;   /* [n_particles] C per macroparticle, or NULL for -e each      */
} lw_traj_t;

/* Detector pixels and their uniform observer grid. */
typedef struct {
    int64_t n_pix;        /* >= 0                                          */
    const double *x_det;  /* [n_pix][3] m, |x_m| > 0                       */
    double t0;            /* s, relative to |x_m|/c                        */
    double dt_obs;        /* s, > 0                                        */
    int64_t n_obs;        /* 1 <= n_obs < 2^31; power of two >= 4 for FFTs */
} lw_grid_t;

/* which-argument of lw_workspace_bytes */
#define LW_WS_DEPOSIT 1
#define LW_WS_FFT 2
#define LW_WS_DIRECT_FD 3
#define LW_WS_DEPOSIT_BWD 4
#define LW_WS_FFT_BWD 5
#define LW_WS_DIRECT_FD_BWD 6
#define LW_WS_DEPOSIT_BORIS 7
#define LW_WS_DEPOSIT_BWD_BORIS 8
#define LW_WS_DEPOSIT_DET_ACC 9

/*
 * Workspace (scratch device memory) that the call `which` needs, in bytes:
 * n_a = n_particles (deposit, deposit_bwd, deposit_boris, deposit_bwd_boris), n_pix
 * (fft, fft_bwd, direct_fd, direct_fd_bwd); n_b = n_samples (deposit*), n_obs
 * (fft, fft_bwd), n_omega (direct_fd, direct_fd_bwd).  LW_WS_DEPOSIT_BORIS sizes
 * the pushed batches and spans of LW_TRAJ_BORIS deposits (~16 GiB at most by
 * default: min(n_particles, 65536) particles over the longest spans that fit);
 * any workspace that holds a two-sample span of one particle is accepted and
 * sets batch and span.  LW_WS_DEPOSIT_BWD_BORIS does the same for the adjoint
 * (min(n_particles, 28086) particles, seven tangents each).
 * LW_WS_DEPOSIT_DET_ACC (n_a = n_pix, n_b = n_obs) is the accumulator buffer of
 * lw_deposit_td_det: 8 bytes per trace element and 8 per trace row.  Returns 0 for
 * an unknown `which`.  Larger workspaces are accepted; for the FFT a larger
 * workspace lets more pixels be transformed per pass.
 */
size_t lw_workspace_bytes(int which, int64_t n_a, int64_t n_b, int prec);

/*
 * lw_deposit_td -- the time-domain method's hot loop (Algorithm 2 with the
 * piecewise-linear interpolation of Sec. "Interpolation"), for every
 * (particle k, sample i, pixel m):
 *   arrival time  tau = (t_i + shift(x_m, r_i) - t0) / dt_obs   in grid units
 *        exact:    shift = (|x_m - r_i| - |x_m|)/c                (Eq. advanced_condition)
 *        far field: shift = -(x_m/|x_m|) . r_i / c                 (Eq. far_adv)
 *   field         E = q/(4 pi eps0) [F_vel (1-b^2)(n-b)/(kappa^3 R^2)
 *                                    + F_acc n x ((n-b) x bd)/(c kappa^3 R)]
 *                 kappa = 1 - n.b  (Eqs. lw_fields_retarded, far_efield)
 *   deposit       for every grid point u with tau_{i-1} < u <= tau_i, 0 <= u < n_obs:
 *                 E_tot[m][.][u] += (1-w) E_{i-1} + w E_i,  w = (u - tau_{i-1})/(tau_i - tau_{i-1})
 * Readings: sample 0 primes the one-step buffer (nothing is deposited before
 * tau_0); an interval with tau_i <= tau_{i-1} is skipped; an interval touching a
 * sample with a non-finite value or |beta| >= 1 is skipped.
 *
 * traj:       LW_TRAJ_SAMPLES, or LW_TRAJ_BORIS: the samples are then recomputed
 *             inside the call by the FP64 Boris pusher of lw_trajectory_boris, a
 *             batch of particles over a span of samples at a time into the workspace
 *             (never the whole set), each span deposited and discarded.  Spans share
 *             their boundary sample and the pusher's state carries over between
 *             them, so the samples equal those of lw_trajectory_boris bit for bit
 *             and n_samples is not limited by memory.  Batch and span follow from
 *             ws_bytes (traj->span = 0), or traj->span >= 2 fixes the span; ws then
 *             needs lw_workspace_bytes(LW_WS_DEPOSIT_BORIS, n_particles, n_samples,
 *             prec) bytes, or less (smaller batches and spans).
 * grid:       pixels and observer grid.
 * prec:       LW_PREC_FP64 (E is double) or LW_PREC_MIXED (E is float; tau and
 *             the crossing decisions are still computed in double).  In the exact
 *             geometry, a particle with max_i |r_i|^2 <= 1e-8 |x_m|^2 over its whole
 *             trajectory (for LW_TRAJ_BORIS the max over every pushed sample, found
 *             by a first pass of the pusher) has its path correction expanded in
 *             |r|/|x_m|: to third order in FP64 mode (exact to rounding), to first
 *             order in MIXED mode (relative error of the correction <= 1.25e-8);
 *             where every pixel of a 128-pixel tile is at the first pixel's
 *             distance, the series is evaluated as a polynomial in the pixel
 *             variable, leaving out its highest terms where their bound over the
 *             particle and the tile is at most 1e-12 (FP64) or 1e-7 (MIXED) grid
 *             units; other particles use the square-root form.  The arrival base
 *             (t_i - t0 - z_i/c)/dt_obs is summed in double-double and rounded once.
 * field_mask: LW_FIELD_ACCEL and/or LW_FIELD_VELOCITY (non-zero).
 * geom:       LW_GEOM_EXACT or LW_GEOM_FARFIELD, optionally | LW_ACCUMULATE, | LW_CULL.
 * E:          [n_pix][3][n_obs] float or double, overwritten (or accumulated).
 * diag:       NULL or int64[4]: {skipped non-monotone intervals, skipped
 *             intervals touching an unusable sample, grid points of deposited
 *             intervals outside [0, n_obs), deposited grid points}; overwritten
 *             (or accumulated).
 * ws:         a pixel table (2 MiB: 16384 pixels; larger grids are deposited in
 *             passes of 16384 pixels), 16 B per particle and per-sample records of
 *             the arrival time (arrival base, position and, in the exact geometry,
 *             its coefficients in the pixel variable: 64 B per sample with MIXED,
 *             80 B with FP64).  lw_workspace_bytes(LW_WS_DEPOSIT, n_particles,
 *             n_samples, prec) holds every particle's records; any workspace that
 *             holds one particle's (lw_workspace_bytes(LW_WS_DEPOSIT, 1, n_samples,
 *             prec)) is accepted, and the particles are then deposited in as many
 *             launches as needed.
 * Contributions are summed with device atomics: results are reproducible to
 * rounding, not bit-for-bit, across runs (lw_deposit_td_det is).
 */
lw_status lw_deposit_td(const lw_traj_t *traj, const lw_grid_t *grid, int prec, int field_mask, int geom, void *E,
                        int64_t *diag, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * lw_deposit_td_det -- the deposit of lw_deposit_td (same Algorithm 2 with the
 * interpolation of Sec. "Interpolation"), FP64, with a result that does not depend on
 * the order in which the contributions reach a trace element: the same inputs give the
 * same E bit for bit on every run, and so does any permutation of the particles.
 * Two deposits compute the same contributions v: the first keeps max |v| per element
 * (an order-free maximum), which sets a power-of-two scale s per trace row (pixel and
 * component) with |v| s < 2^62; the second adds round(v s) to a 128-bit fixed-point
 * integer per element, whose sum no ordering changes; each sum is then converted and
 * divided by s (within one ulp).  The rounding of a contribution is at most 2^-62 of its row's largest
 * contribution, so the result agrees with lw_deposit_td's FP64 sum to rounding.  About
 * twice the time of the FP64 call.  A row that receives a non-finite contribution is
 * NaN throughout.
 *
 * traj, grid, field_mask, diag, ws, ws_bytes: as for lw_deposit_td with LW_PREC_FP64
 *             (LW_TRAJ_BORIS pushes the trajectories twice).
 * geom:       LW_GEOM_EXACT or LW_GEOM_FARFIELD; LW_ACCUMULATE and LW_CULL are
 *             refused (LW_E_ARG).
 * E:          [n_pix][3][n_obs] double, overwritten.
 * acc:        device buffer of acc_bytes >= lw_workspace_bytes(LW_WS_DEPOSIT_DET_ACC,
 *             n_pix, n_obs, LW_PREC_FP64), 256-byte aligned, owned by the caller; its
 *             contents on entry are ignored (LW_E_WORKSPACE if smaller or NULL,
 *             LW_E_ALIGN if misaligned).
 */
lw_status lw_deposit_td_det(const lw_traj_t *traj, const lw_grid_t *grid, int field_mask, int geom, double *E,
                            int64_t *diag, void *acc, size_t acc_bytes, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * lw_spectrum_fft -- |E(w)|^2 of every pixel's trace on the FFT bins
 * (Eq. efield_xfrom with the rectangle rule on the observer grid):
 *   S[m][j] = (dt_obs^2 / (2 pi)) sum_c | sum_u E[m][c][u] exp(-2 pi i j u / n_obs) |^2,
 *   j = 0..n_obs/2, w_j = 2 pi j / (n_obs dt_obs).
 * (The paper's +j sign and the phase of the grid origin only conjugate or
 * rotate each term; |.|^2 is unchanged.)  The spectral-angular intensity is
 * (2/(c mu0)) |x_m|^2 S (the relation before Eq. efield_xfrom).
 * E: [n_pix][3][n_obs], S: [n_pix][n_obs/2 + 1], both float (MIXED) or double
 * (FP64).  n_obs must be a power of two, 4 <= n_obs <= 2^22.
 * ws: >= lw_workspace_bytes(LW_WS_FFT, n_pix, n_obs, prec) bytes (minimum: one
 * pixel pair per pass).
 */
lw_status lw_spectrum_fft(const void *E, int64_t n_pix, int64_t n_obs, double dt_obs, int prec, void *S, void *ws,
                          size_t ws_bytes, hipStream_t stream);

/*
 * lw_spectrum_fft_noalloc -- lw_spectrum_fft for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same transform and outputs, with the library's own static scratch
 * array (lw_noalloc_scratch_bytes() = 64 MiB per GPU, held from library load until the
 * process ends) in place of the workspace.  It calls no allocating routine.  E, S, n_pix,
 * n_obs, dt_obs, prec as for lw_spectrum_fft; E and S are caller-owned device memory.
 * One pixel pair's intermediate, 3 n_obs complex values (24 n_obs bytes in MIXED, 48 n_obs
 * in FP64), must fit the scratch: n_obs <= 2^21 (MIXED) or 2^20 (FP64); larger n_obs
 * return LW_E_WORKSPACE.  Pixels are transformed in batches of as many pairs as fit.
 * Every call on one GPU shares that GPU's scratch: calls that may overlap on one GPU
 * (different streams or host threads without ordering between them) race and give
 * undefined results; calls ordered on one stream are safe.  The scratch needs no
 * clearing (each batch writes it fully before reading it).
 */
lw_status lw_spectrum_fft_noalloc(const void *E, int64_t n_pix, int64_t n_obs, double dt_obs, int prec, void *S,
                                  hipStream_t stream);
size_t lw_noalloc_scratch_bytes(void);

/*
 * lw_direct_fd -- the frequency-domain method (Eq. inty_dft, Algorithm 1)
 * generalised to the exact geometry and the velocity term:
 *   F_c(w) = (dt/sqrt(2 pi)) sum_k sum_{i=0}^{n_samples-1} E_{k,i,c} kappa_{k,i}
 *            exp(+j w (t_i + shift_{k,i} - t0)),   S[m][w] = sum_c |F_c(w)|^2
 * with E, kappa, shift as in lw_deposit_td (kappa = dt_a/dt).  Unusable
 * samples are skipped.  In the far field with the acceleration term only,
 * 2 eps0 c |x_m|^2 S is the right-hand side of Eq. inty_dft.
 * grid: x_det and t0 are used (dt_obs, n_obs ignored).  omega: [n_omega]
 * rad/s (device).  prec: FP64 = all double; MIXED = phase in double reduced
 * to one revolution, sin/cos and the sums' terms in float, sums in double;
 * where each block of 512 consecutive frequencies is equally spaced (to 1e-13
 * relative), the phasors of 8 consecutive frequencies come from one float
 * sin/cos pair and a recurrence over frequency (any other frequencies: one
 * sin/cos pair per phasor).
 * S: [n_pix][n_omega] double.
 * ws: >= lw_workspace_bytes(LW_WS_DIRECT_FD, n_pix, n_omega, prec) bytes.
 */
lw_status lw_direct_fd(const lw_traj_t *traj, const lw_grid_t *grid, const double *omega, int64_t n_omega, int prec,
                       int field_mask, int geom, double *S, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * lw_trajectory_boris -- FP64 Boris trajectories of electrons (q = -e, m_e)
 * in the laser pulse of traj->laser (the paper integrates the equations of
 * motion with the Boris method; leap-frog form):
 *   u_{1/2}   = Boris kick of u_0 over dt/2 with the fields at (r_0, t_0)
 *   r_{i+1}   = r_i + c u_{i+1/2}/gamma_{i+1/2} dt
 *   u_{i+3/2} = Boris kick of u_{i+1/2} over dt with the fields at (r_{i+1}, t_{i+1})
 * Samples: beta_0 from u_0, beta_i from (u_{i-1/2} + u_{i+1/2})/2 for i >= 1,
 * beta_dot_i = q/(gamma_i m c) [E + c beta_i x B - beta_i (beta_i.E)] at (r_i, t_i).
 * traj: kind LW_TRAJ_BORIS with init, laser, n_particles, n_samples, t_start, dt.
 * r, beta, beta_dot: outputs [n_particles][n_samples][3] double.
 */
lw_status lw_trajectory_boris(const lw_traj_t *traj, double *r, double *beta, double *beta_dot, hipStream_t stream);

/*
 * lw_trajectory_boris_bwd -- gradient of a scalar J through lw_trajectory_boris
 * (chains the sample gradients of lw_deposit_td_bwd to the beam's initial phase
 * space and to the laser amplitude a0).  Given g_r = dJ/dr, g_beta = dJ/dbeta,
 * g_beta_dot = dJ/dbeta_dot [n_particles][n_samples][3] (double), writes
 *   grad_init[k][c] = dJ/d init[k][c]        [n_particles][6]   (overwritten)
 *   grad_a0[k]      = the part of dJ/d a0 carried by particle k   [n_particles]
 *                     (dJ/d a0 = sum_k grad_a0[k]; overwritten)
 * The pusher is the one of lw_trajectory_boris, recomputed in FP64 with forward-mode
 * tangents, one per particle and parameter (each trajectory depends only on its own
 * initial condition and on a0).  traj: kind LW_TRAJ_BORIS, as for
 * lw_trajectory_boris.  All arrays device memory, 8-byte aligned, non-NULL when
 * n_particles > 0.
 */
lw_status lw_trajectory_boris_bwd(const lw_traj_t *traj, const double *g_r, const double *g_beta,
                                  const double *g_beta_dot, double *grad_init, double *grad_a0, hipStream_t stream);

/*
 * lw_spectrum_fft_bwd -- adjoint of lw_spectrum_fft: given dJ/dS (same layout
 * as S) and the trace E the forward pass used, writes
 *   dE[m][c][u] = dJ/dE[m][c][u] = (dt_obs^2/2pi) sum_j dS[m][j] * 2 Re( conj(F_c[j]) dF_c[j]/dE[c][u] ).
 * E, dS, dE follow the precision of `prec`.
 * ws: >= lw_workspace_bytes(LW_WS_FFT_BWD, n_pix, n_obs, prec) bytes.
 */
lw_status lw_spectrum_fft_bwd(const void *E, const void *dS, int64_t n_pix, int64_t n_obs, double dt_obs, int prec,
                              void *dE, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * lw_deposit_td_bwd -- adjoint of lw_deposit_td with respect to the
 * trajectory samples: given dE = dJ/dE_tot, accumulates (adds into)
 * d_r, d_beta, d_beta_dot [n_particles][n_samples][3] (double) the gradient
 * of J through the interpolation weights, the arrival times and the field
 * formula.  Each sample gathers from the grid points of the (at most two)
 * intervals that touch it; no atomics on the trace.  The derivative of the
 * weights is taken piecewise (the trace is not differentiable where a grid
 * point coincides with an arrival time).  prec: FP64 only in this version
 * (MIXED returns LW_E_UNSUPPORTED).  traj: kind LW_TRAJ_SAMPLES.  dE: double
 * [n_pix][3][n_obs].  ws: >= lw_workspace_bytes(LW_WS_DEPOSIT_BWD, n_particles,
 * n_samples, prec) bytes (each particle's max |r_i|^2).  Arrival times take the
 * forward FP64 deposit's forms: for pixels at the distance of pixel 0 and
 * particles with max_i |r_i|^2 <= 1e-8 |x_m|^2 the polynomial in the pixel term
 * b of the deposit's records (the same coefficients), else from the compensated
 * arrival base with the third-order series of the path correction in that range
 * (exact to rounding) or the square-root form.
 */
lw_status lw_deposit_td_bwd(const lw_traj_t *traj, const lw_grid_t *grid, int prec, int field_mask, int geom,
                            const void *dE, double *d_r, double *d_beta, double *d_beta_dot, void *ws,
                            size_t ws_bytes, hipStream_t stream);

/*
 * lw_deposit_td_bwd_boris -- adjoint of lw_deposit_td for LW_TRAJ_BORIS
 * trajectories with respect to the initial conditions and the laser amplitude:
 * given dE = dJ/dE_tot (double [n_pix][3][n_obs]), writes
 *   grad_init[k][c] = dJ/d init[k][c]   [n_particles][6]  (overwritten)
 *   grad_a0[k]      = particle k's part of dJ/d a0 [n_particles] (overwritten)
 * For a batch of particles over a span of samples at a time (spans as in
 * lw_deposit_td: shared boundary samples, pusher and tangent states carried
 * over; traj->span = 0 lets the workspace choose, >= 2 fixes it) it recomputes
 * the samples, runs the sample adjoint (lw_deposit_td_bwd) over the span's
 * intervals into the workspace and contracts it with the pusher's tangents
 * (lw_trajectory_boris_bwd) over the span.  prec: FP64 only.
 * ws: >= lw_workspace_bytes(LW_WS_DEPOSIT_BWD_BORIS, n_particles, n_samples, prec)
 * bytes, or any size that holds a two-sample span of one particle.
 */
lw_status lw_deposit_td_bwd_boris(const lw_traj_t *traj, const lw_grid_t *grid, int prec, int field_mask, int geom,
                                  const void *dE, double *grad_init, double *grad_a0, void *ws, size_t ws_bytes,
                                  hipStream_t stream);

/*
 * lw_direct_fd_bwd -- adjoint of lw_direct_fd with respect to the trajectory
 * samples.  With dS = dJ/dS [n_pix][n_omega] (double), F_c(w) = sum E_c kappa e^{i w t}
 * the forward sums (recomputed here in FP64 into ws) and t = t_i + shift - t0:
 *   dJ/d(E_c kappa) = 2f sum_w dS (Re F_c cos wt + Im F_c sin wt),
 *   dJ/dt           = 2f sum_w dS w sum_c E_c kappa (Im F_c cos wt - Re F_c sin wt),
 * f = dt^2/2pi, chained through the field formula, kappa = 1 - n.beta and the arrival
 * time (dt/dr = -n/c).  Adds (accumulates) into d_r, d_beta, d_beta_dot
 * [n_particles][n_samples][3] (double); each sample is written by one thread, no
 * atomics.  prec: LW_PREC_FP64 only (MIXED returns LW_E_UNSUPPORTED).  Unusable
 * samples get no gradient.  ws: >= lw_workspace_bytes(LW_WS_DIRECT_FD_BWD, n_pix,
 * n_omega, prec) bytes, 256-byte aligned.
 */
lw_status lw_direct_fd_bwd(const lw_traj_t *traj, const lw_grid_t *grid, const double *omega, int64_t n_omega,
                           int prec, int field_mask, int geom, const double *dS, double *d_r, double *d_beta,
                           double *d_beta_dot, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Kernel timing (a measurement aid; off by default).  lw_timing_enable(1) makes
 * every later launch of the kernel named by `which` record a pair of HIP events
 * on the launch's stream around it; lw_timing_enable(0) stops and discards what
 * was recorded.  lw_timing_read waits for the recorded events (host
 * synchronisation on them), writes the summed elapsed time in milliseconds and
 * the number of launches, and clears them.  which: LW_KERNEL_DEPOSIT (the
 * fast-path evaluate-and-deposit kernel of lw_deposit_td, once per launch: per
 * call, per particle chunk of a small workspace, or per pushed span for
 * LW_TRAJ_BORIS), LW_KERNEL_DEPOSIT_BWD (the sample-gradient kernel of
 * lw_deposit_td_bwd and of each span of lw_deposit_td_bwd_boris),
 * LW_KERNEL_BORIS_TANGENT (the pusher's tangent kernel of each span of
 * lw_deposit_td_bwd_boris).  The events are owned by the library (created
 * on first use, reused).  Returns LW_E_ARG for an unknown `which` or NULL
 * outputs, LW_E_HIP if an event call fails.  Not meant for concurrent use from
 * several host threads.
 */
#define LW_KERNEL_DEPOSIT 1
#define LW_KERNEL_DEPOSIT_BWD 2
#define LW_KERNEL_BORIS_TANGENT 3
lw_status lw_timing_enable(int on);
lw_status lw_timing_read(int which, double *total_ms, int64_t *launches);

/* Thread-local text of the last error ("" if none). */
const char *lw_last_error(void);

/* Library version string. */
const char *lw_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LW_H */
