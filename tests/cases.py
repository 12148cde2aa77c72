"""Shared seeded test cases (inputs only; expected values always come from the oracle)."""
import numpy as np

import oracle
from paper_2206_03015_amd import inputs


def single_electron(n_steps=20000, n_obs=1 << 16, thetas=(0.0,)):
    """The single-electron workload (analytic plane-wave trajectory)."""
    W = inputs.workload("single").scaled(n_steps=n_steps, n_obs=n_obs)
    L = W.laser
    r, b, bd, _ = oracle.planewave_trajectory(W.gamma, L.a0, L.lam, L.n_cycles, W.n_samples, W.t_start, W.dt)
    th = np.asarray(thetas, dtype=float)
    x = np.stack([np.zeros_like(th), np.sin(th), np.cos(th)], axis=-1) * W.D
    return dict(r=r, beta=b, beta_dot=bd, t_start=W.t_start, dt=W.dt, x_det=x, t0=W.t0, dt_obs=W.dt_obs,
                n_obs=W.n_obs, W=W)


def small_bunch(n_p=24, n_steps=3000, n_side=10, n_obs=1 << 12, key="bunch", theta_scale=1.0,
                samples_per_period=None):
    """A bunch workload scaled down so that the oracle runs in seconds: trajectories from the
    oracle's Boris pusher, n_side^2 pixels (several 64-pixel tiles and a ragged tail)."""
    W = inputs.workload(key)
    kw = dict(n_p=n_p, n_steps=n_steps, n_side=n_side, n_obs=n_obs, theta_max=W.theta_max * theta_scale)
    if samples_per_period is not None:
        kw["samples_per_period"] = samples_per_period
    full = inputs.bunch_init(W)  # the workload's full seeded draw
    W = W.scaled(**kw)
    # keep the particles nearest the bunch centre so that the small window catches them
    zc = np.sqrt(1.0 - 1.0 / W.gamma ** 2) * inputs.C_LIGHT * W.t_start  # bunch centre at t_start
    init = np.ascontiguousarray(full[np.argsort(np.abs(full[:, 2] - zc))[:n_p]])
    L = W.laser
    r, b, bd = oracle.boris(init, W.n_samples, W.t_start, W.dt, L.a0, L.lam, L.w0, L.n_cycles)
    x = inputs.pixel_positions(W.n_side, W.theta_max, W.D)
    return dict(r=r, beta=b, beta_dot=bd, t_start=W.t_start, dt=W.dt, x_det=x, t0=W.t0, dt_obs=W.dt_obs,
                n_obs=W.n_obs, W=W, init=init)


def synthetic(n_p=5, n_samples=700, n_pix=70, n_obs=600, seed=0, dt=2e-18):
    """Smooth synthetic trajectories (no laser physics) with a window that cuts through them."""
    r, b, bd = inputs.random_trajectory(n_p, n_samples, seed=seed, dt=dt, spread=2e-10)
    rng = np.random.default_rng(seed)
    th = rng.uniform(-0.03, 0.03, size=(n_pix, 2))
    x = np.stack([np.sin(th[:, 0]), np.cos(th[:, 0]) * np.sin(th[:, 1]), np.cos(th[:, 0]) * np.cos(th[:, 1])], -1)
    tau, _, _ = oracle.eval_samples(0.0, dt, r, b, bd, x[:1], 0.0, 1.0)
    mid = np.median(tau)
    span = np.ptp(tau[0, 0])
    dt_obs = span / (0.7 * n_obs)
    t0 = mid - 0.5 * n_obs * dt_obs
    charge = -1.602176634e-19 * (1.0 + rng.random(n_p))
    return dict(r=r, beta=b, beta_dot=bd, t_start=0.0, dt=dt, x_det=x, t0=t0, dt_obs=dt_obs, n_obs=n_obs,
                charge=charge)


def smooth_directions(c, rng):
    """Perturbation directions (v_r, v_beta, v_beta_dot) for finite-difference checks: per particle
    and component a sinusoid over the samples with a seeded period (1/8 to 1/2 of the run) and
    phase, of amplitude c dt_obs (positions: arrival times move by ~h grid units), max|beta_perp|
    and max|beta_dot|.  Coherent over many samples, so the objective responds far above the
    round-off of the arrival times (random per-sample directions mostly cancel)."""
    n_p, ns, _ = c["r"].shape
    i = np.arange(ns)[None, :, None]
    out = []
    for scale in (oracle.C_LIGHT * c["dt_obs"], np.max(np.abs(c["beta"][..., :2])), np.max(np.abs(c["beta_dot"]))):
        per = ns / (2.0 + 6.0 * rng.random((n_p, 1, 3)))
        ph = 2.0 * np.pi * rng.random((n_p, 1, 3))
        out.append(scale * np.sin(2.0 * np.pi * i / per + ph))
    return tuple(out)


# Central-difference tolerances (relative) at h = 1e-6 along smooth_directions.  The position
# direction is limited by round-off of the arrival times, which are differences of the sample
# time and the path term (~1e-16 of t_i/dt_obs grid units, against h ~ 1e-6 grid units of motion).
FD_REL_TOL = {"r": 2e-4, "beta": 1e-6, "beta_dot": 1e-6}


# (relative step, relative tolerance) of central differences in gamma_mean and a0 through the
# whole chain.  J is piecewise smooth: its slope jumps wherever a grid point crosses an arrival
# time, and a step that moves the arrival times by d grid units crosses ~d of them per
# interval, so the difference converges only linearly in the step until round-off of the
# arrival times takes over (below ~1e-8).  A 1e-7 step in gamma_mean moves arrival times by
# ~1e-4 grid units on the small bunch cut (measured errors 5e-5 to 1e-3 depending on the
# weights); a0 moves them ~20x less.  The exact check of these derivatives is the comparison
# with the oracle's complex step; this one guards against gross errors.
PARAM_FD = {"gamma": (1e-7, 2e-3), "a0": (1e-6, 1e-3)}
