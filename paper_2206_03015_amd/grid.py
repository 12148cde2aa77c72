"""Host-side set-up helpers of the time-domain method (Sec. "Time-Domain Method",
Sec. "Parallelization" and Sec. "Performance").

These are the paper's estimates for the observer grid and its cost models.
They run on the host in FP64 and feed diagnostics; the observer grid actually
used by a workload is chosen in ``inputs.py``.
"""
from __future__ import annotations

import math

import numpy as np

C_LIGHT = 299792458.0


def t_u_min(t_start, x_det, r_start):
    """Eq. tu_min: earliest far-field arrival time over particles and observers,
    t_start + |x_m|/c - n_m . x_k(t_start)/c.  x_det [n_pix][3], r_start [n_p][3]."""
    x_det = np.asarray(x_det, dtype=np.float64).reshape(-1, 3)
    r_start = np.asarray(r_start, dtype=np.float64).reshape(-1, 3)
    D = np.linalg.norm(x_det, axis=1)
    n = x_det / D[:, None]
    ta = t_start + D[:, None] / C_LIGHT - (n @ r_start.T) / C_LIGHT
    return float(ta.min())


def t_rad(t_laser, gamma):
    """Eq. Tu_second: single-particle radiation duration T_laser / (2 gamma^2)."""
    return t_laser / (2.0 * gamma * gamma)


def t_bunch(l_bx, l_by, l_bz, gamma, c=C_LIGHT):
    """Eq. Tu_first: bound on the spread of arrival times over the bunch,
    l_bx/(gamma c) + l_by/(gamma c) + l_bz/c."""
    return l_bx / (gamma * c) + l_by / (gamma * c) + l_bz / c


def t_u_estimate(l_bx, l_by, l_bz, t_laser, gamma, c=C_LIGHT):
    """Eq. time:Tu_estimation: T_u = T_bunch + T_rad."""
    return t_bunch(l_bx, l_by, l_bz, gamma, c) + t_rad(t_laser, gamma)


def bunch_extent(r):
    """Size of a particle set in each direction (max - min), the l_b of Eq. Tu_first."""
    r = np.asarray(r, dtype=np.float64).reshape(-1, 3)
    return tuple(float(v) for v in (r.max(axis=0) - r.min(axis=0)))


def n_tu_estimate(l_bx, l_by, l_bz, t_laser, gamma, lam0, c=C_LIGHT):
    """Eqs. NTu_estimation_1..3 combined: N_Tu = 2 w_max / dw with w_max = 4 gamma^2 w0 and
    dw = 2 pi / T_u, i.e. 8 gamma^2 (l_bx/(gamma lam0) + l_by/(gamma lam0) + l_bz/lam0
    + c T_laser/(2 gamma^2 lam0))."""
    return 8.0 * gamma * gamma * (l_bx / (gamma * lam0) + l_by / (gamma * lam0) + l_bz / lam0
                                  + c * t_laser / (2.0 * gamma * gamma * lam0))


def memory_ratio_phi(P, n_p, n_obs, n_tu):
    """Eq. time:parallel_scheme_function: M_beam / M_detector."""
    m_beam = 12.0 * n_p / P + n_obs * (4.0 * n_p / P + 3.0 * n_tu)
    m_det = 12.0 * n_p + n_obs / P * (4.0 * n_p + 3.0 * n_tu)
    return m_beam / m_det


def fd_break_even_log_exponent(c_omega, c2_t, n_s, n_p):
    """Exponent of the criterion that follows Eq. performance_model_ratio with N_Tu = 2 N_w:
    the frequency-domain method wins only if N_w > 0.5 exp(X), X = 0.5 (C_w/C2_t) N_s N_p.
    Returns X."""
    return 0.5 * (c_omega / c2_t) * n_s * n_p


def wallclock_ratio(c1_t, c2_t, c_omega, n_s, n_p, n_tu, n_omega, log=math.log):
    """Eq. performance_model_ratio: (W1_t + W2_t) / W_w."""
    return (c1_t * n_s * n_p + c2_t * n_tu * log(n_tu)) / (c_omega * n_s * n_p * n_omega)


def arrival_far(t, r, x_det, t0, dt_obs, c=C_LIGHT):
    """Far-field arrival times of the samples r [n_p][3] emitted at time t (scalar), in grid units of
    each pixel's observer grid: tau = (t - n_m . r/c - t0)/dt_obs, i.e. the t_a^{k,m}(t) below
    Eq. tu_min with |x_m|/c taken out (the grid of pixel m starts at |x_m|/c + t0).  [n_pix][n_p]."""
    x_det = np.asarray(x_det, dtype=np.float64).reshape(-1, 3)
    r = np.asarray(r, dtype=np.float64).reshape(-1, 3)
    n = x_det / np.linalg.norm(x_det, axis=1)[:, None]
    return ((t - t0) - (n @ r.T) / c) / dt_obs


def _hull_points(r):
    """Vertices of the convex hull of the points r [n][3] (all points when there are few or they
    are degenerate)."""
    if r.shape[0] <= 64:
        return r
    try:
        from scipy.spatial import ConvexHull
        return r[ConvexHull(r).vertices]
    except Exception:  # degenerate (coplanar, collinear) sets: every point
        return r


def window_diagnostics(t_start, t_end, r_first, r_last, x_det, t0, dt_obs, n_obs, gamma, lam0, n_sampled=64,
                       chunk=1024):
    """Observer-window diagnostics of a workload (Sec. "Time-Domain Method", the bounds of the
    uniform time grid), from the first and last samples of every particle (r_first, r_last
    [n_p][3] at t_start and t_end) and the pixels x_det [n_pix][3]:

    * t_u_min, t_u_max: Eqs. tu_min, tu_max over all particles and pixels (far-field arrival
      times, measured from |x_m|/c), and their distance T_u_trajectories;
    * T_rad, T_bunch, T_u_estimate: Eqs. Tu_second, Tu_first, time:Tu_estimation with the bunch
      extent l_b of the first samples and T_laser = t_end - t_start;
    * N_Tu_estimate: Eqs. NTu_estimation_1..3 combined;
    * the observer window actually used (t0, n_obs dt_obs), t_u_min in its grid units, and the
      fraction of (particle, pixel) pairs whose arrival interval [tau_first, tau_last] holds a
      window grid point (pairs_captured, over n_sampled evenly spaced pixels) and the fraction of
      particles captured by at least one of those pixels (particles_captured)."""
    x_det = np.asarray(x_det, dtype=np.float64).reshape(-1, 3)
    r_first = np.asarray(r_first, dtype=np.float64).reshape(-1, 3)
    r_last = np.asarray(r_last, dtype=np.float64).reshape(-1, 3)
    # the extremes over particles of a linear function of the position are taken at vertices of
    # the particles' convex hull, so only those enter the min/max over every pixel
    hf, hl = _hull_points(r_first), _hull_points(r_last)
    lo, hi = np.inf, -np.inf
    for m0 in range(0, x_det.shape[0], chunk):
        xs = x_det[m0:m0 + chunk]
        lo = min(lo, float(arrival_far(t_start, hf, xs, 0.0, 1.0).min()))
        hi = max(hi, float(arrival_far(t_end, hl, xs, 0.0, 1.0).max()))
    lbx, lby, lbz = bunch_extent(r_first)
    t_laser = t_end - t_start
    sel = np.unique(np.linspace(0, x_det.shape[0] - 1, min(n_sampled, x_det.shape[0])).round().astype(int))
    tf = arrival_far(t_start, r_first, x_det[sel], t0, dt_obs)
    tl = arrival_far(t_end, r_last, x_det[sel], t0, dt_obs)
    # a window grid point u (0 <= u < n_obs) lies in (tau_first, tau_last]
    first_u = np.maximum(np.floor(tf) + 1.0, 0.0)
    cap = (first_u <= np.minimum(np.floor(tl), n_obs - 1.0))
    return {
        "t_u_min_s": lo, "t_u_max_s": hi, "T_u_trajectories_s": hi - lo,
        "T_rad_s": t_rad(t_laser, gamma), "T_bunch_s": t_bunch(lbx, lby, lbz, gamma),
        "T_u_estimate_s": t_u_estimate(lbx, lby, lbz, t_laser, gamma),
        "N_Tu_estimate": n_tu_estimate(lbx, lby, lbz, t_laser, gamma, lam0),
        "window_t0_s": t0, "window_s": n_obs * dt_obs, "n_obs": int(n_obs),
        "t_u_min_grid": (lo - t0) / dt_obs,
        "pairs_captured": float(cap.mean()) if cap.size else 0.0,
        "particles_captured": float(cap.any(axis=0).mean()) if cap.size else 0.0,
        "pixels_sampled": int(sel.size),
    }
