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
