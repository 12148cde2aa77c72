"""Analytic trajectory of an electron in a plane-wave pulse (test infrastructure).

The paper drives its particles with a sinusoidal plane wave and integrates the
motion with the Boris method.  For a plane wave that depends on
phi = w_L (t + z/c) only (propagation along -z) the motion is known in closed
form, which gives an independent check of the Boris pusher and exact inputs
for the single-electron configuration.

Pulse (same reading as the C oracle's laser): normalised vector potential
    a_x(phi) = a0 S(phi),  S = g(phi) sin(phi),  g = cos^2(phi / (2 n)) for |phi| < n pi, else 0,
with n the number of cycles.  For an electron (charge -e) that is at rest
transversally before the pulse:
  * canonical transverse momentum:  u_x = a0 S(phi)          (u = gamma beta)
  * light-front momentum:           h = gamma + u_z = const
  * hence gamma = (h^2 + 1 + u_x^2)/(2h),  u_z = (h^2 - 1 - u_x^2)/(2h),
    d phi/dt = w_L h / gamma,
  * and, with the electron at the origin when phi = 0 (t = 0):
        t(phi) = [(h^2 + 1) phi + a0^2 I2(phi)] / (2 w_L h^2)
        z(phi) = c [(h^2 - 1) phi - a0^2 I2(phi)] / (2 w_L h^2)
        x(phi) = c a0 I1(phi) / (w_L h)
    where I1 = int_0^phi S, I2 = int_0^phi S^2 (closed forms below).
Samples at t_i = t_start + i dt solve t(phi) = t_i by Newton's method.
"""
from __future__ import annotations

import numpy as np

C_LIGHT = 299792458.0


def _terms(n_cycles):
    # g sin(phi) = 1/2 sin(phi) + 1/4 sin((1+1/n) phi) + 1/4 sin((1-1/n) phi)
    A = np.array([0.5, 0.25, 0.25])
    K = np.array([1.0, 1.0 + 1.0 / n_cycles, 1.0 - 1.0 / n_cycles])
    return A, K


def _clip(phi, n_cycles):
    lim = np.pi * n_cycles
    return np.clip(phi, -lim, lim), np.abs(phi) < lim


def S_of(phi, n_cycles):
    A, K = _terms(n_cycles)
    pc, inside = _clip(phi, n_cycles)
    s = sum(A[j] * np.sin(K[j] * pc) for j in range(3))
    return np.where(inside, s, 0.0)


def dS_of(phi, n_cycles):
    A, K = _terms(n_cycles)
    pc, inside = _clip(phi, n_cycles)
    s = sum(A[j] * K[j] * np.cos(K[j] * pc) for j in range(3))
    return np.where(inside, s, 0.0)


def I1_of(phi, n_cycles):
    A, K = _terms(n_cycles)
    pc, _ = _clip(phi, n_cycles)
    return sum(A[j] * (1.0 - np.cos(K[j] * pc)) / K[j] for j in range(3))


def _cint(kap, p):
    # int_0^p cos(kap s) ds
    if kap == 0.0:
        return p
    return np.sin(kap * p) / kap


def I2_of(phi, n_cycles):
    A, K = _terms(n_cycles)
    pc, _ = _clip(phi, n_cycles)
    tot = 0.0
    for j in range(3):
        for l in range(3):
            tot = tot + 0.5 * A[j] * A[l] * (_cint(K[j] - K[l], pc) - _cint(K[j] + K[l], pc))
    return tot


def planewave_trajectory(gamma0, a0, lam, n_cycles, n_samples, t_start, dt):
    """Exact r, beta, beta_dot [1][n_samples][3] at t_i = t_start + i dt, plus
    a dict with h and the phases.  gamma0: Lorentz factor before the pulse,
    electron moving along +z."""
    wl = 2.0 * np.pi * C_LIGHT / lam
    h = gamma0 + np.sqrt(gamma0 * gamma0 - 1.0)
    t = t_start + np.arange(n_samples, dtype=np.float64) * dt

    def t_of(phi):
        return ((h * h + 1.0) * phi + a0 * a0 * I2_of(phi, n_cycles)) / (2.0 * wl * h * h)

    def gam_of(phi):
        ux = a0 * S_of(phi, n_cycles)
        return (h * h + 1.0 + ux * ux) / (2.0 * h)

    phi = 2.0 * wl * h * h * t / (h * h + 1.0)
    for _ in range(60):
        step = (t_of(phi) - t) * wl * h / gam_of(phi)
        phi = phi - step
        if np.all(np.abs(step) <= 4.0 * np.finfo(float).eps * np.maximum(np.abs(phi), 1.0)):
            break
    ux = a0 * S_of(phi, n_cycles)
    uxp = a0 * dS_of(phi, n_cycles)
    gam = (h * h + 1.0 + ux * ux) / (2.0 * h)
    uz = (h * h - 1.0 - ux * ux) / (2.0 * h)
    gp = ux * uxp / h
    uzp = -ux * uxp / h
    x = C_LIGHT * a0 * I1_of(phi, n_cycles) / (wl * h)
    z = C_LIGHT * ((h * h - 1.0) * phi - a0 * a0 * I2_of(phi, n_cycles)) / (2.0 * wl * h * h)
    dphidt = wl * h / gam
    bx = ux / gam
    bz = uz / gam
    bdx = (uxp * gam - ux * gp) / (gam * gam) * dphidt
    bdz = (uzp * gam - uz * gp) / (gam * gam) * dphidt
    zero = np.zeros_like(x)
    r = np.stack([x, zero, z], axis=-1)[None]
    beta = np.stack([bx, zero, bz], axis=-1)[None]
    beta_dot = np.stack([bdx, zero, bdz], axis=-1)[None]
    return r, beta, beta_dot, {"h": h, "phi": phi, "omega_L": wl, "t": t}
