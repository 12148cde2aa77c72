"""Pins of the oracle direct frequency-domain sum (Eq. inty_dft, Algorithm 1)."""
import math

import numpy as np
import pytest

import oracle
from oracle.spectrum import intensity, omega_bins

C = oracle.C_LIGHT


def test_single_sample_is_flat():
    """One sample: S(w) = (dt^2/2 pi) |E kappa|^2 for every w."""
    r = np.array([[[1e-7, 0, 2e-7]]])
    b = np.array([[[0.01, 0.0, 0.99]]])
    bd = np.array([[[3e14, 1e13, 0.0]]])
    x = np.array([[0.001, 0.002, 1.0]])
    w = np.linspace(1e17, 1e19, 7)
    S = oracle.direct_fd(0.0, 2e-18, r, b, bd, x, 0.0, w)
    tt, E, kap = oracle.eval_one(x[0], r[0, 0], b[0, 0], bd[0, 0])
    ref = (2e-18) ** 2 / (2 * math.pi) * np.sum((E * kap) ** 2)
    assert np.allclose(S, ref, rtol=1e-14, atol=0)


def test_far_field_matches_paper_prefactor():
    """Far field, acceleration term: the spectral-angular intensity of the oracle's direct sum,
    ``intensity(S, D)`` = (2/(c mu0)) D^2 S(w), equals the right-hand side of Eq. inty_dft,
    q^2 dt^2/(16 pi^3 eps0 c) |sum_k sum_i A_k(i dt) exp(j w (i dt - n.x_k/c))|^2, with
    A_k = n x ((n - beta) x beta_dot) / (1 - n.beta)^2 (Eq. const_phase_drop).  (1/(c mu0) = eps0 c
    to the 1e-10 of the CODATA values of mu0 and eps0.)"""
    rng = np.random.default_rng(3)
    n_p, n_s = 2, 50
    dt = 1e-18
    b = np.zeros((n_p, n_s, 3))
    b[..., 2] = 0.995
    b[..., 0] = 0.05 * np.sin(np.linspace(0, 3, n_s))[None]
    bd = rng.normal(size=(n_p, n_s, 3)) * 1e15
    r = np.cumsum(b * C * dt, axis=1)
    D = 1.0
    x = np.array([[0.003, -0.001, 1.0]])
    x = D * x / np.linalg.norm(x)
    n = x[0] / D
    w = np.linspace(2e17, 4e18, 11)
    S = oracle.direct_fd(0.0, dt, r, b, bd, x, 0.0, w, geom=oracle.GEOM_FARFIELD)
    q = -oracle.Q_E
    eps0 = oracle.EPS0
    acc = np.zeros((len(w), 3), complex)
    for k in range(n_p):
        for i in range(n_s):
            nb = n - b[k, i]
            A = np.cross(n, np.cross(nb, bd[k, i])) / (1 - n @ b[k, i]) ** 2
            acc += A[None, :] * np.exp(1j * w[:, None] * (i * dt - n @ r[k, i] / C))
    rhs = q * q * dt * dt / (16 * math.pi ** 3 * eps0 * C) * np.sum(np.abs(acc) ** 2, axis=1)
    lhs = intensity(S[0], D)
    assert np.allclose(lhs, rhs, rtol=1e-9, atol=0)
    # the helper scales linearly in S and quadratically in D
    assert np.allclose(intensity(S[0], 2 * D), 4 * lhs, rtol=1e-15, atol=0)


def _td_fd_error(n_samples, n_obs):
    """Single electron (analytic plane-wave trajectory, gamma 5, 4 cycles): relative max
    difference between the deposit+FFT spectrum and the direct sum at the FFT bins."""
    lam, n_cycles, gamma, a0 = 1e-6, 4.0, 5.0, 0.3
    T = 1.05 * n_cycles * lam / (2 * C)
    dt = T / (n_samples - 1)
    r, b, bd, _ = oracle.planewave_trajectory(gamma, a0, lam, n_cycles, n_samples, -T / 2, dt)
    x = np.array([[0.0, 0.02, 1.0]])
    x /= np.linalg.norm(x)
    Trad = T / (2 * gamma ** 2) * 1.6
    win = 4.0 * Trad
    dt_obs = win / n_obs
    t0 = -win / 2
    E, diag = oracle.deposit_td(-T / 2, dt, r, b, bd, x, t0, dt_obs, n_obs)
    assert diag[2] == 0  # window covers the whole pulse
    S_td = oracle.spectrum(E, dt_obs)[0]
    w = omega_bins(n_obs, dt_obs)
    sel = slice(1, n_obs // 8)
    S_fd = oracle.direct_fd(-T / 2, dt, r, b, bd, x, t0, w[sel])[0]
    return np.max(np.abs(S_td[sel] - S_fd)) / np.max(S_fd)


def test_time_and_frequency_domain_converge_at_second_order():
    """Both paths discretise the same integral (Eq. far_bunch_inty); halving the emission
    step and the observer step together cuts the difference by about 4."""
    e = [_td_fd_error(ns, no) for ns, no in ((1001, 1024), (2001, 2048), (4001, 4096))]
    assert e[-1] < 5e-3
    for a, b in zip(e, e[1:]):
        assert 3.0 < a / b < 5.0
