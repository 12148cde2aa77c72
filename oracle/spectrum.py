"""Spectrum of a time-domain trace, for the oracle (test infrastructure only).

Eq. efield_xfrom defines E(x, w) = (2 pi)^-1/2 int E(x, t) exp(+j w t) dt.  On the
uniform observer grid t_u = t_origin + u dt_obs (u = 0..N-1) the rectangle rule
gives, at the FFT bins w_j = 2 pi j / (N dt_obs),

    E_c(w_j) = (dt_obs / sqrt(2 pi)) exp(+j w_j t_origin) sum_u E_c[u] exp(+2 pi j ju/N)

and the returned spectrum is S_j = sum_c |E_c(w_j)|^2 for j = 0..N/2.  The
phase factor and the sign of the exponent (a complex conjugation for real
input) do not change |.|^2, so S_j = (dt_obs^2 / 2 pi) sum_c |rfft(E_c)[j]|^2.
The spectral-angular intensity is (2/(c mu0)) |x|^2 S (the relation quoted
before Eq. efield_xfrom); ``intensity`` applies it.
"""
from __future__ import annotations

import numpy as np

C_LIGHT = 299792458.0
MU0 = 1.25663706212e-6


def spectrum(E_tot, dt_obs):
    """S[..., N/2+1] from a trace E_tot[..., 3, N] (numpy.fft.rfft in FP64)."""
    E_tot = np.asarray(E_tot, dtype=np.float64)
    F = np.fft.rfft(E_tot, axis=-1)
    return (dt_obs * dt_obs / (2.0 * np.pi)) * np.sum(F.real ** 2 + F.imag ** 2, axis=-2)


def spectrum_bruteforce(E_tot, dt_obs):
    """O(N^2) evaluation of the same sums with the +j sign of Eq. efield_xfrom
    (small N only; used to pin ``spectrum``)."""
    E_tot = np.asarray(E_tot, dtype=np.float64)
    N = E_tot.shape[-1]
    j = np.arange(N // 2 + 1)[:, None]
    u = np.arange(N)[None, :]
    ph = 2.0 * np.pi * ((j * u) % N) / N
    C = np.cos(ph)
    Sn = np.sin(ph)
    re = E_tot @ C.T
    im = E_tot @ Sn.T
    return (dt_obs * dt_obs / (2.0 * np.pi)) * np.sum(re ** 2 + im ** 2, axis=-2)


def omega_bins(n_obs, dt_obs):
    """Angular frequencies of the returned bins, w_j = 2 pi j/(N dt_obs)."""
    return 2.0 * np.pi * np.arange(n_obs // 2 + 1) / (n_obs * dt_obs)


def intensity(S, D):
    """d^2 I / dw dOmega = (2/(c mu0)) D^2 S."""
    return 2.0 / (C_LIGHT * MU0) * D * D * np.asarray(S)
