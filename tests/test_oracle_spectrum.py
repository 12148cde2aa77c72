"""Pins of the oracle spectrum (Eq. efield_xfrom on the FFT bins)."""
import numpy as np
import pytest

import oracle
from oracle.spectrum import omega_bins


@pytest.mark.parametrize("N", [2, 8, 64, 256, 1024])
def test_matches_bruteforce_dft(N):
    rng = np.random.default_rng(N)
    E = rng.normal(size=(2, 3, N))
    S = oracle.spectrum(E, 2.5e-19)
    Sb = oracle.spectrum_bruteforce(E, 2.5e-19)
    assert np.max(np.abs(S - Sb)) <= 1e-12 * np.max(Sb)


@pytest.mark.parametrize("N", [16, 4096])
def test_parseval(N):
    """sum_u,c E^2 dt = dw [S_0 + 2 sum_{0<j<N/2} S_j + S_{N/2}], dw = 2 pi/(N dt)."""
    rng = np.random.default_rng(1)
    dt = 7e-20
    E = rng.normal(size=(3, N))
    S = oracle.spectrum(E, dt)
    dw = 2 * np.pi / (N * dt)
    lhs = np.sum(E * E) * dt
    rhs = dw * (S[0] + 2 * np.sum(S[1:-1]) + S[-1])
    assert abs(lhs - rhs) <= 1e-13 * lhs


def test_single_cosine_is_one_line():
    N, j0, dt = 512, 37, 1e-19
    u = np.arange(N)
    E = np.zeros((3, N))
    E[1] = 2.0 * np.cos(2 * np.pi * j0 * u / N)
    S = oracle.spectrum(E, dt)
    ref = dt * dt / (2 * np.pi) * N * N  # |sum 2 cos e^{...}| = N at the bin
    assert S[j0] == pytest.approx(ref, rel=1e-13, abs=0)
    S[j0] = 0
    assert np.max(S) <= 1e-20 * ref
    w = omega_bins(N, dt)
    assert w[j0] == pytest.approx(2 * np.pi * j0 / (N * dt))
