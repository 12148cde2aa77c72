"""Physics pin of the whole oracle chain (trajectory -> deposit -> spectrum) on the
single-electron workload: the inverse-Compton line sits at the Doppler-upshifted
frequency (Introduction, lambda_rad = lambda_L (1 + a0^2/2)/(4 gamma^2)), and off axis
it moves to 4 gamma^2 w_L / (1 + a0^2/2 + gamma^2 theta^2) (standard Doppler kinematics)."""
import numpy as np
import pytest

import oracle
from oracle.spectrum import omega_bins
from paper_2206_03015_amd import inputs


def line_centroid(S, w, w_guess):
    sel = (w > 0.7 * w_guess) & (w < 1.2 * w_guess)
    return float(np.sum(S[sel] * w[sel]) / np.sum(S[sel]))


def test_ics_line_single_electron():
    W = inputs.workload("single")
    L = W.laser
    r, b, bd, info = oracle.planewave_trajectory(W.gamma, L.a0, L.lam, L.n_cycles, W.n_samples, W.t_start, W.dt)
    thetas = np.array([0.0, 0.5 / W.gamma, 1.0 / W.gamma])
    x = np.stack([np.zeros(3), np.sin(thetas) * W.D, np.cos(thetas) * W.D], axis=-1)
    E, diag = oracle.deposit_td(W.t_start, W.dt, r, b, bd, x, W.t0, W.dt_obs, W.n_obs)
    assert diag[0] == 0 and diag[1] == 0
    S = oracle.spectrum(E, W.dt_obs)
    w = omega_bins(W.n_obs, W.dt_obs)
    peaks = []
    for m, th in enumerate(thetas):
        w1 = W.omega1(th)
        wc = line_centroid(S[m], w, w1)
        peaks.append(wc)
        # the line sits within 1 % of the Doppler formula (envelope shifts it by <= a0^2/2)
        assert wc == pytest.approx(w1, rel=1e-2, abs=0)
        jmax = int(np.argmax(S[m][1:])) + 1
        assert w[jmax] == pytest.approx(w1, rel=1.5e-2, abs=0)
    # off-axis scaling 1 / (1 + a0^2/2 + gamma^2 theta^2)
    base = 1 + 0.5 * L.a0 ** 2
    for th, wc in zip(thetas[1:], peaks[1:]):
        assert wc / peaks[0] == pytest.approx(base / (base + (W.gamma * th) ** 2), rel=5e-3)
    # the spectrum is dominated by the line: < 5 % of the energy above 1.5 w1 (higher harmonics
    # are weak at a0 = 0.1)
    for m in range(3):
        w1 = W.omega1(thetas[m])
        assert np.sum(S[m][w > 1.5 * w1]) < 0.05 * np.sum(S[m])
