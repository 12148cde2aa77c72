"""Pins of the oracle's Algorithm-2 interpolation step (Sec. "Interpolation",
Algorithm 2) against exact properties of piecewise-linear interpolation."""
import numpy as np
import pytest

import oracle
from paper_2206_03015_amd import inputs


def covered(tau, n_obs):
    """Grid points u in (tau_0, tau_last] within [0, n_obs)."""
    lo = int(np.floor(tau[0])) + 1
    hi = int(np.floor(tau[-1]))
    return np.arange(max(lo, 0), min(hi, n_obs - 1) + 1)


def test_two_sample_hand_case():
    # tau = 0.25 -> 2.5, E_x = 1 -> 5: u=1: w=0.75/2.25=1/3 -> 7/3; u=2: w=1.75/2.25=7/9 -> 37/9
    out, diag = oracle.interp_deposit([0.25, 2.5], [[1, 0, 0], [5, 0, 0]], 4)
    assert out[0].tolist() == pytest.approx([0.0, 7.0 / 3.0, 37.0 / 9.0, 0.0], abs=1e-15)
    assert np.all(out[1:] == 0)
    assert diag.tolist() == [0, 0, 0, 2]


def test_partition_of_unity():
    """Constant field on every sample -> exactly that constant on every covered grid point."""
    rng = np.random.default_rng(0)
    for trial in range(10):
        n = 200
        tau = np.cumsum(rng.uniform(0.01, 1.7, n)) - 30.0
        E0 = rng.normal(size=3)
        E = np.tile(E0, (n, 1))
        n_obs = 150
        out, diag = oracle.interp_deposit(tau, E, n_obs)
        cov = covered(tau, n_obs)
        ref = np.zeros((3, n_obs))
        ref[:, cov] = E0[:, None]
        assert np.max(np.abs(out - ref)) <= 4e-16 * np.max(np.abs(E0))
        assert diag[3] == cov.size
        total = int(np.floor(tau[-1]) - np.floor(tau[0]))
        assert diag[2] == total - cov.size
        assert diag[0] == 0 and diag[1] == 0


def test_linear_field_is_reproduced():
    """E linear in the arrival time -> grid values equal the line at the grid point."""
    rng = np.random.default_rng(1)
    n = 300
    tau = np.cumsum(rng.uniform(0.05, 2.5, n)) - 10.0
    a = rng.normal(size=3)
    b = rng.normal(size=3)
    E = a[None, :] + b[None, :] * tau[:, None]
    n_obs = 400
    out, _ = oracle.interp_deposit(tau, E, n_obs)
    cov = covered(tau, n_obs)
    ref = a[:, None] + b[:, None] * cov[None, :]
    scale = np.max(np.abs(ref))
    assert np.max(np.abs(out[:, cov] - ref)) <= 1e-13 * scale
    mask = np.ones(n_obs, bool)
    mask[cov] = False
    assert np.all(out[:, mask] == 0)


def test_nonmonotone_and_unusable_are_skipped():
    # (0,2] deposits u=1,2 ; (2,1] skipped (non-monotone) ; (1,3] deposits u=2 (w=.5), u=3 (w=1)
    E = [[1, 0, 0], [3, 0, 0], [10, 0, 0], [20, 0, 0]]
    out, diag = oracle.interp_deposit([0.0, 2.0, 1.0, 3.0], E, 5)
    assert out[0].tolist() == pytest.approx([0.0, 2.0, 3.0 + 15.0, 20.0, 0.0])
    assert diag.tolist() == [1, 0, 0, 4]
    # a NaN sample removes both intervals that touch it
    out, diag = oracle.interp_deposit([0.0, np.nan, 2.0, 3.0], E, 5)
    assert out[0].tolist() == pytest.approx([0.0, 0.0, 0.0, 20.0, 0.0])
    assert diag.tolist() == [0, 2, 0, 1]


def test_tie_goes_to_the_closing_sample():
    """Half-open intervals: a grid point equal to tau_i takes weight 1 on E_i, once."""
    out, diag = oracle.interp_deposit([0.5, 1.0, 1.5], [[1, 0, 0], [2, 0, 0], [4, 0, 0]], 3)
    assert out[0].tolist() == [0.0, 2.0, 0.0]
    assert diag[3] == 1


def test_static_charge_deposit_is_coulomb_plateau():
    """Full deposit of a charge at rest (velocity field): every sample has the same Coulomb
    field, so the trace is that field on every covered grid point and zero elsewhere."""
    n_s, n_obs = 301, 128
    r = np.zeros((1, n_s, 3)) + np.array([1e-6, -2e-6, 3e-6])
    b = np.zeros_like(r)
    x = inputs.pixel_positions(3, 0.01)
    dt = 1e-18
    dt_obs = 3.3e-18
    # grid origin a little after the first arrival at the central pixel (arrival shift ~ -n.r/c)
    t0 = (np.linalg.norm(x[4] - r[0, 0]) - np.linalg.norm(x[4])) / oracle.C_LIGHT + 20e-18
    out, diag = oracle.deposit_td(0.0, dt, r, b, b, x, t0, dt_obs, n_obs, field_mask=oracle.FIELD_VELOCITY)
    for m in range(x.shape[0]):
        d = x[m] - r[0, 0]
        Eref = -oracle.Q_E / (4 * np.pi * oracle.EPS0) * d / np.linalg.norm(d) ** 3
        D = np.linalg.norm(x[m])
        tau = (np.arange(n_s) * dt + (np.linalg.norm(d) - D) / oracle.C_LIGHT - t0) / dt_obs
        cov = covered(tau, n_obs)
        assert cov.size > 10
        assert np.max(np.abs(out[m][:, cov] - Eref[:, None])) <= 1e-14 * np.max(np.abs(Eref))
        mask = np.ones(n_obs, bool)
        mask[cov] = False
        assert np.all(out[m][:, mask] == 0)


def test_deposit_counts_match_arrival_span():
    """Hit count of the full deposit = number of grid points in (tau_0, tau_last] per
    (particle, pixel), using arrival times from the evaluation step."""
    r, b, bd = inputs.random_trajectory(3, 400, seed=4, dt=2e-18)
    x = inputs.pixel_positions(2, 0.02)
    t0, dt_obs, n_obs = -50e-18, 0.4e-18, 700
    out, diag = oracle.deposit_td(0.0, 2e-18, r, b, bd, x, t0, dt_obs, n_obs)
    tau, _, _ = oracle.eval_samples(0.0, 2e-18, r, b, bd, x, t0, dt_obs)
    hits = sum(covered(tau[m, k], n_obs).size for m in range(4) for k in range(3))
    span = sum(int(np.floor(tau[m, k, -1]) - np.floor(tau[m, k, 0])) for m in range(4) for k in range(3))
    assert diag[3] == hits
    assert diag[2] == span - hits
    assert diag[0] == 0 and diag[1] == 0
