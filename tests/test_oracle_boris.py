"""Pins of the oracle trajectory sources: the analytic plane-wave motion and the
FP64 Boris pusher (the integrator the paper names in Sec. "Time-Domain Method")."""
import numpy as np
import pytest

import oracle
from oracle import trajectory as tj

C = oracle.C_LIGHT
QE, ME = oracle.Q_E, oracle.M_E


def lorentz_beta_dot(beta, E, B):
    """d beta/dt for an electron from the Lorentz force (textbook, independent of the oracle C)."""
    g = 1.0 / np.sqrt(1.0 - np.sum(beta * beta, axis=-1, keepdims=True))
    q = -QE
    return q / (g * ME * C) * (E + C * np.cross(beta, B) - beta * np.sum(beta * E, axis=-1, keepdims=True))


def c0_setup(n_samples=4001, a0=0.1, gamma=50.0, n_cycles=20.0):
    lam = 1e-6
    T = 1.05 * n_cycles * lam / (2 * C)
    return dict(gamma0=gamma, a0=a0, lam=lam, n_cycles=n_cycles, n_samples=n_samples, t_start=-T / 2,
                dt=T / (n_samples - 1))


def test_analytic_trajectory_solves_equations_of_motion():
    """r' = c beta and beta' = Lorentz force, checked with centred differences."""
    p = c0_setup(n_samples=20001, a0=0.5, gamma=5.0, n_cycles=4.0)
    r, b, bd, info = oracle.planewave_trajectory(**p)
    dt = p["dt"]
    r, b, bd = r[0], b[0], bd[0]
    vdiff = (r[2:] - r[:-2]) / (2 * dt)
    assert np.max(np.abs(vdiff - C * b[1:-1])) <= 1e-6 * C * np.max(np.abs(b[:, 0])) + 1e-9 * C
    bdiff = (b[2:] - b[:-2]) / (2 * dt)
    scale = np.max(np.abs(bd))
    assert np.max(np.abs(bdiff - bd[1:-1])) <= 1e-5 * scale
    t = info["t"]
    E, B = oracle.laser_fields(r, t, p["a0"], p["lam"], 0.0, p["n_cycles"])
    assert np.max(np.abs(lorentz_beta_dot(b, E, B) - bd)) <= 1e-9 * scale


def test_analytic_trajectory_conserved_quantities():
    p = c0_setup(a0=1.0, gamma=20.0, n_cycles=6.0)
    r, b, bd, info = oracle.planewave_trajectory(**p)
    g = 1.0 / np.sqrt(1.0 - np.sum(b[0] ** 2, axis=-1))
    u = g[:, None] * b[0]
    h = info["h"]
    assert np.max(np.abs((g + u[:, 2]) / h - 1.0)) < 1e-12
    assert np.max(np.abs(u[:, 0] - p["a0"] * tj.S_of(info["phi"], p["n_cycles"]))) < 1e-12
    # phase consistency phi = w (t + z/c)
    wl = info["omega_L"]
    assert np.max(np.abs(wl * (info["t"] + r[0, :, 2] / C) - info["phi"])) < 1e-9 * np.max(np.abs(info["phi"]))


def test_field_free_boris_is_a_straight_line():
    rng = np.random.default_rng(2)
    init = np.zeros((4, 6))
    init[:, :3] = 1e-6 * rng.normal(size=(4, 3))
    init[:, 3:] = rng.normal(size=(4, 3)) * [0.01, 0.01, 40.0]
    n, dt = 500, 3e-18
    r, b, bd = oracle.boris(init, n, -1e-15, dt, 0.0, 1e-6, 0.0, 20.0)
    g = np.sqrt(1 + np.sum(init[:, 3:] ** 2, axis=1))
    beta = init[:, 3:] / g[:, None]
    t = np.arange(n) * dt
    ref = init[:, None, :3] + C * beta[:, None, :] * t[None, :, None]
    assert np.max(np.abs(r - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert np.max(np.abs(b - beta[:, None, :])) <= 1e-15
    assert np.all(bd == 0)


def _boris_vs_analytic(n_samples):
    p = c0_setup(n_samples=n_samples, a0=0.5, gamma=10.0, n_cycles=6.0)
    r, b, bd, info = oracle.planewave_trajectory(**p)
    u0 = b[0, 0] / np.sqrt(1 - np.sum(b[0, 0] ** 2))
    init = np.concatenate([r[0, 0], u0])[None]
    rb, bb, bdb = oracle.boris(init, n_samples, p["t_start"], p["dt"], p["a0"], p["lam"], 0.0, p["n_cycles"])
    ex = np.max(np.abs(rb[0, :, 0] - r[0, :, 0])) / np.max(np.abs(r[0, :, 0]))
    eb = np.max(np.abs(bdb[0] - bd[0])) / np.max(np.abs(bd[0]))
    return ex, eb


def test_boris_converges_to_analytic_at_second_order():
    e1 = _boris_vs_analytic(2001)
    e2 = _boris_vs_analytic(4001)
    e3 = _boris_vs_analytic(8001)
    for a, b in ((e1, e2), (e2, e3)):
        for x, y in zip(a, b):
            assert 3.3 < x / y < 4.7
    assert e3[0] < 1e-4 and e3[1] < 1e-3
