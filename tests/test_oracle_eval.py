"""Pins of the oracle's per-sample evaluation (arrival time, LW field) against
closed forms that do not share its formula.

Eq. lw_fields_retarded gives the acceleration field; the velocity field is the
Coulomb-like term of the textbook LW field that the paper drops; Eq.
advanced_condition gives the arrival time; Eqs. far_efield/far_adv the far-field
approximation.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import oracle

C = oracle.C_LIGHT
K = 1.0 / (4.0 * math.pi * oracle.EPS0)
Q = -oracle.Q_E
ACC, VEL = oracle.FIELD_ACCEL, oracle.FIELD_VELOCITY
EXACT, FAR = oracle.GEOM_EXACT, oracle.GEOM_FARFIELD


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("geom", [EXACT, FAR])
def test_coulomb_at_rest(geom):
    """Charge at rest: E = q (x - r) / (4 pi eps0 |x - r|^3) (exact geometry); the far-field
    mode replaces x - r by x."""
    rng = np.random.default_rng(1)
    for _ in range(20):
        x = rng.normal(size=3)
        x *= 0.7 / np.linalg.norm(x)
        r = 1e-3 * rng.normal(size=3)
        tt, E, kap = oracle.eval_one(x, r, np.zeros(3), np.zeros(3), Q, VEL, geom)
        d = x - r if geom == EXACT else x
        ref = K * Q * d / np.linalg.norm(d) ** 3
        assert rel(E, ref) < 1e-14
        assert kap == 1.0
        # no acceleration -> no radiation field
        _, E2, _ = oracle.eval_one(x, r, np.zeros(3), np.zeros(3), Q, ACC, geom)
        assert np.all(E2 == 0.0)


def heaviside_field(q, x, r_now, beta):
    """Field of a uniformly moving charge in terms of its present position (Heaviside):
    E = q (1 - b^2) R / (4 pi eps0 |R|^3 (1 - b^2 sin^2 psi)^(3/2)), R = x - r_now."""
    R = x - r_now
    b2 = beta @ beta
    cospsi = (R @ beta) / (np.linalg.norm(R) * math.sqrt(b2))
    sin2 = 1.0 - cospsi ** 2
    return K * q * (1.0 - b2) * R / (np.linalg.norm(R) ** 3 * (1.0 - b2 * sin2) ** 1.5)


@pytest.mark.parametrize("gamma", [1.5, 10.0, 200.0])
def test_uniform_motion_matches_heaviside(gamma):
    """Velocity field at the arrival time equals the closed-form field of a charge in
    uniform motion, evaluated at the charge's position at that time."""
    rng = np.random.default_rng(int(gamma))
    bmag = math.sqrt(1.0 - 1.0 / gamma ** 2)
    for _ in range(20):
        d = rng.normal(size=3)
        beta = bmag * d / np.linalg.norm(d)
        x = rng.normal(size=3)
        x *= 0.5 / np.linalg.norm(x)
        r = 1e-2 * rng.normal(size=3)
        t = 0.0
        tt, E, _ = oracle.eval_one(x, r, beta, np.zeros(3), Q, VEL, EXACT)
        ta = t + tt + np.linalg.norm(x) / C  # arrival time at x
        r_now = r + beta * C * (ta - t)
        ref = heaviside_field(Q, x, r_now, beta)
        assert rel(E, ref) < 2e-11 * gamma ** 2


def test_linear_acceleration_closed_form():
    """beta parallel to beta_dot: |E_acc| = |q| |bd| sin(theta) / (4 pi eps0 c R (1 - b cos theta)^3),
    E_acc transverse to n (textbook linear-acceleration radiation field)."""
    rng = np.random.default_rng(7)
    for gamma in (1.2, 5.0, 50.0):
        b = math.sqrt(1.0 - 1.0 / gamma ** 2)
        for _ in range(10):
            e = rng.normal(size=3)
            e /= np.linalg.norm(e)
            beta = b * e
            bd = 3.7e13 * e
            x = rng.normal(size=3)
            x *= 2.0 / np.linalg.norm(x)
            tt, E, _ = oracle.eval_one(x, np.zeros(3), beta, bd, Q, ACC, FAR)
            n = x / np.linalg.norm(x)
            cth = n @ e
            sth = math.sqrt(max(0.0, 1.0 - cth * cth))
            mag = K * abs(Q) * np.linalg.norm(bd) * sth / (C * 2.0 * (1.0 - b * cth) ** 3)
            assert abs(np.linalg.norm(E) - mag) <= 1e-12 * mag + 1e-300
            assert abs(E @ n) <= 1e-12 * np.linalg.norm(E)


def test_circular_acceleration_closed_form():
    """beta perpendicular to beta_dot: |n x ((n - b) x bd)|^2 =
    |bd|^2 [(1 - b cos th)^2 - (1 - b^2) sin^2 th cos^2 ph] (textbook circular-motion result;
    th = angle(n, beta), ph = azimuth of n around beta measured from beta_dot)."""
    rng = np.random.default_rng(11)
    for gamma in (1.1, 3.0, 30.0):
        b = math.sqrt(1.0 - 1.0 / gamma ** 2)
        for _ in range(10):
            e1 = rng.normal(size=3)
            e1 /= np.linalg.norm(e1)
            e2 = rng.normal(size=3)
            e2 -= (e2 @ e1) * e1
            e2 /= np.linalg.norm(e2)
            e3 = np.cross(e1, e2)
            th = rng.uniform(0, math.pi)
            ph = rng.uniform(0, 2 * math.pi)
            n = math.cos(th) * e1 + math.sin(th) * (math.cos(ph) * e2 + math.sin(ph) * e3)
            beta, bd = b * e1, 2.5e14 * e2
            D = 1.3
            tt, E, kap = oracle.eval_one(D * n, np.zeros(3), beta, bd, Q, ACC, FAR)
            k = 1.0 - b * math.cos(th)
            num2 = (2.5e14) ** 2 * (k * k - (1.0 - b * b) * math.sin(th) ** 2 * math.cos(ph) ** 2)
            ref = K * abs(Q) * math.sqrt(num2) / (C * k ** 3 * D)
            assert abs(np.linalg.norm(E) - ref) <= 1e-11 * ref


def test_kappa_against_50_digits():
    """kappa (cancellation-free form) against 1 - n.beta in 50-digit arithmetic on the
    same double inputs; error bounded by the rounding of 1 - |beta|^2."""
    mp.mp.dps = 50
    rng = np.random.default_rng(3)
    for gamma in (2.0, 50.0, 200.0, 1000.0):
        b = math.sqrt(1.0 - 1.0 / gamma ** 2)
        for _ in range(20):
            e = np.array([1e-3 * rng.normal(), 1e-3 * rng.normal(), 1.0])
            e /= np.linalg.norm(e)
            beta = b * e
            x = np.array([rng.uniform(-2, 2) / gamma, rng.uniform(-2, 2) / gamma, 1.0])
            _, _, kap = oracle.eval_one(x, np.zeros(3), beta, np.zeros(3), Q, ACC, FAR)
            D = mp.sqrt(sum(mp.mpf(v) ** 2 for v in x))
            ref = 1 - sum(mp.mpf(x[c]) / D * mp.mpf(beta[c]) for c in range(3))
            assert abs(kap - float(ref)) <= 8.0 * gamma ** 2 * 2.2e-16 * float(ref)


def test_arrival_time_against_50_digits():
    """Exact-geometry arrival shift tt = (|x - r| - |x|)/c, checked in 50-digit arithmetic;
    the far-field shift is -n.r/c."""
    mp.mp.dps = 50
    rng = np.random.default_rng(5)
    for _ in range(50):
        x = np.array([rng.uniform(-0.02, 0.02), rng.uniform(-0.02, 0.02), 1.0])
        r = np.array([3e-6 * rng.normal(), 3e-6 * rng.normal(), 5e-5 * rng.normal()])
        tt, _, _ = oracle.eval_one(x, r, np.zeros(3), np.zeros(3), Q, ACC, EXACT)
        R = mp.sqrt(sum((mp.mpf(x[c]) - mp.mpf(r[c])) ** 2 for c in range(3)))
        D = mp.sqrt(sum(mp.mpf(v) ** 2 for v in x))
        ref = (R - D) / C
        assert abs(tt - float(ref)) <= 1e-15 * abs(float(ref)) + 1e-35
        ttf, _, _ = oracle.eval_one(x, r, np.zeros(3), np.zeros(3), Q, ACC, FAR)
        nref = -sum(mp.mpf(x[c]) / D * mp.mpf(r[c]) for c in range(3)) / C
        assert abs(ttf - float(nref)) <= 1e-15 * abs(float(nref)) + 1e-35


def test_exact_tends_to_far_field():
    """Exact geometry -> far-field approximation as |x| grows: the field difference shrinks
    like |r|/|x| and the arrival-shift difference like |r_perp|^2/(2 c |x|)."""
    rng = np.random.default_rng(9)
    r = np.array([2e-6, -1e-6, 3e-6])
    beta = np.array([0.01, 0.0, 0.999])
    bd = np.array([1e14, 2e13, -1e12])
    n = np.array([0.01, 0.005, 1.0])
    n /= np.linalg.norm(n)
    errs = []
    for D in (1e-2, 1e-1, 1.0, 10.0):
        tte, Ee, _ = oracle.eval_one(D * n, r, beta, bd, Q, ACC, EXACT)
        ttf, Ef, _ = oracle.eval_one(D * n, r, beta, bd, Q, ACC, FAR)
        errs.append(rel(Ee, Ef))
        rp = r - (n @ r) * n
        assert abs((tte - ttf) - (rp @ rp) / (2.0 * C * D)) <= 1e-3 * (rp @ rp) / (2.0 * C * D)
    for a, b in zip(errs, errs[1:]):
        assert 7.0 < a / b < 13.0
    assert rng is not None


@pytest.mark.parametrize("geom", [EXACT, FAR])
def test_arrival_time_in_grid_units_against_50_digits(geom):
    """The arrival time in grid units, tau = (t_i + shift - t0)/dt_obs, at the sizes of the
    largest workloads (gamma 200: t_i up to 1e-13 s, |r| up to 60 um, dt_obs = 1.9 zs, so
    t_i/dt_obs and n.r/(c dt_obs) reach ~5e7 grid units and cancel to the window's size), with
    each sample's window origin t0 placed so that tau lies inside a 2^18-point window, against
    the definition in 50-digit arithmetic on the same double inputs.  A double evaluation loses
    ~1e-8 grid units here; the oracle's extended-precision sum stays within 5e-11: a few
    roundings of the 64-bit significand on terms of ~5e7 grid units (~2e-12 each) plus the final
    double rounding of tau < 2^18 (up to 2.9e-11)."""
    mp.mp.dps = 50
    rng = np.random.default_rng(11)
    n = 200
    t_start, dt, dt_obs = -8.33e-14, 8.33e-18, 1.94e-21
    i = rng.integers(0, 20001, size=n)
    beta = 1.0 - 1.25e-5
    th = rng.uniform(-0.014, 0.014, size=(n, 2))
    x = np.stack([np.sin(th[:, 0]), np.cos(th[:, 0]) * np.sin(th[:, 1]), np.cos(th[:, 0]) * np.cos(th[:, 1])], -1)
    t_i = t_start + i * dt
    z0 = rng.normal(size=n) * 5e-6
    r = np.stack([rng.normal(size=n) * 6e-6, rng.normal(size=n) * 6e-6, z0 + beta * C * t_i], -1)
    worst, worst_double, big = 0.0, 0.0, 0.0
    for j in range(n):
        X = [mp.mpf(v) for v in x[j]]
        Rv = [mp.mpf(v) for v in r[j]]
        D = mp.sqrt(sum(v * v for v in X))
        if geom == EXACT:
            shift = (mp.sqrt(sum((X[c] - Rv[c]) ** 2 for c in range(3))) - D) / C
        else:
            shift = -sum(X[c] / D * Rv[c] for c in range(3)) / C
        ti = mp.mpf(t_start) + int(i[j]) * mp.mpf(dt)
        # a window origin that puts this arrival at a random place of a 2^18-point window
        t0 = float(ti + shift) - rng.uniform(0.0, 2.0 ** 18) * dt_obs
        tau = oracle.arrival_tau(x[j], r[j], [i[j]], t_start, dt, t0, dt_obs, geom)[0]
        ref = (ti + shift - mp.mpf(t0)) / mp.mpf(dt_obs)
        assert 0.0 <= float(ref) < 2.0 ** 18 + 1
        worst = max(worst, abs(float(tau - ref)))
        big = max(big, abs(float(ti / mp.mpf(dt_obs))))
        # the same expression in plain double arithmetic (the oracle's shift, summed in double)
        tt, _, _ = oracle.eval_one(x[j], r[j], np.zeros(3), np.zeros(3), Q, ACC, geom)
        tau_double = ((t_start + float(i[j]) * dt + tt) - t0) / dt_obs
        worst_double = max(worst_double, abs(float(tau_double - ref)))
    print(f"max |tau - tau_50digits| = {worst:.2e} grid units, plain double {worst_double:.2e} "
          f"(largest cancelling term {big:.1e})")
    assert big > 3e7  # the comparison is meaningful: the cancelling terms are this large
    assert worst <= 5e-11
    assert worst_double > 4 * 5e-11  # a double evaluation would not pass
