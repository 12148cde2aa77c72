"""Pins of the host-side grid and cost helpers against values the paper prints."""
import os

import numpy as np
import pytest

from paper_2206_03015_amd import grid

G = os.path.join(os.path.dirname(__file__), "golden")


def rows(name):
    out = []
    for line in open(os.path.join(G, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            out.append(line.split())
    return out


def test_table1_theory_columns():
    c = 0.3  # um/fs
    for lx, ly, lz, T, g, tb, tr, tu in (list(map(float, r)) for r in rows("table1_tu_estimate.txt")):
        assert grid.t_bunch(lx, ly, lz, g, c=c) == pytest.approx(tb, abs=5e-5 + 1e-9)
        assert grid.t_rad(T, g) == pytest.approx(tr, abs=5e-7)
        assert grid.t_u_estimate(lx, ly, lz, T, g, c=c) == pytest.approx(tu, abs=5e-5 + 1e-9)


def test_table2_break_even_ratio():
    for name, E, lz, Q, T, lam, ratio in rows("table2_projects.txt"):
        E, lz, Q, T, lam, ratio = map(float, (E, lz, Q, T, lam, ratio))
        gamma = E / 0.511
        n_p = Q * 1e-12 / 1.602176634e-19
        n_tu = grid.n_tu_estimate(0.0, 0.0, lz * 1e-6, T * 1e-12, gamma, lam * 1e-6, c=3e8)
        assert 4 * n_p / n_tu == pytest.approx(ratio, rel=3e-3, abs=0), name


def test_break_even_exponent():
    (c1, c2, cw, ns, npart, expo), = (list(map(float, r)) for r in rows("break_even_1pC.txt"))
    assert grid.fd_break_even_log_exponent(cw, c2, ns, npart) == pytest.approx(expo, rel=5e-5, abs=0)


def test_memory_ratio_criterion():
    """phi >= 1 exactly when N_obs N_Tu >= 4 N_p (Eq. time:parallel_scheme_function_2)."""
    rng = np.random.default_rng(0)
    for _ in range(200):
        P = int(rng.integers(2, 64))
        n_p, n_obs, n_tu = (float(v) for v in rng.integers(1, 10000, 3))
        phi = grid.memory_ratio_phi(P, n_p, n_obs, n_tu)
        assert (phi >= 1.0) == (n_obs * n_tu >= 4 * n_p)


def test_t_u_min_far_field():
    x = np.array([[0.0, 0.0, 1.0], [0.01, 0.0, 1.0]])
    r = np.array([[0.0, 0.0, 1e-6], [0.0, 0.0, -1e-6]])
    c = grid.C_LIGHT
    expected = min(-1e-15 + np.linalg.norm(xm) / c - (xm / np.linalg.norm(xm)) @ rk / c for xm in x for rk in r)
    assert grid.t_u_min(-1e-15, x, r) == pytest.approx(expected, rel=1e-15, abs=0)


def test_window_diagnostics_against_brute_force():
    """The observer-window diagnostics: t_u_min / t_u_max of Eqs. tu_min, tu_max (taken at the
    convex-hull vertices of the particles) equal the minimum / maximum over every (particle, pixel)
    pair; the captured fractions equal a direct count of window grid points in (tau_first,
    tau_last]; the estimates are those of Eqs. Tu_first, Tu_second, time:Tu_estimation."""
    rng = np.random.default_rng(5)
    c = grid.C_LIGHT
    n_p = 3000
    r0 = rng.normal(size=(n_p, 3)) * np.array([2e-6, 2e-6, 5e-6])
    t_start, t_end = -5e-14, 5e-14
    r1 = r0 + np.array([0.0, 0.0, c * (t_end - t_start) * (1 - 1e-4)])
    th = rng.uniform(-0.02, 0.02, size=(50, 2))
    x = np.stack([np.sin(th[:, 0]), np.cos(th[:, 0]) * np.sin(th[:, 1]), np.cos(th[:, 0]) * np.cos(th[:, 1])], -1)
    dt_obs, n_obs = 1e-18, 1024
    t0 = t_start - 512 * dt_obs
    d = grid.window_diagnostics(t_start, t_end, r0, r1, x, t0, dt_obs, n_obs, 50.0, 1e-6, n_sampled=50)
    n = x / np.linalg.norm(x, axis=1)[:, None]
    ta0 = t_start - (n @ r0.T) / c
    ta1 = t_end - (n @ r1.T) / c
    assert d["t_u_min_s"] == pytest.approx(float(ta0.min()), rel=0, abs=1e-28)
    assert d["t_u_max_s"] == pytest.approx(float(ta1.max()), rel=0, abs=1e-28)
    tf, tl = (ta0 - t0) / dt_obs, (ta1 - t0) / dt_obs
    u = np.arange(n_obs, dtype=float)
    cap = np.zeros(tf.shape, bool)
    for m in range(tf.shape[0]):  # every window grid point against every interval
        cap[m] = np.any((u[:, None] > tf[m][None, :]) & (u[:, None] <= tl[m][None, :]), axis=0)
    assert d["pairs_captured"] == pytest.approx(cap.mean(), abs=1e-12)
    assert d["particles_captured"] == pytest.approx(cap.any(axis=0).mean(), abs=1e-12)
    assert 0 < d["pairs_captured"] < 0.5
    lb = r0.max(axis=0) - r0.min(axis=0)
    assert d["T_u_estimate_s"] == pytest.approx(lb[0] / (50 * c) + lb[1] / (50 * c) + lb[2] / c
                                                + (t_end - t_start) / (2 * 50.0 ** 2), rel=1e-14)
    assert d["t_u_min_grid"] == pytest.approx((d["t_u_min_s"] - t0) / dt_obs, rel=1e-14)
