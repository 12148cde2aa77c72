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
