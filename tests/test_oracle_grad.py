"""Pins of the oracle gradients: the spectrum adjoint against the exact central difference of
the quadratic spectrum, and the complex-step chain against the real C oracle (value) and its
central finite differences (derivative)."""
import numpy as np
import pytest

import oracle
from oracle import gradient as og
from cases import synthetic


@pytest.mark.parametrize("N", [8, 64, 1024])
def test_spectrum_vjp_exact_on_quadratic(N):
    """S is quadratic in E, so (S(E + d) - S(E - d))/2 is its exact linearisation along d."""
    rng = np.random.default_rng(N)
    E = rng.normal(size=(2, 3, N))
    d = rng.normal(size=(2, 3, N))
    dS = rng.normal(size=(2, N // 2 + 1))
    dt = 3e-20
    lin = (oracle.spectrum(E + d, dt) - oracle.spectrum(E - d, dt)) / 2.0
    lhs = np.sum(dS * lin)
    rhs = np.sum(og.spectrum_vjp(E, dS, dt) * d)
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(dS * lin))


def small_case(seed=0, n_p=3, n_samples=300, n_pix=5, n_obs=256):
    return synthetic(n_p=n_p, n_samples=n_samples, n_pix=n_pix, n_obs=n_obs, seed=seed)


@pytest.mark.parametrize("geom", [0, 1])
def test_complex_chain_value_matches_c_oracle(geom):
    c = small_case()
    E_c = og.deposit_complex(c["t_start"], c["dt"], c["r"], c["beta"], c["beta_dot"], c["x_det"], c["t0"],
                             c["dt_obs"], c["n_obs"], charge=c["charge"], field_mask=3, geom=geom)
    E_o, _ = oracle.deposit_td(c["t_start"], c["dt"], c["r"], c["beta"], c["beta_dot"], c["x_det"], c["t0"],
                               c["dt_obs"], c["n_obs"], charge=c["charge"], field_mask=3, geom=geom)
    assert np.max(np.abs(E_c.imag)) == 0.0
    assert np.max(np.abs(E_c.real - E_o)) <= 1e-10 * np.max(np.abs(E_o))
    S_c = og.spectrum_complex(E_c, c["dt_obs"]).real
    assert np.max(np.abs(S_c - oracle.spectrum(E_o, c["dt_obs"]))) <= 1e-9 * np.max(S_c)


def J_real(c, r, b, a, W, geom):
    E, _ = oracle.deposit_td(c["t_start"], c["dt"], r, b, a, c["x_det"], c["t0"], c["dt_obs"], c["n_obs"],
                             charge=c["charge"], field_mask=3, geom=geom)
    return np.sum(W * oracle.spectrum(E, c["dt_obs"]))


@pytest.mark.parametrize("geom", [0, 1])
def test_complex_step_matches_central_differences(geom):
    c = small_case(seed=2)
    rng = np.random.default_rng(5)
    W = rng.random((c["x_det"].shape[0], c["n_obs"] // 2 + 1))
    # one direction per input family; r scaled by c dt_obs so that h = 1e-6 moves arrival
    # times by ~1e-6 grid units (a central difference must not straddle a grid crossing)
    vr = rng.normal(size=c["r"].shape) * oracle.C_LIGHT * c["dt_obs"]
    vb = rng.normal(size=c["beta"].shape) * 1e-6
    va = rng.normal(size=c["beta_dot"].shape) * np.max(np.abs(c["beta_dot"]))
    for v in ((vr, 0 * vb, 0 * va), (0 * vr, vb, 0 * va), (0 * vr, 0 * vb, va)):
        d_cs, J0 = og.directional_derivative(c["t_start"], c["dt"], c["r"], c["beta"], c["beta_dot"], *v,
                                             c["x_det"], c["t0"], c["dt_obs"], c["n_obs"], weights=W,
                                             charge=c["charge"], field_mask=3, geom=geom)
        h = 1e-6
        Jp = J_real(c, c["r"] + h * v[0], c["beta"] + h * v[1], c["beta_dot"] + h * v[2], W, geom)
        Jm = J_real(c, c["r"] - h * v[0], c["beta"] - h * v[1], c["beta_dot"] - h * v[2], W, geom)
        fd = (Jp - Jm) / (2 * h)
        assert d_cs == pytest.approx(fd, rel=1e-5)
