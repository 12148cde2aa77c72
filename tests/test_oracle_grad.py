"""Pins of the oracle gradients: the spectrum adjoint against the exact central difference of
the quadratic spectrum, and the complex-step chain against the real C oracle (value) and its
central finite differences (derivative)."""
import numpy as np
import pytest

import oracle
from oracle import gradient as og
from cases import FD_REL_TOL, PARAM_FD, smooth_directions, synthetic


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
    vr, vb, va = smooth_directions(c, rng)
    z = 0.0 * vr
    for name, v in (("r", (vr, z, z)), ("beta", (z, vb, z)), ("beta_dot", (z, z, va))):
        d_cs, J0 = og.directional_derivative(c["t_start"], c["dt"], c["r"], c["beta"], c["beta_dot"], *v,
                                             c["x_det"], c["t0"], c["dt_obs"], c["n_obs"], weights=W,
                                             charge=c["charge"], field_mask=3, geom=geom)
        h = 1e-6
        Jp = J_real(c, c["r"] + h * v[0], c["beta"] + h * v[1], c["beta_dot"] + h * v[2], W, geom)
        Jm = J_real(c, c["r"] - h * v[0], c["beta"] - h * v[1], c["beta_dot"] - h * v[2], W, geom)
        fd = (Jp - Jm) / (2 * h)
        assert d_cs == pytest.approx(fd, rel=FD_REL_TOL[name], abs=0), name


# ---- the pusher's tangents and the (gamma_mean, a0) chain ----------------------------------------

def boris_case():
    from cases import small_bunch
    return small_bunch(n_p=6, n_steps=1500, n_side=3, n_obs=1 << 11)


def test_boris_complex_value_matches_c_oracle():
    c = boris_case()
    W, L = c["W"], c["W"].laser
    r, b, bd = og.boris_complex(c["init"], W.n_samples, W.t_start, W.dt, L.a0, L.lam, L.w0, L.n_cycles)
    assert np.max(np.abs(r - c["r"])) <= 1e-14 * np.max(np.abs(c["r"]))
    assert np.max(np.abs(b - c["beta"])) <= 1e-14
    assert np.max(np.abs(bd - c["beta_dot"])) <= 1e-11 * np.max(np.abs(c["beta_dot"]))


def test_boris_complex_step_matches_central_differences():
    """G = sum g.(r, beta, beta_dot) with random g: its complex-step derivative along a random
    initial-condition direction and along a0 equals the central difference of the C pusher
    (step 1e-4 relative: the difference converges quadratically, ~2e-7 there, before round-off
    takes over below 1e-5)."""
    c = boris_case()
    W, L = c["W"], c["W"].laser
    rng = np.random.default_rng(17)
    g = [rng.normal(size=c["r"].shape) / np.maximum(np.std(x), 1e-300) for x in (c["r"], c["beta"], c["beta_dot"])]

    def G(parts):
        return sum(np.sum(gi * pi) for gi, pi in zip(g, parts))

    scale = np.array([1e-6, 1e-6, 1e-6, 0.1, 0.1, 1.0])  # metres and u = gamma beta
    v = rng.normal(size=c["init"].shape) * scale
    for which in ("init", "a0"):
        h = 1e-30
        if which == "init":
            z = og.boris_complex(c["init"] + 1j * h * v, W.n_samples, W.t_start, W.dt, L.a0, L.lam, L.w0, L.n_cycles)
            eps = 1e-4
            p = oracle.boris(c["init"] + eps * v, W.n_samples, W.t_start, W.dt, L.a0, L.lam, L.w0, L.n_cycles)
            m = oracle.boris(c["init"] - eps * v, W.n_samples, W.t_start, W.dt, L.a0, L.lam, L.w0, L.n_cycles)
        else:
            z = og.boris_complex(c["init"], W.n_samples, W.t_start, W.dt, L.a0 + 1j * h, L.lam, L.w0, L.n_cycles)
            eps = 1e-4 * L.a0
            p = oracle.boris(c["init"], W.n_samples, W.t_start, W.dt, L.a0 + eps, L.lam, L.w0, L.n_cycles)
            m = oracle.boris(c["init"], W.n_samples, W.t_start, W.dt, L.a0 - eps, L.lam, L.w0, L.n_cycles)
        d_cs = G([x.imag for x in z]) / h
        fd = (G(p) - G(m)) / (2 * eps)
        assert d_cs == pytest.approx(fd, rel=2e-6, abs=0), which


def test_boris_tangent_free_flight_closed_form():
    """With the laser off (a0 = 0) u stays constant and r_i = r_0 + c (u/gamma) i dt, so
    dr_i/du = c i dt (I/gamma - u u^T/gamma^3) and dbeta_i/du = I/gamma - u u^T/gamma^3."""
    rng = np.random.default_rng(4)
    n_p, ns, dt = 3, 50, 1e-16
    init = np.concatenate([rng.normal(size=(n_p, 3)) * 1e-6, rng.normal(size=(n_p, 3)) * [0.1, 0.1, 1.0]], axis=1)
    init[:, 5] += 30.0
    h = 1e-30
    for j in range(3):
        e = np.zeros_like(init)
        e[:, 3 + j] = 1.0
        r, b, bd = og.boris_complex(init + 1j * h * e, ns, 0.0, dt, 0.0, 1e-6, 0.0, 20.0)
        u = init[:, 3:]
        gam = np.sqrt(1.0 + np.sum(u * u, axis=1))
        J = np.eye(3)[None] / gam[:, None, None] - u[:, :, None] * u[:, None, :] / gam[:, None, None] ** 3
        col = J[:, :, j]
        i = np.arange(ns)
        want_r = oracle.C_LIGHT * dt * i[None, :, None] * col[:, None, :]
        assert np.max(np.abs(r.imag / h - want_r)) <= 1e-12 * np.max(np.abs(want_r))
        assert np.max(np.abs(b.imag / h - col[:, None, :])) <= 1e-13 * np.max(np.abs(col))
        assert np.max(np.abs(bd.imag)) == 0.0
    # positions: dr_i/dx_0 = I
    e = np.zeros_like(init)
    e[:, 1] = 1.0
    r, _, _ = og.boris_complex(init + 1j * h * e, ns, 0.0, dt, 0.0, 1e-6, 0.0, 20.0)
    assert np.all(r.imag[:, :, 1] / h == 1.0) and np.all(r.imag[:, :, [0, 2]] == 0.0)


def params_case():
    from paper_2206_03015_amd import inputs
    c = boris_case()
    W = c["W"]
    full_w = inputs.workload("bunch")
    full = inputs.bunch_init(full_w)
    zc = np.sqrt(1.0 - 1.0 / W.gamma ** 2) * inputs.C_LIGHT * W.t_start
    rows = np.argsort(np.abs(full[:, 2] - zc))[: c["init"].shape[0]]
    assert np.array_equal(full[rows], c["init"])
    rng = np.random.default_rng(21)
    Wt = np.zeros((c["x_det"].shape[0], c["n_obs"] // 2 + 1))
    Wt[:, 20:200] = rng.random((Wt.shape[0], 180))
    return c, (lambda g: inputs.bunch_init(full_w, gamma=g)[rows]), Wt




@pytest.mark.parametrize("which", ["gamma", "a0"])
def test_params_derivative_matches_central_differences(which):
    """dJ/dgamma_mean and dJ/da0 by complex step through draw, pusher, deposit and spectrum, against
    the central difference of the real C oracle chain."""
    c, init_of, Wt = params_case()
    W, L = c["W"], c["W"].laser
    d_cs, J0 = og.params_derivative(init_of, W.gamma, L.a0, (L.lam, L.w0, L.n_cycles), W.n_samples, W.t_start, W.dt,
                                    c["x_det"], c["t0"], c["dt_obs"], c["n_obs"], Wt, which)

    def J(gamma, a0):
        r, b, bd = oracle.boris(init_of(gamma), W.n_samples, W.t_start, W.dt, a0, L.lam, L.w0, L.n_cycles)
        E, _ = oracle.deposit_td(W.t_start, W.dt, r, b, bd, c["x_det"], c["t0"], c["dt_obs"], c["n_obs"])
        return np.sum(Wt * oracle.spectrum(E, c["dt_obs"]))

    x0 = W.gamma if which == "gamma" else L.a0
    rel_step, tol = PARAM_FD[which]
    eps = rel_step * x0
    if which == "gamma":
        fd = (J(x0 + eps, L.a0) - J(x0 - eps, L.a0)) / (2 * eps)
    else:
        fd = (J(W.gamma, x0 + eps) - J(W.gamma, x0 - eps)) / (2 * eps)
    assert J0 == pytest.approx(J(W.gamma, L.a0), rel=1e-10, abs=0)
    assert abs(d_cs * x0 / J0) > 0.1  # the objective really depends on the parameter
    assert d_cs == pytest.approx(fd, rel=tol, abs=0)


# ---- the direct frequency-domain sum in complex arithmetic -------------------------------------

def fd_case(seed=2):
    c = small_case(seed=seed, n_pix=4)
    tau, _, _ = oracle.eval_samples(c["t_start"], c["dt"], c["r"], c["beta"], c["beta_dot"], c["x_det"][:1], 0.0, 1.0)
    w1 = 2 * np.pi / (np.ptp(tau) / 30)  # ~30 periods over the arrival-time span
    return c, np.linspace(0.2, 2.0, 37) * w1


@pytest.mark.parametrize("geom", [0, 1])
def test_direct_fd_complex_matches_c_oracle_and_differences(geom):
    """Value equals orc_direct_fd; the complex-step derivative equals its central differences
    (the FD sum is smooth in the samples: step 1e-4 along smooth directions)."""
    c, omega = fd_case()
    args = (c["t_start"], c["dt"])
    So = oracle.direct_fd(*args, c["r"], c["beta"], c["beta_dot"], c["x_det"], c["t0"], omega, charge=c["charge"],
                          field_mask=3, geom=geom)
    Sc = og.direct_fd_complex(*args, c["r"], c["beta"], c["beta_dot"], c["x_det"], c["t0"], omega,
                              charge=c["charge"], field_mask=3, geom=geom)
    assert np.max(np.abs(Sc.imag)) == 0.0
    assert np.max(np.abs(Sc.real - So)) <= 1e-12 * np.max(So)
    rng = np.random.default_rng(1)
    dS = rng.random(So.shape)
    vr, vb, va = smooth_directions(c, rng)
    z = 0.0 * vr
    for name, v in (("r", (vr, z, z)), ("beta", (z, vb, z)), ("beta_dot", (z, z, va))):
        d, J = og.fd_directional_derivative(*args, c["r"], c["beta"], c["beta_dot"], *v, c["x_det"], c["t0"], omega,
                                            dS, charge=c["charge"], field_mask=3, geom=geom)
        h = 1e-4
        Jp = np.sum(dS * oracle.direct_fd(*args, c["r"] + h * v[0], c["beta"] + h * v[1], c["beta_dot"] + h * v[2],
                                          c["x_det"], c["t0"], omega, charge=c["charge"], field_mask=3, geom=geom))
        Jm = np.sum(dS * oracle.direct_fd(*args, c["r"] - h * v[0], c["beta"] - h * v[1], c["beta_dot"] - h * v[2],
                                          c["x_det"], c["t0"], omega, charge=c["charge"], field_mask=3, geom=geom))
        assert d == pytest.approx((Jp - Jm) / (2 * h), rel=1e-6, abs=0), name
