"""GPU adjoints (lw_spectrum_fft_bwd, lw_deposit_td_bwd, lw_trajectory_boris_bwd) and the autograd
chain against the oracle: the spectrum adjoint against its plain formula, the trajectory and
(gamma_mean, a0) gradients against complex-step derivatives of the FP64 oracle chain, and
against central differences of the GPU forward."""
import numpy as np
import pytest
import torch

import oracle
from oracle import gradient as og
from cases import FD_REL_TOL, PARAM_FD, small_bunch, smooth_directions, synthetic

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
GEOMS = {"exact": 0, "farfield": 1}


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), device=DEV)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("n_obs", [4, 64, 1024, 1 << 14])
@pytest.mark.parametrize("n_pix", [1, 2, 3])
def test_spectrum_bwd_matches_formula(prec, n_obs, n_pix):
    from paper_2206_03015_amd import lw
    rng = np.random.default_rng(n_obs * 7 + n_pix)
    E = rng.normal(size=(n_pix, 3, n_obs)) * 1e5
    dS = rng.normal(size=(n_pix, n_obs // 2 + 1))
    dt = 2.3e-20
    dtype = torch.float64 if prec == "fp64" else torch.float32
    Et, dSt = torch.as_tensor(E, dtype=dtype, device=DEV), torch.as_tensor(dS, dtype=dtype, device=DEV)
    dE = lw.spectrum_fft_bwd(Et, dSt, dt, prec).double().cpu().numpy()
    ref = og.spectrum_vjp(Et.double().cpu().numpy(), dSt.double().cpu().numpy(), dt)
    err = np.max(np.abs(dE - ref)) / np.max(np.abs(ref))
    print(f"spectrum bwd {prec} n_obs={n_obs} n_pix={n_pix}: rel err {err:.2e}")
    assert err <= (1e-11 if prec == "fp64" else 3e-5)


def directions(c, rng):
    return (rng.normal(size=c["r"].shape) * oracle.C_LIGHT * c["dt_obs"],
            rng.normal(size=c["beta"].shape) * 1e-6,
            rng.normal(size=c["beta_dot"].shape) * np.max(np.abs(c["beta_dot"])))


def gpu_grads(c, dE, field_mask, geom, charge=None):
    from paper_2206_03015_amd import lw
    g = lw.deposit_td_bwd(T(c["r"]), T(c["beta"]), T(c["beta_dot"]), c["t_start"], c["dt"], T(c["x_det"]),
                          c["t0"], c["dt_obs"], c["n_obs"], T(dE), field_mask=field_mask, geom=geom,
                          charge=None if charge is None else T(charge))
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in g]


@pytest.mark.parametrize("geom", ["exact", "farfield"])
@pytest.mark.parametrize("field_mask", [1, 3])
def test_deposit_bwd_against_complex_step(geom, field_mask):
    """J = sum(dE * E_tot): the deposit adjoint dotted with random directions equals the
    complex-step derivative of the oracle's deposit."""
    c = synthetic(n_p=3, n_samples=300, n_pix=70, n_obs=256, seed=11)
    rng = np.random.default_rng(3)
    dE = rng.normal(size=(c["x_det"].shape[0], 3, c["n_obs"]))
    gr, gb, ga = gpu_grads(c, dE, field_mask, geom, c["charge"])
    vr, vb, va = directions(c, rng)
    for w in ((vr, 0 * vb, 0 * va), (0 * vr, vb, 0 * va), (0 * vr, 0 * vb, va)):
        d_cs, _ = og.directional_derivative(c["t_start"], c["dt"], c["r"], c["beta"], c["beta_dot"], *w,
                                            c["x_det"], c["t0"], c["dt_obs"], c["n_obs"], dE=dE,
                                            charge=c["charge"], field_mask=field_mask, geom=GEOMS[geom])
        d_gpu = np.sum(gr * w[0]) + np.sum(gb * w[1]) + np.sum(ga * w[2])
        print(f"{geom} mask {field_mask}: complex-step {d_cs:.6e} gpu {d_gpu:.6e}")
        assert d_gpu == pytest.approx(d_cs, rel=1e-8, abs=0)


def forward_J(c, W, geom, r=None, b=None, a=None):
    from paper_2206_03015_amd import lw
    r = c["r"] if r is None else r
    b = c["beta"] if b is None else b
    a = c["beta_dot"] if a is None else a
    E, _ = lw.deposit_td(T(r), T(b), T(a), c["t_start"], c["dt"], T(c["x_det"]), c["t0"], c["dt_obs"],
                         c["n_obs"], prec="fp64", geom=geom)
    S = lw.spectrum_fft(E, c["dt_obs"], "fp64")
    return float(torch.sum(T(W) * S).cpu()), E, S


def chain_grads(c, W, geom):
    from paper_2206_03015_amd import lw
    J, E, S = forward_J(c, W, geom)
    dE = lw.spectrum_fft_bwd(E, T(W), c["dt_obs"], "fp64")
    g = lw.deposit_td_bwd(T(c["r"]), T(c["beta"]), T(c["beta_dot"]), c["t_start"], c["dt"], T(c["x_det"]), c["t0"],
                          c["dt_obs"], c["n_obs"], dE, geom=geom)
    torch.cuda.synchronize()
    return J, [x.cpu().numpy() for x in g]


@pytest.mark.parametrize("geom", ["exact", "farfield"])
def test_full_chain_gradient(geom):
    """J = sum over a band of S on the bunch cut: GPU forward + FFT adjoint + deposit adjoint
    against complex-step derivatives of the oracle chain (random directions) and central
    differences of the GPU forward (smooth directions)."""
    c = small_bunch(n_p=6, n_steps=1500, n_side=3, n_obs=1 << 11)
    rng = np.random.default_rng(9)
    W = np.zeros((c["x_det"].shape[0], c["n_obs"] // 2 + 1))
    W[:, 20:200] = rng.random((W.shape[0], 180))
    J, (gr, gb, ga) = chain_grads(c, W, geom)
    vr, vb, va = directions(c, rng)
    for w in ((vr, 0 * vb, 0 * va), (0 * vr, vb, 0 * va), (0 * vr, 0 * vb, va)):
        d_cs, J0 = og.directional_derivative(c["t_start"], c["dt"], c["r"], c["beta"], c["beta_dot"], *w,
                                             c["x_det"], c["t0"], c["dt_obs"], c["n_obs"], weights=W,
                                             geom=GEOMS[geom])
        d_gpu = np.sum(gr * w[0]) + np.sum(gb * w[1]) + np.sum(ga * w[2])
        print(f"{geom}: J {J:.6e} (oracle {J0:.6e}); complex-step {d_cs:.6e} gpu-adjoint {d_gpu:.6e}")
        assert J == pytest.approx(J0, rel=1e-9, abs=0)
        assert d_gpu == pytest.approx(d_cs, rel=1e-8, abs=0)
    vr, vb, va = smooth_directions(c, rng)
    z = 0.0 * vr
    for name, w in (("r", (vr, z, z)), ("beta", (z, vb, z)), ("beta_dot", (z, z, va))):
        d_gpu = np.sum(gr * w[0]) + np.sum(gb * w[1]) + np.sum(ga * w[2])
        h = 1e-6
        Jp, _, _ = forward_J(c, W, geom, c["r"] + h * w[0], c["beta"] + h * w[1], c["beta_dot"] + h * w[2])
        Jm, _, _ = forward_J(c, W, geom, c["r"] - h * w[0], c["beta"] - h * w[1], c["beta_dot"] - h * w[2])
        fd = (Jp - Jm) / (2 * h)
        print(f"{geom} {name}: gpu-adjoint {d_gpu:.6e} gpu-fd {fd:.6e}")
        assert fd == pytest.approx(d_gpu, rel=FD_REL_TOL[name], abs=0)


def test_boris_bwd_against_complex_step():
    """lw_trajectory_boris_bwd contracted with random directions of the initial conditions and
    with a0 equals the complex-step derivative of the oracle pusher's G = sum g.(r, beta, beta_dot)."""
    from paper_2206_03015_amd import lw
    c = small_bunch(n_p=70, n_steps=1200, n_side=2)  # 70 particles: 490 lanes, a ragged last block
    W, L = c["W"], c["W"].laser
    rng = np.random.default_rng(31)
    g = [rng.normal(size=c["r"].shape) / np.maximum(np.std(x), 1e-300) for x in (c["r"], c["beta"], c["beta_dot"])]
    gi, ga0 = lw.trajectory_boris_bwd(T(c["init"]), W.n_samples, W.t_start, W.dt, L.a0, L.lam, L.w0, L.n_cycles,
                                      *(T(x) for x in g))
    torch.cuda.synchronize()
    gi, ga0 = gi.cpu().numpy(), ga0.cpu().numpy()
    h = 1e-30
    G = lambda parts: sum(np.sum(gk * p.imag) for gk, p in zip(g, parts)) / h
    scale = np.array([1e-6, 1e-6, 1e-6, 0.1, 0.1, 1.0])
    for trial in range(2):
        v = rng.normal(size=c["init"].shape) * scale
        d_cs = G(og.boris_complex(c["init"] + 1j * h * v, W.n_samples, W.t_start, W.dt, L.a0, L.lam, L.w0,
                                  L.n_cycles))
        d_gpu = np.sum(gi * v)
        print(f"init direction {trial}: complex-step {d_cs:.9e} gpu {d_gpu:.9e}")
        assert d_gpu == pytest.approx(d_cs, rel=1e-9, abs=0)
    d_cs = G(og.boris_complex(c["init"], W.n_samples, W.t_start, W.dt, L.a0 + 1j * h, L.lam, L.w0, L.n_cycles))
    print(f"a0: complex-step {d_cs:.9e} gpu {np.sum(ga0):.9e}")
    assert np.sum(ga0) == pytest.approx(d_cs, rel=1e-9, abs=0)
    # per-particle a0 parts: compare one particle alone
    k = 5
    d_k = G([x * (np.arange(x.shape[0]) == k)[:, None, None] for x in
             og.boris_complex(c["init"], W.n_samples, W.t_start, W.dt, L.a0 + 1j * h, L.lam, L.w0, L.n_cycles)])
    assert ga0[k] == pytest.approx(d_k, rel=1e-9, abs=0)


def params_setup():
    from paper_2206_03015_amd import inputs
    c = small_bunch(n_p=6, n_steps=1500, n_side=3, n_obs=1 << 11)
    full_w = inputs.workload("bunch")
    full = inputs.bunch_init(full_w)
    zc = np.sqrt(1.0 - 1.0 / c["W"].gamma ** 2) * inputs.C_LIGHT * c["W"].t_start
    rows = np.argsort(np.abs(full[:, 2] - zc))[: c["init"].shape[0]]
    rng = np.random.default_rng(21)
    Wt = np.zeros((c["x_det"].shape[0], c["n_obs"] // 2 + 1))
    Wt[:, 20:200] = rng.random((Wt.shape[0], 180))
    Wt[1] = 0.0  # one pixel without weight: the backward leaves it out
    return c, full_w, rows, Wt


def gpu_J(c, full_w, rows, Wt, gamma, a0, geom="exact"):
    from paper_2206_03015_amd import autograd as ag
    W = c["W"]
    init = ag.bunch_init(full_w, rows, gamma)
    r, b, bd = ag.boris_trajectory(init, a0, W)
    S, _ = ag.lw_spectrum(r, b, bd, W.t_start, W.dt, T(c["x_det"]), c["t0"], c["dt_obs"], c["n_obs"], geom=geom)
    return torch.sum(T(Wt) * S)


@pytest.mark.parametrize("geom", ["exact", "farfield"])
def test_params_gradient_autograd(geom):
    """torch.autograd through BunchInit -> BorisTrajectory -> LWSpectrum gives dJ/dgamma_mean and
    dJ/da0 equal to the oracle's complex step through draw, pusher, deposit and spectrum, and to
    central differences of the GPU forward (steps and tolerances of the oracle's own check)."""
    from paper_2206_03015_amd import inputs
    c, full_w, rows, Wt = params_setup()
    W, L = c["W"], c["W"].laser
    gamma = torch.tensor(W.gamma, dtype=torch.float64, requires_grad=True)
    a0 = torch.tensor(L.a0, dtype=torch.float64, requires_grad=True)
    J = gpu_J(c, full_w, rows, Wt, gamma, a0, geom)
    J.backward()
    dg, da = float(gamma.grad), float(a0.grad)
    init_of = lambda g: inputs.bunch_init(full_w, gamma=g)[rows]
    checks = []
    for which, d_gpu, x0 in (("gamma", dg, W.gamma), ("a0", da, L.a0)):
        d_cs, J0 = og.params_derivative(init_of, W.gamma, L.a0, (L.lam, L.w0, L.n_cycles), W.n_samples, W.t_start,
                                        W.dt, c["x_det"], c["t0"], c["dt_obs"], c["n_obs"], Wt, which,
                                        geom=GEOMS[geom])
        rel_step, tol = PARAM_FD[which]
        eps = rel_step * x0
        with torch.no_grad():
            if which == "gamma":
                Jp = float(gpu_J(c, full_w, rows, Wt, torch.tensor(x0 + eps, dtype=torch.float64), a0.detach(), geom))
                Jm = float(gpu_J(c, full_w, rows, Wt, torch.tensor(x0 - eps, dtype=torch.float64), a0.detach(), geom))
            else:
                Jp = float(gpu_J(c, full_w, rows, Wt, gamma.detach(), torch.tensor(x0 + eps, dtype=torch.float64), geom))
                Jm = float(gpu_J(c, full_w, rows, Wt, gamma.detach(), torch.tensor(x0 - eps, dtype=torch.float64), geom))
        fd = (Jp - Jm) / (2 * eps)
        print(f"{geom} d/d{which}: gpu {d_gpu:.9e} oracle complex-step {d_cs:.9e} gpu-fd {fd:.9e}; "
              f"J {float(J):.9e} oracle {J0:.9e}")
        checks.append((J0, d_cs, d_gpu, fd, tol))
    for J0, d_cs, d_gpu, fd, tol in checks:
        assert float(J) == pytest.approx(J0, rel=1e-9, abs=0)
        assert d_gpu == pytest.approx(d_cs, rel=1e-8, abs=0)
        assert fd == pytest.approx(d_gpu, rel=tol, abs=0)


def test_lw_spectrum_autograd_matches_entry_points():
    """LWSpectrum's backward equals the explicit fft_bwd + deposit_bwd calls (pixel skipping included)."""
    from paper_2206_03015_amd import autograd as ag
    c = small_bunch(n_p=6, n_steps=1500, n_side=3, n_obs=1 << 11)
    rng = np.random.default_rng(2)
    Wt = rng.random((c["x_det"].shape[0], c["n_obs"] // 2 + 1))
    Wt[[0, 4]] = 0.0
    r, b, bd = (T(c[k]).requires_grad_(True) for k in ("r", "beta", "beta_dot"))
    S, _ = ag.lw_spectrum(r, b, bd, c["t_start"], c["dt"], T(c["x_det"]), c["t0"], c["dt_obs"], c["n_obs"])
    torch.sum(T(Wt) * S).backward()
    _, (gr, gb, ga) = chain_grads(c, Wt, "exact")
    for auto, ref in ((r.grad, gr), (b.grad, gb), (bd.grad, ga)):
        a = auto.cpu().numpy()
        assert np.max(np.abs(a - ref)) <= 1e-12 * np.max(np.abs(ref))


def fd_case(n_omega):
    c = synthetic(n_p=3, n_samples=300, n_pix=5, n_obs=256, seed=2)
    tau, _, _ = oracle.eval_samples(c["t_start"], c["dt"], c["r"], c["beta"], c["beta_dot"], c["x_det"][:1], 0.0, 1.0)
    w1 = 2 * np.pi / (np.ptp(tau) / 30)
    return c, np.linspace(0.2, 2.0, n_omega) * w1


@pytest.mark.parametrize("geom", ["exact", "farfield"])
@pytest.mark.parametrize("n_omega", [37, 100])
def test_direct_fd_bwd(geom, n_omega):
    """lw_direct_fd_bwd against complex-step derivatives of the oracle's direct sum (random
    directions) and central differences of the GPU forward in FP64 (smooth directions)."""
    from paper_2206_03015_amd import lw
    c, omega = fd_case(n_omega)
    rng = np.random.default_rng(n_omega)
    dS = rng.random((c["x_det"].shape[0], n_omega))
    gr, gb, ga = (x.cpu().numpy() for x in lw.direct_fd_bwd(
        T(c["r"]), T(c["beta"]), T(c["beta_dot"]), c["t_start"], c["dt"], T(c["x_det"]), c["t0"], T(omega), T(dS),
        field_mask=3, geom=geom, charge=T(c["charge"])))
    vr, vb, va = directions(c, rng)
    for w in ((vr, 0 * vb, 0 * va), (0 * vr, vb, 0 * va), (0 * vr, 0 * vb, va)):
        d_cs, _ = og.fd_directional_derivative(c["t_start"], c["dt"], c["r"], c["beta"], c["beta_dot"], *w,
                                               c["x_det"], c["t0"], omega, dS, charge=c["charge"], field_mask=3,
                                               geom=GEOMS[geom])
        d_gpu = np.sum(gr * w[0]) + np.sum(gb * w[1]) + np.sum(ga * w[2])
        print(f"{geom} n_omega {n_omega}: complex-step {d_cs:.9e} gpu {d_gpu:.9e}")
        assert d_gpu == pytest.approx(d_cs, rel=1e-8, abs=0)

    def J(r, b, a):
        S = lw.direct_fd(T(r), T(b), T(a), c["t_start"], c["dt"], T(c["x_det"]), c["t0"], T(omega), prec="fp64",
                         field_mask=3, geom=geom, charge=T(c["charge"]))
        return float(torch.sum(T(dS) * S).cpu())

    vr, vb, va = smooth_directions(c, rng)
    z = 0.0 * vr
    for name, w in (("r", (vr, z, z)), ("beta", (z, vb, z)), ("beta_dot", (z, z, va))):
        h = 1e-4
        fd = (J(c["r"] + h * w[0], c["beta"] + h * w[1], c["beta_dot"] + h * w[2]) -
              J(c["r"] - h * w[0], c["beta"] - h * w[1], c["beta_dot"] - h * w[2])) / (2 * h)
        d_gpu = np.sum(gr * w[0]) + np.sum(gb * w[1]) + np.sum(ga * w[2])
        print(f"{geom} {name}: gpu-adjoint {d_gpu:.9e} gpu-fd {fd:.9e}")
        assert fd == pytest.approx(d_gpu, rel=1e-6, abs=0)
