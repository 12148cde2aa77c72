"""The experiment modes of bench.py on the GPU: properties that must hold whatever the timings.

Accuracy experiment (Sec. "Accuracy"): the converged reference is converged (16x against 8x
finer trajectory), the direct sum on the 2e4-step trajectory is far more accurate than the
paper's tolerance, the time-domain error falls as the observer grid is refined and is flat in
N_w (zero padding only).  Wall-clock model (Sec. "Performance"): every single-variate sweep
gives a constant within a factor 2 of the mean, and the crossover rows are complete."""
import os
import sys

import numpy as np
import pytest
import torch

import oracle

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def test_accuracy_experiment():
    out = bench.accuracy(torch, DEV)
    rows = out["rows"]
    assert [r["n_omega"] for r in rows] == [4096, 8192, 16384]
    for r in rows:
        assert r["ref_8x"]["max"] < 1e-7
        assert r["fd"]["max"] < 1e-5
        assert r["td"]["max"] < 0.2
        assert abs(r["td"]["max"] - rows[0]["td"]["max"]) <= 1e-3 * rows[0]["td"]["max"]
    finer = rows[0]["td_finer_grid"]
    errs = [rows[0]["td"]["max"]] + [f["max"] for f in finer]
    assert all(b < a for a, b in zip(errs, errs[1:]))
    assert finer[-1]["max"] < 1e-5


def test_accuracy_experiment_against_oracle():
    """Four observers of the accuracy experiment at N_w = 4096 (N_Tu = 8192): the time-domain
    spectra (FP64 deposit + FFT) and the direct frequency-domain sum (FP64) on the experiment's
    2e4-step trajectory against the oracle's deposit + spectrum and direct sum on the same
    trajectory, element by element: max relative error per observer <= 1e-10; the mixed
    time-domain spectra within 1e-4 band-L2 over the three harmonics."""
    from paper_2206_03015_amd import lw
    A = bench.accuracy_setup(torch, DEV)
    dt, (r, b, bd) = A["traj"](A["n_s"] + 1)
    sel = [0, 25, 50, 90]
    x = A["x_det"][sel].contiguous()
    n_w = 4096
    n_obs, dt_obs, t0, t_start = 2 * n_w, A["dt_obs"], A["t0"], A["t_start"]
    omega = np.arange(n_w + 1) * (A["w_max"] / n_w)
    E, _ = lw.deposit_td(r, b, bd, t_start, dt, x, t0, dt_obs, n_obs, prec="fp64")
    S_td = lw.spectrum_fft(E, dt_obs, "fp64").cpu().numpy()
    Em, _ = lw.deposit_td(r, b, bd, t_start, dt, x, t0, dt_obs, n_obs, prec="mixed")
    S_mix = lw.spectrum_fft(Em, dt_obs, "mixed").double().cpu().numpy()
    S_fd = lw.direct_fd(r, b, bd, t_start, dt, x, t0, torch.as_tensor(omega, device=DEV), prec="fp64").cpu().numpy()
    rn, bn, bdn, xn = (t.cpu().numpy() for t in (r, b, bd, x))
    Eo, do = oracle.deposit_td(t_start, dt, rn, bn, bdn, xn, t0, dt_obs, n_obs)
    So = oracle.spectrum(Eo, dt_obs)
    So_fd = oracle.direct_fd(t_start, dt, rn, bn, bdn, xn, t0, omega)
    assert do[0] == do[1] == do[2] == 0 and do[3] > 0  # the whole pulse inside the window
    for j, m in enumerate(sel):
        e_td = np.max(np.abs(S_td[j] - So[j])) / np.max(So[j])
        e_fd = np.max(np.abs(S_fd[j] - So_fd[j])) / np.max(So_fd[j])
        e_mix = np.linalg.norm(S_mix[j, 1:n_w + 1] - So[j, 1:n_w + 1]) / np.linalg.norm(So[j, 1:n_w + 1])
        print(f"observer {m} (theta {A['theta'][m]:+.3f}): TD FP64 {e_td:.2e}, FD FP64 {e_fd:.2e}, TD mixed {e_mix:.2e}")
        assert e_td <= 1e-10
        assert e_fd <= 1e-10
        assert e_mix <= 1e-4


def test_cost_model_refit():
    out = bench.cost_model(torch, DEV)
    c = out["constants"]
    for name in ("C1_t", "C2_t", "C_w"):
        assert c[name] > 0
        for v in c["per_sweep"][name].values():
            assert 0.5 * c[name] <= v <= 2.0 * c[name]
    x = out["crossover"]
    assert len(x["n_p"]) == len(x["td_s"]) == len(x["fd_s"]) == 13
    assert all(t > 0 for t in x["td_s"] + x["fd_s"])
