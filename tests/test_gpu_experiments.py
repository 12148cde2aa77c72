"""The experiment modes of bench.py on the GPU: properties that must hold whatever the timings.

Accuracy experiment (Sec. "Accuracy"): the converged reference is converged (16x against 8x
finer trajectory), the direct sum on the 2e4-step trajectory is far more accurate than the
paper's tolerance, the time-domain error falls as the observer grid is refined and is flat in
N_w (zero padding only).  Wall-clock model (Sec. "Performance"): every single-variate sweep
gives a constant within a factor 2 of the mean, and the crossover rows are complete."""
import os
import sys

import pytest
import torch

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
