"""Host logic of bench.py's experiment modes (no GPU): the single-variate fits of Sec.
"Performance" recover a known leading constant, the crossover finder, the line bunch of the
crossover setting, and the error measure of Eq. spectra_error."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_fit_recovers_constant_of_exact_data():
    C = 3.7e-13
    sweeps = {"a": [(x, C * x) for x in (1e9, 2e9, 4e9)], "b": [(x, C * x) for x in (5e8, 3e9)]}
    c, per = bench.fit_leading_constant(sweeps)
    assert abs(c - C) <= 1e-15 * C * 10
    assert set(per) == {"a", "b"}


def test_fit_is_least_squares_per_sweep_then_mean():
    # sweep a: t = 2x except one point off; least squares through the origin by hand
    a = [(1.0, 2.0), (2.0, 4.0), (3.0, 7.0)]
    b = [(1.0, 1.0), (2.0, 2.0)]
    c, per = bench.fit_leading_constant({"a": a, "b": b})
    ca = (1 * 2 + 2 * 4 + 3 * 7) / (1 + 4 + 9)
    assert per["a"] == ca and per["b"] == 1.0
    assert c == (ca + 1.0) / 2


def test_crossover():
    n = [1, 2, 5, 10, 20]
    assert bench.crossover(n, [5, 5, 5, 5, 5], [1, 2, 4, 8, 16]) == 10.0
    assert bench.crossover(n, [5, 5, 5, 5, 5], [1, 1, 1, 1, 1]) is None
    # a faster TD point below a slower one does not count
    assert bench.crossover(n, [1, 5, 5, 5, 5], [2, 2, 6, 6, 6]) == 5.0


def test_uniform_line_bunch():
    from paper_2206_03015_amd import inputs
    init = inputs.uniform_line_init(4, 100e-6, 5.0, 0.0)
    assert np.allclose(init[:, 2], [-37.5e-6, -12.5e-6, 12.5e-6, 37.5e-6], rtol=0, atol=1e-18)
    assert np.all(init[:, :2] == 0) and np.all(init[:, 3:5] == 0)
    assert np.allclose(1.0 + init[:, 5] ** 2, 25.0, rtol=1e-15)


def test_spectra_error():
    S_ref = np.array([[1.0, 4.0], [2.0, 0.0]])
    S = np.array([[1.5, 4.0], [2.0, 1.0]])
    mx, mean = bench.spectra_error(S, S_ref)
    assert mx == 0.25 and mean == (0.125 + 0.25) / 4


@pytest.mark.parametrize("name, evals, points", [("precision", 100000 * 20001 * 16384, 52661621409),
                                                  ("bunch", 10000 * 20001 * 4096, 11087079962)])
def test_committed_counter_figures_describe_the_committed_deposit(name, evals, points):
    """The counter summaries under profiles/ carry a SHA-256 of the deposit sources; bench.py
    reports their figures (HBM traffic, VALU instructions, FP64/FP32 flops per step) only while
    the sources are unchanged.  Where the committed summaries match the committed sources, their
    values must be sane."""
    paths = bench.SUMMARIES[name]
    if not all(os.path.exists(os.path.join(bench.ROOT, p)) for p in paths.values()):
        pytest.skip(f"no committed {name} counter summaries")
    traffic = bench._summary_value(paths["traffic"], "hbm_bytes_per_step")
    valu = bench._summary_value(paths["valu"], "valu_insts_per_step")
    f64 = bench._summary_value(paths["types"], "f64_flops_per_step")
    f32 = bench._summary_value(paths["types"], "f32_flops_per_step")
    if None in (traffic, valu, f64, f32):
        pytest.skip(f"the {name} counter summaries predate the current deposit sources")
    # at least the trace once; at most a read-modify-write of three 128-byte trace lines per
    # deposited grid point plus a byte per evaluation (points: the deposited grid points, diag[3])
    assert 12e9 <= traffic < 3 * 2 * 128 * points + evals
    # wavefront instructions: at least one per 64 evaluations, at most 32 lane-instructions per
    # evaluation
    assert evals / 64 <= valu <= 32 * evals / 64
    # the arrival time's FP64 FMA-class work dominates; the fields at the crossings are FP32
    assert f64 > f32 > 0
