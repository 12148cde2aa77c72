"""GPU parity of lw_deposit_td against the FP64 oracle (Algorithm 2), element by element.

Tolerances: FP64 mode, max |E_gpu - E_oracle| <= 1e-9 max|E_oracle| (arrival times enter the
weights with rounding ~1e-16 * |tau| ~ 1e-9 grid units at the largest tau here, and the
trace is continuous in tau); mixed mode (fields and trace in float), <= 2e-5 max|E|.
Diagnostic counters are integers and must match exactly."""
import numpy as np
import pytest
import torch

import oracle
from cases import single_electron, small_bunch, synthetic

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-9, "mixed": 2e-5}


def run_gpu(c, prec, geom, field_mask=1, charge=None, accumulate=False, out=None, cull=False):
    from paper_2206_03015_amd import lw
    dev = torch.device("cuda:0")
    t = {k: torch.as_tensor(np.ascontiguousarray(c[k]), device=dev) for k in ("r", "beta", "beta_dot", "x_det")}
    ch = None if charge is None else torch.as_tensor(charge, device=dev)
    E, diag = lw.deposit_td(t["r"], t["beta"], t["beta_dot"], c["t_start"], c["dt"], t["x_det"], c["t0"], c["dt_obs"],
                            c["n_obs"], prec=prec, field_mask=field_mask, geom=geom, charge=ch, out=out,
                            accumulate=accumulate, cull=cull)
    torch.cuda.synchronize()
    return E.double().cpu().numpy(), diag.cpu().numpy()


def run_oracle(c, geom, field_mask=1, charge=None):
    g = oracle.GEOM_EXACT if geom == "exact" else oracle.GEOM_FARFIELD
    return oracle.deposit_td(c["t_start"], c["dt"], c["r"], c["beta"], c["beta_dot"], c["x_det"], c["t0"],
                             c["dt_obs"], c["n_obs"], charge=charge, field_mask=field_mask, geom=g)


def assert_close(Eg, Eo, prec):
    scale = np.max(np.abs(Eo))
    assert scale > 0
    err = np.max(np.abs(Eg - Eo)) / scale
    print(f"max rel err {err:.3e} (prec {prec})")
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("geom", ["exact", "farfield"])
def test_single_electron(prec, geom):
    c = single_electron(thetas=(0.0, 0.01, 0.02))
    Eo, do = run_oracle(c, geom)
    Eg, dg = run_gpu(c, prec, geom)
    assert_close(Eg, Eo, prec)
    assert dg.tolist() == do.tolist()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("geom", ["exact", "farfield"])
@pytest.mark.parametrize("field_mask", [1, 3])
def test_small_bunch(prec, geom, field_mask):
    """24 Boris-pushed electrons, 10x10 pixels (two 64-pixel tiles, ragged), 2^12 grid points."""
    c = small_bunch()
    Eo, do = run_oracle(c, geom, field_mask)
    Eg, dg = run_gpu(c, prec, geom, field_mask)
    assert_close(Eg, Eo, prec)
    assert dg.tolist() == do.tolist()
    assert do[3] > 100000


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_synthetic_with_charges(prec):
    c = synthetic()
    Eo, do = run_oracle(c, "exact", 3, charge=c["charge"])
    Eg, dg = run_gpu(c, prec, "exact", 3, charge=c["charge"])
    assert_close(Eg, Eo, prec)
    assert dg.tolist() == do.tolist()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_dense_grid_long_intervals(prec):
    """Observer grids much finer than the sample spacing: ~21 grid points per interval
    (synthetic, with charges, both fields) and ~50-60 (a small bunch at 4000 grid points per
    first-harmonic period).  Intervals with more than eight grid points are deposited by the
    whole wavefront, the rest lane by lane."""
    c = synthetic(n_p=5, n_samples=100, n_pix=70, n_obs=6000, seed=5)
    Eo, do = run_oracle(c, "exact", 3, charge=c["charge"])
    assert do[3] > 20 * 5 * 99 * 70
    Eg, dg = run_gpu(c, prec, "exact", 3, charge=c["charge"])
    assert_close(Eg, Eo, prec)
    assert dg.tolist() == do.tolist()
    c = small_bunch(n_p=8, n_steps=600, n_side=3, n_obs=1 << 14, samples_per_period=4000.0)
    for geom in ("exact", "farfield"):
        Eo, do = run_oracle(c, geom)
        assert do[3] > 100000
        Eg, dg = run_gpu(c, prec, geom)
        assert_close(Eg, Eo, prec)
        assert dg.tolist() == do.tolist()


def offset_cluster(offset, th0, D, n_obs, n_p=3, n_samples=700, n_pix=12, seed=3, dt=2e-18):
    """Synthetic trajectories shifted by a common offset, seen by a cluster of pixels at angles
    th0 (+-1e-5 rad) and distance D, with a window cutting through the arrival times; returns
    the case and the bounds, in grid units, of the terms the records leave out in their
    lower-degree evaluation: K e b^3 of degree 3 (mixed) and c_4 b^4 + c_5 b^5 of degree 5 (FP64,
    |c_4| <= 1.3 K e^2, c_5 = 7 K e^3 / 4), with |b| <= C sqrt(2 (1 - n_z)) |r|, e = 1/(C D),
    K = e/2."""
    from paper_2206_03015_amd import inputs
    r, b, bd = inputs.random_trajectory(n_p, n_samples, seed=seed, dt=dt, spread=0.0)
    r = r + np.asarray(offset)[None, None, :]
    rng = np.random.default_rng(seed)
    th = np.asarray(th0) + rng.uniform(-1e-5, 1e-5, size=(n_pix, 2))
    x = D * np.stack([np.sin(th[:, 0]), np.cos(th[:, 0]) * np.sin(th[:, 1]), np.cos(th[:, 0]) * np.cos(th[:, 1])], -1)
    tau, _, _ = oracle.eval_samples(0.0, dt, r, b, bd, x[:1], 0.0, 1.0)
    dt_obs = np.ptp(tau[0, 0]) / (0.7 * n_obs)
    t0 = np.median(tau) - 0.5 * n_obs * dt_obs
    C = 1.0 / (oracle.C_LIGHT * dt_obs)
    rb2 = np.max(np.sum(r * r, -1))
    s2 = np.max(2.0 * (1.0 - x[:, 2] / np.linalg.norm(x, axis=1)))
    bmax = C * np.sqrt(rb2 * s2)
    e = 1.0 / (C * D)
    K = 0.5 * e
    tails = {"mixed": K * e * bmax ** 3, "fp64": (1.3 * K * e * e + 1.75 * K * e ** 3 * bmax) * bmax ** 4}
    return dict(r=r, beta=b, beta_dot=bd, t_start=0.0, dt=dt, x_det=x, t0=t0, dt_obs=dt_obs, n_obs=n_obs), tails


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("regime", ["tail_negligible", "tail_kept"])
def test_record_polynomial_lower_degree(prec, regime):
    """The records are evaluated to a lower degree (2 of 3 with single-precision fields, 3 of 5
    with double ones) where the bound of the terms left out over the particle and the tile is at
    most 1e-7, resp. 1e-12 grid units, in full otherwise: one case on each side of both bounds
    (trajectories near the origin, pixels at ~0.02 rad and 1 m; trajectories offset by ~8.5 um,
    pixels at ~0.36 rad and 0.1 m, a finer window), against the oracle element by element,
    counters exact."""
    bound = {"mixed": 1e-7, "fp64": 1e-12}[prec]
    if regime == "tail_negligible":
        c, tails = offset_cluster((0.0, 0.0, 0.0), (0.02, 0.01), 1.0, 600)
        assert tails[prec] < 1e-2 * bound
    else:
        c, tails = offset_cluster((6e-6, 6e-6, 0.0), (0.3, 0.2), 0.1, 6000)
        assert tails[prec] > 1e2 * bound and np.max(np.sum(c["r"] ** 2, -1)) <= 1e-8 * 0.1 ** 2  # series range
    Eo, do = run_oracle(c, "exact")
    assert do[3] > 10000
    Eg, dg = run_gpu(c, prec, "exact")
    assert_close(Eg, Eo, prec)
    assert dg.tolist() == do.tolist()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("geom", ["exact", "farfield"])
def test_cull_changes_work_not_results(prec, geom):
    """LW_CULL skips fast-path particles whose arrival span holds no window grid point of a
    wavefront's pixels: same spectra and counters as the full evaluation (the trace up to the
    order of floating-point atomic additions), and both match the oracle.  Most of these 256
    particles miss the window; the synthetic case adds careful-path particles, never skipped."""
    c = small_bunch(n_p=256, n_steps=1000, n_side=12, n_obs=1 << 12)
    Eo, do = run_oracle(c, geom)
    Ef, df = run_gpu(c, prec, geom)
    Ec, dc = run_gpu(c, prec, geom, cull=True)
    assert dc.tolist() == df.tolist() == do.tolist()
    assert do[2] > 4 * do[3] > 0  # mostly outside the window
    assert np.max(np.abs(Ec - Ef)) <= (1e-13 if prec == "fp64" else 1e-6) * np.max(np.abs(Ef))
    assert_close(Ec, Eo, prec)
    c = synthetic(n_p=4, seed=3)
    c["r"] = c["r"].copy()
    c["r"][1, 300:305] = c["r"][1, 299]  # a particle at rest for a few samples: careful path
    Eo, do = run_oracle(c, geom)
    Ec, dc = run_gpu(c, prec, geom, cull=True)
    assert dc.tolist() == do.tolist()
    assert_close(Ec, Eo, prec)


def test_unusable_samples_and_nonmonotone_take_the_careful_path():
    c = synthetic(n_p=4, seed=3)
    c["r"] = c["r"].copy()
    c["beta"] = c["beta"].copy()
    c["beta"][1, 100, 0] = np.nan  # unusable sample
    c["beta"][2, 50] = [0.0, 0.0, 1.0]  # |beta| = 1: unusable
    c["r"][3, 300:303] = c["r"][3, 300:303][::-1]  # swapped samples -> non-monotone intervals
    c["x_det"] = c["x_det"].copy()
    c["x_det"][5] = 0.0  # pixel at the origin: every interval unusable
    Eo, do = run_oracle(c, "exact")
    Eg, dg = run_gpu(c, "fp64", "exact")
    assert do[0] > 0 and do[1] > 0
    assert dg.tolist() == do.tolist()
    assert_close(Eg, Eo, "fp64")


def test_accumulate_equals_one_call():
    """Particle-chunked calls with LW_ACCUMULATE add up to the single call."""
    c = small_bunch(n_p=10, n_steps=1500, n_side=4)
    Eo, do = run_oracle(c, "exact")
    a = {k: c[k] for k in c}
    a.update(r=c["r"][:4], beta=c["beta"][:4], beta_dot=c["beta_dot"][:4])
    b = {k: c[k] for k in c}
    b.update(r=c["r"][4:], beta=c["beta"][4:], beta_dot=c["beta_dot"][4:])
    from paper_2206_03015_amd import lw
    dev = torch.device("cuda:0")
    E = torch.full((c["x_det"].shape[0], 3, c["n_obs"]), 7.0, dtype=torch.float64, device=dev)
    run_gpu(a, "fp64", "exact", out=E)  # overwrite
    Eg, _ = run_gpu(b, "fp64", "exact", out=E, accumulate=True)
    assert_close(Eg, Eo, "fp64")
    assert lw is not None


def test_degenerate_sizes():
    from paper_2206_03015_amd import lw
    dev = torch.device("cuda:0")
    c = synthetic(n_p=2, n_samples=50, n_pix=3, n_obs=16)
    # no particles: trace overwritten with zeros
    z = {k: c[k] for k in c}
    z.update(r=c["r"][:0], beta=c["beta"][:0], beta_dot=c["beta_dot"][:0])
    out = torch.full((3, 3, 16), 5.0, dtype=torch.float64, device=dev)
    Eg, dg = run_gpu(z, "fp64", "exact", out=out)
    assert np.all(Eg == 0) and dg.tolist() == [0, 0, 0, 0]
    # one sample per particle: no interval
    one = {k: c[k] for k in c}
    one.update(r=c["r"][:, :1].copy(), beta=c["beta"][:, :1].copy(), beta_dot=c["beta_dot"][:, :1].copy())
    Eg, dg = run_gpu(one, "mixed", "farfield")
    assert np.all(Eg == 0) and dg.tolist() == [0, 0, 0, 0]
    # no pixels
    nop = {k: c[k] for k in c}
    nop["x_det"] = c["x_det"][:0]
    Eg, dg = run_gpu(nop, "fp64", "exact")
    assert Eg.shape == (0, 3, 16)
    # a one-point observer grid, and two points, against the oracle
    for n_obs in (1, 2):
        c1 = synthetic(n_p=3, n_samples=50, n_pix=3, n_obs=n_obs)
        for prec in ("fp64", "mixed"):
            Eg, dg = run_gpu(c1, prec, "exact")
            Eo, do = run_oracle(c1, "exact")
            assert_close(Eg, Eo, prec)
            assert dg.tolist() == do.tolist()
    assert lw is not None


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_largest_grid(prec):
    """The largest observer grid the library takes, n_obs = 2^31 - 1 (grid indices are 32-bit):
    the same trajectories as a 4096-point window, with t0 moved back by the K = 2^31 - 1 - 4096
    extra grid steps, so that grid point u of the small window is point u + K of the large one.
    The large trace's last 4096 points equal the oracle's small-window trace (within the
    rounding of arrival times of magnitude ~2^31 grid units: 1e-6 of the maximum), and every
    interval's grid points are counted once either way (the small window's points below it are
    inside the large one)."""
    from paper_2206_03015_amd import lw
    dev = torch.device("cuda:0")
    c = synthetic(n_p=3, n_samples=300, n_pix=1, n_obs=4096)
    Eo, do = run_oracle(c, "exact")
    n_big = (1 << 31) - 1
    K = n_big - c["n_obs"]
    t = {k: torch.as_tensor(np.ascontiguousarray(c[k]), device=dev) for k in ("r", "beta", "beta_dot", "x_det")}
    E, diag = lw.deposit_td(t["r"], t["beta"], t["beta_dot"], c["t_start"], c["dt"], t["x_det"],
                            c["t0"] - K * c["dt_obs"], c["dt_obs"], n_big, prec=prec)
    tail = E[:, :, K:].double().cpu().numpy()
    below = E[:, :, :K]  # points the small window drops below its start
    head = max(below.max().item(), -below.min().item())
    del below
    diag = diag.cpu().numpy()
    del E
    torch.cuda.empty_cache()
    scale = np.max(np.abs(Eo))
    assert scale > 0
    err = np.max(np.abs(tail - Eo)) / scale
    print(f"n_obs = 2^31 - 1, {prec}: tail vs oracle {err:.2e}, below-window max {head:.2e}, diag {diag.tolist()}")
    assert err <= (1e-6 if prec == "fp64" else 2e-5)
    assert int(diag[2] + diag[3]) == int(do[2] + do[3])
    assert int(diag[3]) >= int(do[3]) > 0
    assert (head > 0) == (int(diag[3]) > int(do[3]))
