"""lw_spectrum_fft_noalloc (the entry point for callers that cannot allocate) against
lw_spectrum_fft with a workspace: two calls in a row on one GPU, the second on a smaller input,
both precisions, through the C ABI.  The scratch is shared and keeps the previous call's
contents, so the second call also shows that nothing in it needs clearing.  The two entry
points run the same kernels on the same pixel pairs (only the batching differs), so the spectra
must agree bit for bit; both are also checked against the oracle at the FFT's parity bounds."""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_fft_equals_workspace_fft(prec):
    from paper_2206_03015_amd import lw
    dtype = torch.float64 if prec == "fp64" else torch.float32
    dt_obs = 2.3e-20
    # the second call is smaller (fewer pixels, shorter grid); the first spans several batches of
    # the 64 MiB scratch (2^18 points: 6 or 12 MiB per pixel pair) with a ragged last pair
    for n_pix, n_obs, seed in ((41, 1 << 18, 1), (5, 1 << 12, 2)):
        rng = np.random.default_rng(seed)
        E = torch.as_tensor(rng.normal(size=(n_pix, 3, n_obs)) * 1e5, dtype=dtype, device=DEV)
        S_ws = lw.spectrum_fft(E, dt_obs, prec)
        S_na = torch.full_like(S_ws, float("nan"))
        lw.spectrum_fft_noalloc(E, dt_obs, S_na, prec)
        torch.cuda.synchronize()
        a, b = S_na.double().cpu().numpy(), S_ws.double().cpu().numpy()
        assert np.isfinite(a).all()
        assert np.array_equal(a, b), f"{prec} {n_pix}x{n_obs}: max diff {np.max(np.abs(a - b))}"
        So = oracle.spectrum(E.double().cpu().numpy(), dt_obs)
        err = np.max(np.abs(a - So)) / np.max(So)
        print(f"{prec} n_pix={n_pix} n_obs={n_obs}: equal to the workspace call; oracle rel err {err:.2e}")
        assert err <= (1e-12 if prec == "fp64" else 2e-5)


def test_noalloc_fft_rejects_grids_beyond_its_scratch():
    from paper_2206_03015_amd import lw
    assert lw.noalloc_scratch_bytes() == 64 << 20
    n_obs = 1 << 21  # one FP64 pixel pair needs 3 * 2^21 * 16 bytes = 96 MiB
    E = torch.zeros((1, 3, n_obs), dtype=torch.float64, device=DEV)
    S = torch.zeros((1, n_obs // 2 + 1), dtype=torch.float64, device=DEV)
    with pytest.raises(lw.LWError) as ei:
        lw.spectrum_fft_noalloc(E, 1e-20, S, "fp64")
    assert ei.value.status == -4 and "static scratch" in str(ei.value)
