"""The C-ABI library loads and exports every entry point that include/lw.h declares
(no GPU needed: only host-side calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lw.h")
LIB = os.environ.get("LW_LIBRARY") or os.path.join(ROOT, "paper_2206_03015_amd", "liblw.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*?\**\s*\b(lw_[a-z0-9_]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("liblw.so is not built (run __graft_entry__.build())")
    from paper_2206_03015_amd import lw
    return lw.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("lw_deposit_td", "lw_spectrum_fft", "lw_direct_fd", "lw_deposit_td_bwd", "lw_spectrum_fft_bwd",
              "lw_direct_fd_bwd", "lw_trajectory_boris", "lw_workspace_bytes", "lw_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for n in declared_functions():
        assert n in exported, n
        assert getattr(lib, n) is not None


def test_binding_covers_the_header():
    from paper_2206_03015_amd import lw
    assert set(declared_functions()) == set(lw._SIGS)


def test_workspace_sizes(lib):
    from paper_2206_03015_amd import lw
    assert lw.workspace_bytes(lw.WS_DEPOSIT, 1000, 20001) >= 1000 * 4 + 20001 * 8
    fft = lw.workspace_bytes(lw.WS_FFT, 7, 1 << 12, "fp64")
    assert fft >= 3 * (1 << 12) * 16 and fft % (3 * (1 << 12) * 16) == 0
    assert lw.workspace_bytes(lw.WS_DIRECT_FD, 3, 5) >= 3 * 5 * 6 * 8
    assert lw.workspace_bytes(lw.WS_DIRECT_FD_BWD, 3, 5, "fp64") == lw.workspace_bytes(lw.WS_DIRECT_FD, 3, 5)
    # Boris batches and spans: the whole set when small, capped near 16 GiB when large
    small = lw.workspace_bytes(lw.WS_DEPOSIT_BORIS, 10, 1000)
    assert small >= 10 * 1000 * 72
    big = lw.workspace_bytes(lw.WS_DEPOSIT_BORIS, 100000, 20001)
    assert 15.5 * 2**30 < big < 16.5 * 2**30
    assert lw.workspace_bytes(lw.WS_DEPOSIT_BWD_BORIS, 10, 1000) >= 10 * 1000 * 144
    assert 15.5 * 2**30 < lw.workspace_bytes(lw.WS_DEPOSIT_BWD_BORIS, 100000, 20001) < 16.5 * 2**30
    assert lib.lw_workspace_bytes(999, 1, 1, 0) == 0
    # order-independent deposit: a high word per trace element and a scale per trace row
    assert lw.workspace_bytes(lw.WS_DEPOSIT_DET_ACC, 7, 64, "fp64") >= 7 * 3 * 64 * 8 + 7 * 3 * 8
    assert lw.workspace_bytes(lw.WS_DEPOSIT_DET_ACC, -1, 64, "fp64") == 0


def test_host_validation_rejects_bad_arguments(lib):
    """Each call returns its error code before any HIP call for these inputs."""
    from paper_2206_03015_amd import lw
    tr = lw.Traj()
    tr.kind = lw.TRAJ_SAMPLES
    tr.n_particles = 1
    tr.n_samples = 10
    tr.t_start = 0.0
    tr.dt = 1e-18
    gr = lw.Grid()
    gr.n_pix = 1
    gr.t0 = 0.0
    gr.dt_obs = 1e-20
    gr.n_obs = 64
    st = lib.lw_deposit_td(None, ctypes.byref(gr), 0, 1, 0, None, None, None, 0, None)
    assert st == -1 and b"traj is NULL" in lib.lw_last_error()
    st = lib.lw_deposit_td(ctypes.byref(tr), ctypes.byref(gr), 0, 1, 0, None, None, None, 0, None)
    assert st == -1  # NULL trajectory arrays
    tr.dt = -1.0
    assert lib.lw_deposit_td(ctypes.byref(tr), ctypes.byref(gr), 0, 1, 0, None, None, None, 0, None) == -1
    tr.dt = 1e-18
    tr.n_samples = 0
    assert lib.lw_deposit_td(ctypes.byref(tr), ctypes.byref(gr), 0, 1, 0, None, None, None, 0, None) == -2
    tr.n_samples = 10
    tr.kind = lw.TRAJ_BORIS  # accepted kind, but init is NULL
    assert lib.lw_deposit_td(ctypes.byref(tr), ctypes.byref(gr), 0, 1, 0, None, None, None, 0, None) == -1
    # spectrum: n_obs must be a power of two >= 4
    assert lib.lw_spectrum_fft(None, 1, 100, 1e-20, 0, None, None, 0, None) == -2
    assert lib.lw_spectrum_fft(None, 1, 2, 1e-20, 0, None, None, 0, None) == -2
    assert lib.lw_spectrum_fft(None, 1, 64, -1.0, 0, None, None, 0, None) == -1
    assert lib.lw_spectrum_fft(None, 1, 64, 1e-20, 7, None, None, 0, None) == -1
    # misaligned pointers are refused
    assert lib.lw_spectrum_fft(ctypes.c_void_p(8), 1, 64, 1e-20, 0, ctypes.c_void_p(16), None, 0, None) == -3
    # adjoints: FP64 only
    tr.kind = lw.TRAJ_SAMPLES
    p = ctypes.c_void_p(256)
    tr.r = tr.beta = tr.beta_dot = p
    gr.x_det = p
    # geometry flags: LW_ACCUMULATE and LW_CULL are accepted, other bits are not (checked
    # before the NULL trace, which is reported next)
    for flags in (lw.ACCUMULATE, lw.CULL, lw.CULL | lw.ACCUMULATE | lw.GEOM["farfield"]):
        assert lib.lw_deposit_td(ctypes.byref(tr), ctypes.byref(gr), 0, 1, flags, None, None, None, 0, None) == -1
        assert b"E is NULL" in lib.lw_last_error()
    assert lib.lw_deposit_td(ctypes.byref(tr), ctypes.byref(gr), 0, 1, 1 << 10, None, None, None, 0, None) == -1
    assert b"unknown geometry" in lib.lw_last_error()
    assert lib.lw_deposit_td_bwd(ctypes.byref(tr), ctypes.byref(gr), 1, 1, 0, p, p, p, p, None, 0, None) == -6
    assert lib.lw_direct_fd_bwd(ctypes.byref(tr), ctypes.byref(gr), p, 4, 1, 1, 0, p, p, p, p, None, 0, None) == -6
    assert lib.lw_direct_fd_bwd(ctypes.byref(tr), ctypes.byref(gr), p, 4, 0, 1, 0, p, p, p, p, None, 0, None) == -4
    tb = lw.Traj()
    tb.kind = lw.TRAJ_SAMPLES
    tb.n_particles = 1
    tb.n_samples = 10
    tb.dt = 1e-18
    assert lib.lw_trajectory_boris_bwd(ctypes.byref(tb), p, p, p, p, p, None) == -1  # kind must be BORIS
    # traj->span: 0 for stored samples and for every call but lw_deposit_td, 0 or >= 2 there
    tr.span = 5
    assert lib.lw_deposit_td(ctypes.byref(tr), ctypes.byref(gr), 0, 1, 0, p, None, None, 0, None) == -1
    assert b"span" in lib.lw_last_error()
    tr.span = 0
    tb.kind = lw.TRAJ_BORIS
    tb.laser.lam, tb.laser.n_cycles = 1e-6, 10.0
    tb.init = p
    for span in (1, -3):
        tb.span = span
        assert lib.lw_deposit_td(ctypes.byref(tb), ctypes.byref(gr), 0, 1, 0, p, None, None, 0, None) == -1
        assert b"span" in lib.lw_last_error()
    tb.span = 2  # accepted; the missing workspace is reported next
    assert lib.lw_deposit_td(ctypes.byref(tb), ctypes.byref(gr), 0, 1, 0, p, None, None, 0, None) == -4
    assert lib.lw_trajectory_boris(ctypes.byref(tb), p, p, p, None) == -1
    assert b"span" in lib.lw_last_error()
    assert lib.lw_trajectory_boris_bwd(ctypes.byref(tb), p, p, p, p, p, None) == -1
    assert b"span" in lib.lw_last_error()
    # the deposit adjoint takes spans too: span 2 passes, the missing workspace is reported
    assert lib.lw_deposit_td_bwd_boris(ctypes.byref(tb), ctypes.byref(gr), 0, 1, 0, p, p, p, None, 0, None) == -4
    # lw_deposit_td_det: an accumulator buffer of the documented size, no accumulate or cull flag
    need = lw.workspace_bytes(lw.WS_DEPOSIT_DET_ACC, gr.n_pix, gr.n_obs, "fp64")
    det = lib.lw_deposit_td_det
    assert det(ctypes.byref(tr), ctypes.byref(gr), 1, 0, p, None, None, 0, p, 1 << 20, None) == -4
    assert b"no accumulator" in lib.lw_last_error()
    assert det(ctypes.byref(tr), ctypes.byref(gr), 1, 0, p, None, p, need - 8, p, 1 << 20, None) == -4
    assert det(ctypes.byref(tr), ctypes.byref(gr), 1, 0, p, None, ctypes.c_void_p(264), need, p, 1 << 20, None) == -3
    for flags in (lw.ACCUMULATE, lw.CULL):
        assert det(ctypes.byref(tr), ctypes.byref(gr), 1, flags, p, None, p, need, p, 1 << 20, None) == -1
        assert b"not taken" in lib.lw_last_error()
    assert det(None, ctypes.byref(gr), 1, 0, p, None, p, need, p, 1 << 20, None) == -1
    tb.span = 1
    assert lib.lw_deposit_td_bwd_boris(ctypes.byref(tb), ctypes.byref(gr), 0, 1, 0, p, p, p, None, 0, None) == -1
    assert lib.lw_version().startswith(b"liblw")
