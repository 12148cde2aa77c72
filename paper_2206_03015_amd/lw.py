"""Thin ctypes binding of liblw.so (include/lw.h).

Argument marshalling only: tensors are passed as device pointers, the stream is
torch's current stream, and workspaces are allocated with torch.  Every step of
the hot path runs inside the library's HIP kernels.  There is no fallback: if
liblw.so is missing or fails to load, ``load()`` raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime liblw.so binds to)

HERE = os.path.dirname(os.path.abspath(__file__))
# LW_LIBRARY selects another build of the same library (e.g. one with host-side sanitizers).
LIB_PATH = os.environ.get("LW_LIBRARY") or os.path.join(HERE, "liblw.so")

LW_OK = 0
PREC = {"fp64": 0, "mixed": 1}
FIELD_ACCEL = 1
FIELD_VELOCITY = 2
GEOM = {"exact": 0, "farfield": 1}
ACCUMULATE = 1 << 8
CULL = 1 << 9
TRAJ_SAMPLES = 0
TRAJ_BORIS = 1
WS_DEPOSIT, WS_FFT, WS_DIRECT_FD, WS_DEPOSIT_BWD, WS_FFT_BWD, WS_DIRECT_FD_BWD = 1, 2, 3, 4, 5, 6
WS_DEPOSIT_BORIS, WS_DEPOSIT_BWD_BORIS, WS_DEPOSIT_DET_ACC = 7, 8, 9
KERNEL_DEPOSIT, KERNEL_DEPOSIT_BWD, KERNEL_BORIS_TANGENT = 1, 2, 3

c_d = ctypes.c_double
c_i64 = ctypes.c_int64
c_vp = ctypes.c_void_p


class Laser(ctypes.Structure):
    _fields_ = [("a0", c_d), ("lam", c_d), ("w0", c_d), ("n_cycles", c_d)]


class Traj(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("span", ctypes.c_int32), ("n_particles", c_i64),
                ("n_samples", c_i64), ("t_start", c_d), ("dt", c_d), ("r", c_vp), ("beta", c_vp),
                ("beta_dot", c_vp), ("init", c_vp), ("laser", Laser), ("charge", c_vp)]


class Grid(ctypes.Structure):
    _fields_ = [("n_pix", c_i64), ("x_det", c_vp), ("t0", c_d), ("dt_obs", c_d), ("n_obs", c_i64)]


class LWError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"liblw status {status}: {msg}")
        self.status = status


# every function declared in include/lw.h, with its ctypes signature
_SIGS = {
    "lw_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int, c_i64, c_i64, ctypes.c_int]),
    "lw_deposit_td": (ctypes.c_int, [ctypes.POINTER(Traj), ctypes.POINTER(Grid), ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp]),
    "lw_spectrum_fft": (ctypes.c_int, [c_vp, c_i64, c_i64, c_d, ctypes.c_int, c_vp, c_vp, ctypes.c_size_t, c_vp]),
    "lw_spectrum_fft_noalloc": (ctypes.c_int, [c_vp, c_i64, c_i64, c_d, ctypes.c_int, c_vp, c_vp]),
    "lw_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "lw_direct_fd": (ctypes.c_int, [ctypes.POINTER(Traj), ctypes.POINTER(Grid), c_vp, c_i64, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, c_vp, c_vp, ctypes.c_size_t, c_vp]),
    "lw_trajectory_boris": (ctypes.c_int, [ctypes.POINTER(Traj), c_vp, c_vp, c_vp, c_vp]),
    "lw_trajectory_boris_bwd": (ctypes.c_int, [ctypes.POINTER(Traj), c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    "lw_spectrum_fft_bwd": (ctypes.c_int, [c_vp, c_vp, c_i64, c_i64, c_d, ctypes.c_int, c_vp, c_vp,
                                           ctypes.c_size_t, c_vp]),
    "lw_deposit_td_bwd": (ctypes.c_int, [ctypes.POINTER(Traj), ctypes.POINTER(Grid), ctypes.c_int, ctypes.c_int,
                                         ctypes.c_int, c_vp, c_vp, c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp]),
    "lw_deposit_td_det": (ctypes.c_int, [ctypes.POINTER(Traj), ctypes.POINTER(Grid), ctypes.c_int, ctypes.c_int,
                                         c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp, ctypes.c_size_t, c_vp]),
    "lw_deposit_td_bwd_boris": (ctypes.c_int, [ctypes.POINTER(Traj), ctypes.POINTER(Grid), ctypes.c_int, ctypes.c_int,
                                               ctypes.c_int, c_vp, c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp]),
    "lw_direct_fd_bwd": (ctypes.c_int, [ctypes.POINTER(Traj), ctypes.POINTER(Grid), c_vp, c_i64, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int, c_vp, c_vp, c_vp, c_vp, c_vp, ctypes.c_size_t,
                                        c_vp]),
    "lw_timing_enable": (ctypes.c_int, [ctypes.c_int]),
    "lw_timing_read": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(c_d), ctypes.POINTER(c_i64)]),
    "lw_last_error": (ctypes.c_char_p, []),
    "lw_version": (ctypes.c_char_p, []),
}

_lib = None


def load():
    """Load liblw.so (raises if it is missing: there is no other implementation)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing; build it with `python -m paper_2206_03015_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _check(status):
    if status != LW_OK:
        raise LWError(status, load().lw_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, dtype, shape=None, name="tensor"):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def timing_enable(on=True):
    """lw_timing_enable: record HIP events around every later launch of the timed kernels."""
    _check(load().lw_timing_enable(1 if on else 0))


def timing_read(which=KERNEL_DEPOSIT):
    """lw_timing_read: (summed milliseconds, launches) of the kernel since the last read."""
    ms, n = c_d(0.0), c_i64(0)
    _check(load().lw_timing_read(int(which), ctypes.byref(ms), ctypes.byref(n)))
    return float(ms.value), int(n.value)


def workspace_bytes(which, n_a, n_b, prec="mixed"):
    return int(load().lw_workspace_bytes(which, int(n_a), int(n_b), PREC[prec]))


def _workspace(nbytes, device):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def make_traj(r, beta, beta_dot, t_start, dt, charge=None):
    """Traj struct over sample tensors [n_p][n_samples][3] (float64, device)."""
    n_p, ns = int(r.shape[0]), int(r.shape[1])
    for t, nm in ((r, "r"), (beta, "beta"), (beta_dot, "beta_dot")):
        _need(t, torch.float64, (n_p, ns, 3), nm)
    if charge is not None:
        _need(charge, torch.float64, (n_p,), "charge")
    tr = Traj()
    tr.kind = TRAJ_SAMPLES
    tr.span = 0
    tr.n_particles = n_p
    tr.n_samples = ns
    tr.t_start = float(t_start)
    tr.dt = float(dt)
    tr.r, tr.beta, tr.beta_dot = (c_vp(t.data_ptr()) for t in (r, beta, beta_dot))
    tr.init = None
    tr.charge = None if charge is None else c_vp(charge.data_ptr())
    return tr


def make_grid(x_det, t0, dt_obs, n_obs):
    _need(x_det, torch.float64, (int(x_det.shape[0]), 3), "x_det")
    g = Grid()
    g.n_pix = int(x_det.shape[0])
    g.x_det = c_vp(x_det.data_ptr())
    g.t0 = float(t0)
    g.dt_obs = float(dt_obs)
    g.n_obs = int(n_obs)
    return g


def deposit_td(r, beta, beta_dot, t_start, dt, x_det, t0, dt_obs, n_obs, prec="mixed", field_mask=FIELD_ACCEL,
               geom="exact", charge=None, out=None, accumulate=False, diag=None, ws=None, cull=False):
    """lw_deposit_td.  Returns (E [n_pix][3][n_obs], diag int64[4])."""
    lib = load()
    tr = make_traj(r, beta, beta_dot, t_start, dt, charge)
    gr = make_grid(x_det, t0, dt_obs, n_obs)
    dtype = torch.float64 if prec == "fp64" else torch.float32
    if out is None:
        out = torch.empty((gr.n_pix, 3, int(n_obs)), dtype=dtype, device=r.device)
    _need(out, dtype, (gr.n_pix, 3, int(n_obs)), "E")
    if diag is None:
        diag = torch.zeros(4, dtype=torch.int64, device=r.device)
    need = workspace_bytes(WS_DEPOSIT, tr.n_particles, tr.n_samples, prec)
    if ws is None:
        ws = _workspace(need, r.device)
    flags = GEOM[geom] | (ACCUMULATE if accumulate else 0) | (CULL if cull else 0)
    _check(lib.lw_deposit_td(ctypes.byref(tr), ctypes.byref(gr), PREC[prec], int(field_mask), flags, _ptr(out),
                             _ptr(diag), _ptr(ws), ws.numel(), _stream()))
    return out, diag


def _deposit_det(tr, gr, device, ws_need, field_mask, geom, out, diag, ws, acc):
    lib = load()
    if out is None:
        out = torch.empty((gr.n_pix, 3, gr.n_obs), dtype=torch.float64, device=device)
    _need(out, torch.float64, (gr.n_pix, 3, gr.n_obs), "E")
    if diag is None:
        diag = torch.zeros(4, dtype=torch.int64, device=device)
    if ws is None:
        ws = _workspace(ws_need, device)
    if acc is None:
        acc = _workspace(workspace_bytes(WS_DEPOSIT_DET_ACC, gr.n_pix, gr.n_obs, "fp64"), device)
    _check(lib.lw_deposit_td_det(ctypes.byref(tr), ctypes.byref(gr), int(field_mask), GEOM[geom], _ptr(out),
                                 _ptr(diag), _ptr(acc), acc.numel(), _ptr(ws), ws.numel(), _stream()))
    return out, diag


def deposit_td_det(r, beta, beta_dot, t_start, dt, x_det, t0, dt_obs, n_obs, field_mask=FIELD_ACCEL, geom="exact",
                   charge=None, out=None, diag=None, ws=None, acc=None):
    """lw_deposit_td_det: the FP64 deposit, the same bits on every run and for any particle order.
    Returns (E [n_pix][3][n_obs] float64, diag int64[4])."""
    tr = make_traj(r, beta, beta_dot, t_start, dt, charge)
    gr = make_grid(x_det, t0, dt_obs, n_obs)
    need = workspace_bytes(WS_DEPOSIT, tr.n_particles, tr.n_samples, "fp64")
    return _deposit_det(tr, gr, r.device, need, field_mask, geom, out, diag, ws, acc)


def deposit_td_det_boris(init, n_samples, t_start, dt, a0, lam, w0, n_cycles, x_det, t0, dt_obs, n_obs,
                         field_mask=FIELD_ACCEL, geom="exact", charge=None, out=None, diag=None, ws=None, acc=None,
                         span=0):
    """lw_deposit_td_det with LW_TRAJ_BORIS (trajectories pushed inside the call, twice)."""
    tr = make_boris_traj(init, n_samples, t_start, dt, a0, lam, w0, n_cycles)
    tr.span = int(span)
    if charge is not None:
        _need(charge, torch.float64, (int(init.shape[0]),), "charge")
        tr.charge = c_vp(charge.data_ptr())
    gr = make_grid(x_det, t0, dt_obs, n_obs)
    need = workspace_bytes(WS_DEPOSIT_BORIS, tr.n_particles, tr.n_samples, "fp64")
    return _deposit_det(tr, gr, init.device, need, field_mask, geom, out, diag, ws, acc)


def spectrum_fft(E, dt_obs, prec=None, out=None, ws=None):
    """lw_spectrum_fft.  E [n_pix][3][n_obs] float32 (mixed) or float64 (fp64)."""
    lib = load()
    if prec is None:
        prec = "fp64" if E.dtype == torch.float64 else "mixed"
    dtype = torch.float64 if prec == "fp64" else torch.float32
    n_pix, _, n_obs = (int(v) for v in E.shape)
    _need(E, dtype, (n_pix, 3, n_obs), "E")
    if out is None:
        out = torch.empty((n_pix, n_obs // 2 + 1), dtype=dtype, device=E.device)
    _need(out, dtype, (n_pix, n_obs // 2 + 1), "S")
    if ws is None:
        ws = _workspace(workspace_bytes(WS_FFT, n_pix, n_obs, prec), E.device)
    _check(lib.lw_spectrum_fft(_ptr(E), n_pix, n_obs, float(dt_obs), PREC[prec], _ptr(out), _ptr(ws), ws.numel(),
                               _stream()))
    return out


def spectrum_fft_noalloc(E, dt_obs, out, prec=None):
    """lw_spectrum_fft_noalloc: the spectrum of E into the caller's S (`out`), with the library's
    static scratch instead of a workspace (nothing is allocated)."""
    lib = load()
    if prec is None:
        prec = "fp64" if E.dtype == torch.float64 else "mixed"
    dtype = torch.float64 if prec == "fp64" else torch.float32
    n_pix, _, n_obs = (int(v) for v in E.shape)
    _need(E, dtype, (n_pix, 3, n_obs), "E")
    _need(out, dtype, (n_pix, n_obs // 2 + 1), "S")
    _check(lib.lw_spectrum_fft_noalloc(_ptr(E), n_pix, n_obs, float(dt_obs), PREC[prec], _ptr(out), _stream()))
    return out


def noalloc_scratch_bytes():
    return int(load().lw_noalloc_scratch_bytes())


def direct_fd(r, beta, beta_dot, t_start, dt, x_det, t0, omega, prec="mixed", field_mask=FIELD_ACCEL,
              geom="exact", charge=None, out=None, ws=None):
    """lw_direct_fd.  Returns S [n_pix][n_omega] float64."""
    lib = load()
    tr = make_traj(r, beta, beta_dot, t_start, dt, charge)
    gr = make_grid(x_det, t0, 1.0, 1)
    _need(omega, torch.float64, (int(omega.shape[0]),), "omega")
    n_w = int(omega.shape[0])
    if out is None:
        out = torch.empty((gr.n_pix, n_w), dtype=torch.float64, device=r.device)
    _need(out, torch.float64, (gr.n_pix, n_w), "S")
    if ws is None:
        ws = _workspace(workspace_bytes(WS_DIRECT_FD, gr.n_pix, n_w, prec), r.device)
    _check(lib.lw_direct_fd(ctypes.byref(tr), ctypes.byref(gr), _ptr(omega), n_w, PREC[prec], int(field_mask),
                            GEOM[geom], _ptr(out), _ptr(ws), ws.numel(), _stream()))
    return out


def make_boris_traj(init, n_samples, t_start, dt, a0, lam, w0, n_cycles):
    """Traj struct of kind LW_TRAJ_BORIS over init [n_p][6] (float64, device)."""
    n_p = int(init.shape[0])
    _need(init, torch.float64, (n_p, 6), "init")
    tr = Traj()
    tr.kind = TRAJ_BORIS
    tr.span = 0
    tr.n_particles = n_p
    tr.n_samples = int(n_samples)
    tr.t_start = float(t_start)
    tr.dt = float(dt)
    tr.init = c_vp(init.data_ptr())
    tr.laser = Laser(float(a0), float(lam), float(w0), float(n_cycles))
    return tr


def trajectory_boris(init, n_samples, t_start, dt, a0, lam, w0, n_cycles, out=None):
    """lw_trajectory_boris.  init [n_p][6] float64 device.  Returns (r, beta, beta_dot)."""
    lib = load()
    n_p = int(init.shape[0])
    tr = make_boris_traj(init, n_samples, t_start, dt, a0, lam, w0, n_cycles)
    if out is None:
        out = tuple(torch.empty((n_p, int(n_samples), 3), dtype=torch.float64, device=init.device) for _ in range(3))
    r, b, bd = out
    _check(lib.lw_trajectory_boris(ctypes.byref(tr), _ptr(r), _ptr(b), _ptr(bd), _stream()))
    return r, b, bd


def trajectory_boris_bwd(init, n_samples, t_start, dt, a0, lam, w0, n_cycles, g_r, g_beta, g_beta_dot):
    """lw_trajectory_boris_bwd.  Returns (grad_init [n_p][6], grad_a0 [n_p]) (float64, device)."""
    lib = load()
    n_p = int(init.shape[0])
    tr = make_boris_traj(init, n_samples, t_start, dt, a0, lam, w0, n_cycles)
    for t, nm in ((g_r, "g_r"), (g_beta, "g_beta"), (g_beta_dot, "g_beta_dot")):
        _need(t, torch.float64, (n_p, int(n_samples), 3), nm)
    grad_init = torch.empty((n_p, 6), dtype=torch.float64, device=init.device)
    grad_a0 = torch.empty((n_p,), dtype=torch.float64, device=init.device)
    _check(lib.lw_trajectory_boris_bwd(ctypes.byref(tr), _ptr(g_r), _ptr(g_beta), _ptr(g_beta_dot), _ptr(grad_init),
                                       _ptr(grad_a0), _stream()))
    return grad_init, grad_a0


def spectrum_fft_bwd(E, dS, dt_obs, prec=None, out=None, ws=None):
    """lw_spectrum_fft_bwd: dJ/dE [n_pix][3][n_obs] from dJ/dS [n_pix][n_obs/2+1] and the trace E."""
    lib = load()
    if prec is None:
        prec = "fp64" if E.dtype == torch.float64 else "mixed"
    dtype = torch.float64 if prec == "fp64" else torch.float32
    n_pix, _, n_obs = (int(v) for v in E.shape)
    _need(E, dtype, (n_pix, 3, n_obs), "E")
    _need(dS, dtype, (n_pix, n_obs // 2 + 1), "dS")
    if out is None:
        out = torch.empty_like(E)
    _need(out, dtype, (n_pix, 3, n_obs), "dE")
    if ws is None:
        ws = _workspace(workspace_bytes(WS_FFT_BWD, n_pix, n_obs, prec), E.device)
    _check(lib.lw_spectrum_fft_bwd(_ptr(E), _ptr(dS), n_pix, n_obs, float(dt_obs), PREC[prec], _ptr(out), _ptr(ws),
                                   ws.numel(), _stream()))
    return out


def deposit_td_bwd(r, beta, beta_dot, t_start, dt, x_det, t0, dt_obs, n_obs, dE, field_mask=FIELD_ACCEL,
                   geom="exact", charge=None, out=None):
    """lw_deposit_td_bwd (FP64): adds dJ/d(r, beta, beta_dot) into `out` (zeros if None) and returns it."""
    lib = load()
    tr = make_traj(r, beta, beta_dot, t_start, dt, charge)
    gr = make_grid(x_det, t0, dt_obs, n_obs)
    _need(dE, torch.float64, (gr.n_pix, 3, int(n_obs)), "dE")
    if out is None:
        out = tuple(torch.zeros_like(r) for _ in range(3))
    d_r, d_b, d_bd = out
    for t, nm in ((d_r, "d_r"), (d_b, "d_beta"), (d_bd, "d_beta_dot")):
        _need(t, torch.float64, tuple(r.shape), nm)
    ws = _workspace(workspace_bytes(WS_DEPOSIT_BWD, tr.n_particles, tr.n_samples, "fp64"), r.device)
    _check(lib.lw_deposit_td_bwd(ctypes.byref(tr), ctypes.byref(gr), PREC["fp64"], int(field_mask), GEOM[geom],
                                 _ptr(dE), _ptr(d_r), _ptr(d_b), _ptr(d_bd), _ptr(ws), ws.numel(), _stream()))
    return d_r, d_b, d_bd


def direct_fd_bwd(r, beta, beta_dot, t_start, dt, x_det, t0, omega, dS, field_mask=FIELD_ACCEL, geom="exact",
                  charge=None, out=None, ws=None):
    """lw_direct_fd_bwd (FP64): adds dJ/d(r, beta, beta_dot) for J = sum(dS * S_FD) into `out` (zeros if None)."""
    lib = load()
    tr = make_traj(r, beta, beta_dot, t_start, dt, charge)
    gr = make_grid(x_det, t0, 1.0, 1)
    n_w = int(omega.shape[0])
    _need(omega, torch.float64, (n_w,), "omega")
    _need(dS, torch.float64, (gr.n_pix, n_w), "dS")
    if out is None:
        out = tuple(torch.zeros_like(r) for _ in range(3))
    d_r, d_b, d_bd = out
    for t, nm in ((d_r, "d_r"), (d_b, "d_beta"), (d_bd, "d_beta_dot")):
        _need(t, torch.float64, tuple(r.shape), nm)
    if ws is None:
        ws = _workspace(workspace_bytes(WS_DIRECT_FD_BWD, gr.n_pix, n_w, "fp64"), r.device)
    _check(lib.lw_direct_fd_bwd(ctypes.byref(tr), ctypes.byref(gr), _ptr(omega), n_w, PREC["fp64"], int(field_mask),
                                GEOM[geom], _ptr(dS), _ptr(d_r), _ptr(d_b), _ptr(d_bd), _ptr(ws), ws.numel(),
                                _stream()))
    return d_r, d_b, d_bd


def deposit_td_boris(init, n_samples, t_start, dt, a0, lam, w0, n_cycles, x_det, t0, dt_obs, n_obs, prec="mixed",
                     field_mask=FIELD_ACCEL, geom="exact", charge=None, out=None, accumulate=False, diag=None, ws=None,
                     cull=False, span=0):
    """lw_deposit_td with LW_TRAJ_BORIS: trajectories recomputed inside the call from init [n_p][6],
    a batch of particles over a span of samples at a time (span=0: chosen from the workspace).
    Returns (E, diag)."""
    lib = load()
    tr = make_boris_traj(init, n_samples, t_start, dt, a0, lam, w0, n_cycles)
    tr.span = int(span)
    if charge is not None:
        _need(charge, torch.float64, (int(init.shape[0]),), "charge")
        tr.charge = c_vp(charge.data_ptr())
    else:
        tr.charge = None
    gr = make_grid(x_det, t0, dt_obs, n_obs)
    dtype = torch.float64 if prec == "fp64" else torch.float32
    if out is None:
        out = torch.empty((gr.n_pix, 3, int(n_obs)), dtype=dtype, device=init.device)
    _need(out, dtype, (gr.n_pix, 3, int(n_obs)), "E")
    if diag is None:
        diag = torch.zeros(4, dtype=torch.int64, device=init.device)
    if ws is None:
        ws = _workspace(workspace_bytes(WS_DEPOSIT_BORIS, tr.n_particles, tr.n_samples, prec), init.device)
    flags = GEOM[geom] | (ACCUMULATE if accumulate else 0) | (CULL if cull else 0)
    _check(lib.lw_deposit_td(ctypes.byref(tr), ctypes.byref(gr), PREC[prec], int(field_mask), flags, _ptr(out),
                             _ptr(diag), _ptr(ws), ws.numel(), _stream()))
    return out, diag


def deposit_td_bwd_boris(init, n_samples, t_start, dt, a0, lam, w0, n_cycles, x_det, t0, dt_obs, n_obs, dE,
                         field_mask=FIELD_ACCEL, geom="exact", charge=None, ws=None, span=0):
    """lw_deposit_td_bwd_boris (FP64), a batch of particles over a span of samples at a time
    (span=0: chosen from the workspace): returns (grad_init [n_p][6], grad_a0 [n_p])."""
    lib = load()
    n_p = int(init.shape[0])
    tr = make_boris_traj(init, n_samples, t_start, dt, a0, lam, w0, n_cycles)
    tr.span = int(span)
    if charge is not None:
        _need(charge, torch.float64, (n_p,), "charge")
        tr.charge = c_vp(charge.data_ptr())
    else:
        tr.charge = None
    gr = make_grid(x_det, t0, dt_obs, n_obs)
    _need(dE, torch.float64, (gr.n_pix, 3, int(n_obs)), "dE")
    grad_init = torch.empty((n_p, 6), dtype=torch.float64, device=init.device)
    grad_a0 = torch.empty((n_p,), dtype=torch.float64, device=init.device)
    if ws is None:
        ws = _workspace(workspace_bytes(WS_DEPOSIT_BWD_BORIS, n_p, tr.n_samples, "fp64"), init.device)
    _check(lib.lw_deposit_td_bwd_boris(ctypes.byref(tr), ctypes.byref(gr), PREC["fp64"], int(field_mask), GEOM[geom],
                                       _ptr(dE), _ptr(grad_init), _ptr(grad_a0), _ptr(ws), ws.numel(), _stream()))
    return grad_init, grad_a0
