"""Plain FP64 CPU oracle for the time-domain Lienard-Wiechert spectrum method
(Kan et al., arXiv:2206.03015).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the HIP library and never imports it; the product path never
imports this package.

Functions and what pins each one (tests named in brackets):

* ``arrival_tau`` -- arrival times in grid units, formed in extended precision (the
  large terms t_i/dt_obs and n.r/(c dt_obs) cancel).  Pinned by: 50-digit evaluations of
  the definition on the same double inputs at the sizes of the largest workloads
  (|error| <= 1e-11 grid units) [test_oracle_eval.py].
* ``eval_one`` / ``eval_samples`` -- per-sample arrival time and LW field
  (Eqs. lw_fields_retarded, advanced_condition, far_efield, far_adv).
  Pinned by: Coulomb field of a charge at rest; the closed-form field of a
  uniformly moving charge; the far-field integrand identity E*kappa = q A /(4 pi
  eps0 c D) (Eq. const_phase_drop); exact -> far-field limit; arrival time
  against a 50-digit evaluation of t + |x - r|/c  [test_oracle_eval.py].
* ``interp_deposit`` / ``deposit_td`` -- Algorithm 2 interpolation.
  Pinned by: partition of unity, exactness on fields linear in arrival time,
  integer hit counts, a hand-computed two-sample case, the counted skips
  [test_oracle_deposit.py].
* ``spectrum`` -- |E(w)|^2 on the FFT bins (Eq. efield_xfrom).  Pinned by: an
  O(N^2) brute-force DFT, Parseval, a single on-bin cosine
  [test_oracle_spectrum.py].
* ``direct_fd`` -- direct frequency-domain sum (Eq. inty_dft, Algorithm 1).
  Pinned by: single-sample closed form, the paper's Eq. inty_dft prefactor,
  agreement with deposit+spectrum converging at second order as the steps
  shrink [test_oracle_fd.py].
* ``boris`` -- FP64 Boris trajectories.  Pinned by: second-order convergence to
  the analytic plane-wave trajectory; field-free straight line
  [test_oracle_boris.py].
* ``planewave_trajectory`` -- analytic electron motion in a plane-wave pulse
  (conserved canonical momentum and light-front momentum).  Pinned by: the
  equations of motion checked by finite differences; conserved quantities
  [test_oracle_boris.py]; the ICS line position, on axis and off axis
  [test_oracle_physics.py].
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .spectrum import spectrum, spectrum_bruteforce  # noqa: F401
from .trajectory import planewave_trajectory  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lw_oracle.c")
_LIB = os.path.join(_HERE, "liblw_oracle.so")
# LW_ORACLE_LIBRARY loads another build of lw_oracle.c (the sanitized one from build_sanitized()).
_LIB_OVERRIDE = os.environ.get("LW_ORACLE_LIBRARY")

C_LIGHT = 299792458.0
Q_E = 1.602176634e-19
EPS0 = 8.8541878128e-12
M_E = 9.1093837015e-31

FIELD_ACCEL = 1
FIELD_VELOCITY = 2
GEOM_EXACT = 0
GEOM_FARFIELD = 1


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, no fast-math, OpenMP over observers)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", _SRC, "-o", tmp, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


def build_sanitized(out: str) -> str:
    """The same oracle with AddressSanitizer + UndefinedBehaviorSanitizer (any report aborts).
    A process that loads it needs gcc's libasan preloaded (``asan_runtime()``)."""
    subprocess.check_call(
        ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
         _SRC, "-o", out, "-lm"]
    )
    return out


def asan_runtime() -> str:
    return subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64 = ctypes.c_int64
        d = ctypes.c_double
        L.orc_eval.argtypes = [dp, dp, dp, dp, d, ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.orc_eval.restype = None
        L.orc_interp_deposit.argtypes = [i64, dp, dp, ctypes.c_void_p, i64, dp, ctypes.POINTER(i64)]
        L.orc_deposit_td.argtypes = [i64, i64, d, d, dp, dp, dp, ctypes.c_void_p, i64, dp, d, d, i64,
                                     ctypes.c_int, ctypes.c_int, dp, ctypes.POINTER(i64)]
        L.orc_eval_samples.argtypes = [i64, i64, d, d, dp, dp, dp, ctypes.c_void_p, i64, dp, d, d,
                                       ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_void_p]
        L.orc_direct_fd.argtypes = [i64, i64, d, d, dp, dp, dp, ctypes.c_void_p, i64, dp, d, dp, i64,
                                    ctypes.c_int, ctypes.c_int, dp]
        L.orc_boris.argtypes = [i64, i64, d, d, dp, d, d, d, d, dp, dp, dp]
        L.orc_arrival_tau.argtypes = [i64, dp, dp, ctypes.c_void_p, d, d, d, d, ctypes.c_int, dp]
        L.orc_arrival_tau.restype = None
        L.orc_laser_fields.argtypes = [i64, dp, dp, d, d, d, d, dp, dp]
        L.orc_laser_fields.restype = None
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def eval_one(x, r, beta, beta_dot, q=-Q_E, field_mask=FIELD_ACCEL, geom=GEOM_EXACT):
    """Arrival-time shift tt (s, relative to t + |x|/c), field E (V/m), kappa = 1 - n.beta."""
    x, r, b, bd = (_f64(v, (3,)) for v in (x, r, beta, beta_dot))
    tt = np.zeros(1)
    E = np.zeros(3)
    kap = np.zeros(1)
    lib().orc_eval(_p(x), _p(r), _p(b), _p(bd), float(q), int(field_mask), int(geom), _p(tt), _p(E), _p(kap))
    return tt[0], E, kap[0]


def arrival_tau(x, r, i, t_start, dt, t0, dt_obs, geom=GEOM_EXACT):
    """Arrival times (grid units) of single samples: sample i[j] emitted from r[j] seen at x[j]
    (the extended-precision evaluation that deposit_td, eval_samples and direct_fd use)."""
    x = _f64(x).reshape(-1, 3)
    r = _f64(r).reshape(-1, 3)
    i = np.ascontiguousarray(np.asarray(i, dtype=np.int64).reshape(-1))
    n = x.shape[0]
    tau = np.empty(n)
    lib().orc_arrival_tau(n, _p(x), _p(r), i.ctypes.data, float(t_start), float(dt), float(t0), float(dt_obs),
                          int(geom), _p(tau))
    return tau


def _traj_args(r, beta, beta_dot, charge):
    r = _f64(r)
    n_p, n_s = r.shape[0], r.shape[1]
    r = r.reshape(n_p, n_s, 3)
    beta = _f64(beta, (n_p, n_s, 3))
    beta_dot = _f64(beta_dot, (n_p, n_s, 3))
    ch = None if charge is None else _f64(charge, (n_p,))
    return n_p, n_s, r, beta, beta_dot, ch


def eval_samples(t_start, dt, r, beta, beta_dot, x_det, t0, dt_obs, charge=None, field_mask=FIELD_ACCEL,
                 geom=GEOM_EXACT):
    """tau[n_pix][n_p][n_samples] (grid units), E[...][3], kappa[...]; NaN for unusable samples."""
    n_p, n_s, r, beta, beta_dot, ch = _traj_args(r, beta, beta_dot, charge)
    x_det = _f64(x_det).reshape(-1, 3)
    n_pix = x_det.shape[0]
    tau = np.empty((n_pix, n_p, n_s))
    E = np.empty((n_pix, n_p, n_s, 3))
    kap = np.empty((n_pix, n_p, n_s))
    lib().orc_eval_samples(n_p, n_s, float(t_start), float(dt), _p(r), _p(beta), _p(beta_dot),
                           None if ch is None else ch.ctypes.data, n_pix, _p(x_det), float(t0), float(dt_obs),
                           int(field_mask), int(geom), _p(tau), _p(E), kap.ctypes.data)
    return tau, E, kap


def interp_deposit(tau, E, n_obs, ok=None):
    """Algorithm 2's interpolation step alone for one sample stream.

    tau: [n] grid units, E: [n][3], ok: [n] bool (default: finite tau).
    Returns (trace [3][n_obs], diag[4])."""
    tau = _f64(tau).reshape(-1)
    n = tau.shape[0]
    E = _f64(E, (n, 3))
    okb = np.isfinite(tau) if ok is None else np.asarray(ok, dtype=bool)
    okb = np.ascontiguousarray(okb.astype(np.uint8))
    out = np.zeros((3, int(n_obs)))
    diag = np.zeros(4, dtype=np.int64)
    rc = lib().orc_interp_deposit(n, _p(tau), _p(E), okb.ctypes.data, int(n_obs), _p(out),
                                  diag.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise ValueError("orc_interp_deposit rejected its arguments")
    return out, diag


def deposit_td(t_start, dt, r, beta, beta_dot, x_det, t0, dt_obs, n_obs, charge=None, field_mask=FIELD_ACCEL,
               geom=GEOM_EXACT):
    """Time-domain trace E_tot[n_pix][3][n_obs] (FP64) and diag[4] (Algorithm 2)."""
    n_p, n_s, r, beta, beta_dot, ch = _traj_args(r, beta, beta_dot, charge)
    x_det = _f64(x_det).reshape(-1, 3)
    n_pix = x_det.shape[0]
    out = np.empty((n_pix, 3, int(n_obs)))
    diag = np.zeros(4, dtype=np.int64)
    rc = lib().orc_deposit_td(n_p, n_s, float(t_start), float(dt), _p(r), _p(beta), _p(beta_dot),
                              None if ch is None else ch.ctypes.data, n_pix, _p(x_det), float(t0), float(dt_obs),
                              int(n_obs), int(field_mask), int(geom), _p(out),
                              diag.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise ValueError(f"orc_deposit_td failed ({rc})")
    return out, diag


def direct_fd(t_start, dt, r, beta, beta_dot, x_det, t0, omega, charge=None, field_mask=FIELD_ACCEL,
              geom=GEOM_EXACT):
    """Direct frequency-domain |E(w)|^2, S[n_pix][n_omega] (Eq. inty_dft generalised)."""
    n_p, n_s, r, beta, beta_dot, ch = _traj_args(r, beta, beta_dot, charge)
    x_det = _f64(x_det).reshape(-1, 3)
    n_pix = x_det.shape[0]
    omega = _f64(omega).reshape(-1)
    S = np.empty((n_pix, omega.shape[0]))
    rc = lib().orc_direct_fd(n_p, n_s, float(t_start), float(dt), _p(r), _p(beta), _p(beta_dot),
                             None if ch is None else ch.ctypes.data, n_pix, _p(x_det), float(t0), _p(omega),
                             omega.shape[0], int(field_mask), int(geom), _p(S))
    if rc != 0:
        raise MemoryError("orc_direct_fd could not allocate")
    return S


def boris(init, n_samples, t_start, dt, a0, lam, w0, n_cycles):
    """FP64 Boris trajectories of electrons: r, beta, beta_dot [n_p][n_samples][3]."""
    init = _f64(init).reshape(-1, 6)
    n_p = init.shape[0]
    r = np.empty((n_p, int(n_samples), 3))
    b = np.empty_like(r)
    bd = np.empty_like(r)
    lib().orc_boris(n_p, int(n_samples), float(t_start), float(dt), _p(init), float(a0), float(lam), float(w0),
                    float(n_cycles), _p(r), _p(b), _p(bd))
    return r, b, bd


def laser_fields(x, t, a0, lam, w0, n_cycles):
    """Laser E, B [n][3] at points x[n][3], times t[n]."""
    x = _f64(x).reshape(-1, 3)
    t = _f64(t).reshape(-1)
    E = np.empty_like(x)
    B = np.empty_like(x)
    lib().orc_laser_fields(x.shape[0], _p(x), _p(t), float(a0), float(lam), float(w0), float(n_cycles), _p(E), _p(B))
    return E, B
