"""Oracle gradients (test infrastructure only).

* ``spectrum_vjp``: dJ/dE of J = sum_j dS_j S_j with S from ``spectrum`` (Eq. efield_xfrom):
  dE_c[u] = (dt^2/pi) Re sum_{j<=N/2} dS_j F_c[j] exp(+2 pi i j u / N),  F_c = rfft(E_c).
  Pinned by the exact central difference of the quadratic S (test_oracle_grad.py).
* ``chain_complex``: the whole chain -- arrival time and field of every sample
  (Eqs. advanced_condition / far_adv, lw_fields_retarded), Algorithm 2 interpolation,
  spectrum, objective -- evaluated in complex arithmetic.  With inputs x + i h v
  (h ~ 1e-30) the imaginary part of the result is h times the exact directional
  derivative of the FP64 chain along v (complex-step differentiation; every
  discrete decision uses real parts).  Pinned against central finite differences of
  the real C oracle and against the real part of the C oracle itself.
* ``boris_complex``: the leap-frog Boris pusher of the C oracle's ``orc_boris`` written
  with numpy over particles in complex arithmetic, so that a complex step in the initial
  phase space or in a0 gives the exact directional derivative of the trajectory (the
  forward-mode tangent of the pusher).  Pinned against the real C oracle (real part) and
  against its central differences (imaginary part).
* ``direct_fd_complex``: the direct frequency-domain sum (Eq. inty_dft, Algorithm 1) in
  complex arithmetic, S(w) = (dt^2/2pi) sum_c (sum E_c kappa cos(w t))^2 + (sum E_c kappa
  sin(w t))^2 with t = t_i + tt - t0; pinned against the C oracle's ``orc_direct_fd``
  (value) and its central differences (derivative).
* ``params_derivative``: dJ/dgamma_mean and dJ/da0 of the band objective by one complex
  step through the seeded bunch draw, the pusher and the chain above.
"""
from __future__ import annotations

import numpy as np

C_LIGHT = 299792458.0
Q_E = 1.602176634e-19
EPS0 = 8.8541878128e-12
M_E = 9.1093837015e-31


def spectrum_vjp(E_tot, dS, dt_obs):
    """dJ/dE for J = sum dS * spectrum(E_tot, dt_obs).  E_tot [..., 3, N], dS [..., N/2+1]."""
    E_tot = np.asarray(E_tot, dtype=np.float64)
    N = E_tot.shape[-1]
    F = np.fft.rfft(E_tot, axis=-1)
    G = np.asarray(dS, dtype=np.float64)[..., None, :] * F
    pad = np.zeros(E_tot.shape[:-1] + (N,), dtype=np.complex128)
    pad[..., : N // 2 + 1] = G
    return (dt_obs * dt_obs / np.pi) * (N * np.fft.ifft(pad, axis=-1)).real


def _dot(a, b):
    return np.sum(a * b, axis=-1)


def eval_complex(x, r, b, a, q, field_mask=1, geom=0, with_kappa=False):
    """Arrival shift tt (relative to t + |x|/c) and field E of samples r, b, a [n][3] (complex
    allowed) at observer x, written with the analytic (complex-differentiable) operations of
    the definitions; the exact-geometry shift uses the cancellation-free identity
    |x - r| - |x| = -s + |r - s n|^2 / (|x - r| + |x| - s).  With with_kappa, also
    kappa = 1 - n.b."""
    x = np.asarray(x, dtype=np.float64)
    D = np.sqrt(x @ x)
    nm = x / D
    s = r @ nm
    if geom == 1:
        n = np.broadcast_to(nm, r.shape)
        R = D
        tt = -s / C_LIGHT
    else:
        rp = r - s[:, None] * nm
        p2 = _dot(rp, rp)
        d = x - r
        R = np.sqrt(_dot(d, d))
        n = d / R[:, None]
        tt = -s / C_LIGHT + p2 / (C_LIGHT * (R + D - s))
    kappa = 1.0 - _dot(n, b)
    pref = q / (4.0 * np.pi * EPS0)
    E = np.zeros(r.shape, dtype=np.result_type(r, b, a))
    nb = n - b
    Rc = R if np.ndim(R) == 0 else R[:, None]
    if field_mask & 2:
        E = E + (pref * (1.0 - _dot(b, b)) / (kappa ** 3))[:, None] * nb / Rc ** 2
    if field_mask & 1:
        w = np.cross(nb, a)
        v = np.cross(n, w)
        E = E + (pref / (C_LIGHT * kappa ** 3))[:, None] * v / Rc
    if with_kappa:
        return tt, E, kappa
    return tt, E


def deposit_complex(t_start, dt, r, b, a, x_det, t0, dt_obs, n_obs, charge=None, field_mask=1, geom=0):
    """Algorithm 2 deposit (all samples assumed usable) in complex arithmetic; decisions on
    real parts.  Returns E_tot [n_pix][3][n_obs] complex."""
    r = np.asarray(r)
    n_p, ns = r.shape[0], r.shape[1]
    x_det = np.asarray(x_det, dtype=np.float64).reshape(-1, 3)
    out = np.zeros((x_det.shape[0], 3, n_obs), dtype=np.complex128)
    ti = t_start + np.arange(ns) * dt
    for m in range(x_det.shape[0]):
        for k in range(n_p):
            q = -Q_E if charge is None else charge[k]
            tt, E = eval_complex(x_det[m], r[k], b[k], a[k], q, field_mask, geom)
            tau = ((ti + tt) - t0) / dt_obs
            tr = tau.real
            lo = np.floor(tr[:-1]) + 1.0
            hi = np.floor(tr[1:])
            good = tr[1:] > tr[:-1]
            lo = np.maximum(lo, 0.0)
            hi = np.minimum(hi, n_obs - 1.0)
            cnt = np.where(good, np.maximum(hi - lo + 1.0, 0.0), 0.0).astype(np.int64)
            if cnt.sum() == 0:
                continue
            idx = np.repeat(np.arange(ns - 1), cnt)
            starts = np.repeat(lo.astype(np.int64), cnt)
            offs = np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt)
            u = starts + offs
            w = (u - tau[idx]) / (tau[idx + 1] - tau[idx])
            val = (1.0 - w)[:, None] * E[idx] + w[:, None] * E[idx + 1]
            for c in range(3):
                np.add.at(out[m, c], u, val[:, c])
    return out


def spectrum_complex(E_tot, dt_obs):
    """S = (dt^2/2pi) sum_c (Re F_c)^2 + (Im F_c)^2 with Re F, Im F the real-linear maps of the
    DFT applied to a complex (complex-step) trace."""
    Er = np.fft.rfft(E_tot.real, axis=-1)
    Ei = np.fft.rfft(E_tot.imag, axis=-1)
    Fre = Er.real + 1j * Ei.real
    Fim = Er.imag + 1j * Ei.imag
    return (dt_obs * dt_obs / (2.0 * np.pi)) * np.sum(Fre * Fre + Fim * Fim, axis=-2)


def chain_complex(t_start, dt, r, b, a, x_det, t0, dt_obs, n_obs, weights=None, dE=None, charge=None,
                  field_mask=1, geom=0):
    """J = sum(weights * S) (or sum(dE * E_tot) when dE is given) through the complex chain."""
    E = deposit_complex(t_start, dt, r, b, a, x_det, t0, dt_obs, n_obs, charge, field_mask, geom)
    if dE is not None:
        return np.sum(np.asarray(dE) * E)
    S = spectrum_complex(E, dt_obs)
    return np.sum(np.asarray(weights) * S)


def directional_derivative(t_start, dt, r, b, a, v_r, v_b, v_a, x_det, t0, dt_obs, n_obs, weights=None, dE=None,
                           charge=None, field_mask=1, geom=0, h=1e-30):
    """Complex-step derivative of J along (v_r, v_b, v_a) at (r, b, a)."""
    J = chain_complex(t_start, dt, r + 1j * h * v_r, b + 1j * h * v_b, a + 1j * h * v_a, x_det, t0, dt_obs, n_obs,
                      weights, dE, charge, field_mask, geom)
    return J.imag / h, J.real


def _laser_eb(lam, w0, n_cycles, a0, x, y, z, t):
    """E_x and B_y of the x-polarised pulse travelling along -z (normalised vector potential
    a0 g(phi) sin(phi), g = cos^2(phi/(2 n_cycles)) on |phi| < pi n_cycles, phi = wl (t + z/c),
    transverse factor exp(-(x^2+y^2)/w0^2) when w0 > 0): E_x = -E0 T d(g sin)/dphi, B_y = -E_x/c."""
    wl = 2.0 * np.pi * C_LIGHT / lam
    phi = wl * (t + z / C_LIGHT)
    inside = np.abs(phi.real) < np.pi * n_cycles
    g = np.cos(phi / (2.0 * n_cycles)) ** 2
    gp = -np.sin(phi / n_cycles) / (2.0 * n_cycles)
    sp = gp * np.sin(phi) + g * np.cos(phi)
    T = np.exp(-(x * x + y * y) / (w0 * w0)) if w0 > 0.0 else 1.0
    E0 = a0 * M_E * C_LIGHT * wl / Q_E
    Ex = np.where(inside, -E0 * T * sp, 0.0)
    return Ex, -Ex / C_LIGHT


def _kick(u, Ex, By, h):
    """Boris update of u = gamma beta [n][3] over time h for electrons in E = (Ex,0,0), B = (0,By,0):
    half electric kick, magnetic rotation with t = q h B/(2 m gamma), s = 2 t/(1+t^2), half kick."""
    q, m = -Q_E, M_E
    a = q * h / (2.0 * m * C_LIGHT)
    um = u + np.stack([a * Ex, 0.0 * Ex, 0.0 * Ex], axis=-1)
    gm = np.sqrt(1.0 + _dot(um, um))
    tv = np.stack([0.0 * By, q * h * By / (2.0 * m * gm), 0.0 * By], axis=-1)
    sv = 2.0 * tv / (1.0 + _dot(tv, tv))[:, None]
    up = um + np.cross(um, tv)
    return um + np.cross(up, sv) + np.stack([a * Ex, 0.0 * Ex, 0.0 * Ex], axis=-1)


def boris_complex(init, n_samples, t_start, dt, a0, lam, w0, n_cycles):
    """r, beta, beta_dot [n_p][n_samples][3] of electrons from init [n_p][6] (x, y, z, u = gamma beta)
    by the leap-frog Boris scheme: u_{1/2} from a half kick at (r_0, t_0); r_{i+1} = r_i + c u_{i+1/2}
    / gamma_{i+1/2} dt; u_{i+3/2} from a full kick at (r_{i+1}, t_{i+1}); beta_0 from u_0 and
    beta_i from (u_{i-1/2} + u_{i+1/2})/2; beta_dot from the Lorentz force
    q/(gamma m c) [E + c beta x B - beta (beta.E)].  Complex inputs allowed (complex step)."""
    init = np.asarray(init)
    dtype = np.result_type(init, a0, np.float64)
    n_p = init.shape[0]
    r = np.empty((n_p, n_samples, 3), dtype=dtype)
    b = np.empty_like(r)
    bd = np.empty_like(r)
    x = init[:, :3].astype(dtype)
    us = init[:, 3:].astype(dtype)
    q, m = -Q_E, M_E
    Ex, By = _laser_eb(lam, w0, n_cycles, a0, x[:, 0], x[:, 1], x[:, 2], t_start)
    uh = _kick(us, Ex, By, 0.5 * dt)
    for i in range(n_samples):
        ti = t_start + i * dt
        g = np.sqrt(1.0 + _dot(us, us))
        bb = us / g[:, None]
        Ex, By = _laser_eb(lam, w0, n_cycles, a0, x[:, 0], x[:, 1], x[:, 2], ti)
        E = np.stack([Ex, 0.0 * Ex, 0.0 * Ex], axis=-1)
        B = np.stack([0.0 * By, By, 0.0 * By], axis=-1)
        f = q / (g * m * C_LIGHT)
        r[:, i] = x
        b[:, i] = bb
        bd[:, i] = f[:, None] * (E + C_LIGHT * np.cross(bb, B) - bb * _dot(bb, E)[:, None])
        if i + 1 == n_samples:
            break
        gh = np.sqrt(1.0 + _dot(uh, uh))
        x = x + C_LIGHT * uh / gh[:, None] * dt
        Ex, By = _laser_eb(lam, w0, n_cycles, a0, x[:, 0], x[:, 1], x[:, 2], t_start + (i + 1) * dt)
        un = _kick(uh, Ex, By, dt)
        us = 0.5 * (uh + un)
        uh = un
    return r, b, bd


def params_derivative(init_of_gamma, gamma, a0, laser, n_samples, t_start, dt, x_det, t0, dt_obs, n_obs, weights,
                      which, geom=0, h=1e-30):
    """Complex-step dJ/dgamma_mean (which = "gamma") or dJ/da0 (which = "a0") of
    J = sum(weights * S) with trajectories from ``boris_complex`` and initial conditions
    init_of_gamma(gamma) (the seeded bunch draw at mean Lorentz factor gamma).
    laser = (lam, w0, n_cycles).  Returns (derivative, J)."""
    lam, w0, n_cycles = laser
    g = gamma + (1j * h if which == "gamma" else 0.0)
    a = a0 + (1j * h if which == "a0" else 0.0)
    init = init_of_gamma(g)
    r, b, bd = boris_complex(init, n_samples, t_start, dt, a, lam, w0, n_cycles)
    J = chain_complex(t_start, dt, r, b, bd, x_det, t0, dt_obs, n_obs, weights=weights, geom=geom)
    return J.imag / h, J.real


def direct_fd_complex(t_start, dt, r, b, a, x_det, t0, omega, charge=None, field_mask=1, geom=0):
    """Direct FD spectra S [n_pix][n_omega] in complex arithmetic (all samples assumed usable)."""
    r = np.asarray(r)
    n_p, ns = r.shape[0], r.shape[1]
    x_det = np.asarray(x_det, dtype=np.float64).reshape(-1, 3)
    omega = np.asarray(omega, dtype=np.float64)
    ti = t_start + np.arange(ns) * dt
    out = []
    for m in range(x_det.shape[0]):
        Rc = np.zeros((3, omega.size), dtype=np.complex128)
        Ic = np.zeros((3, omega.size), dtype=np.complex128)
        for k in range(n_p):
            q = -Q_E if charge is None else charge[k]
            tt, E, kap = eval_complex(x_det[m], r[k], b[k], a[k], q, field_mask, geom, with_kappa=True)
            t = (ti + tt) - t0
            A = E * kap[:, None]
            ph = omega[None, :] * t[:, None]
            Rc += A.T @ np.cos(ph)
            Ic += A.T @ np.sin(ph)
        out.append((dt * dt / (2.0 * np.pi)) * np.sum(Rc * Rc + Ic * Ic, axis=0))
    return np.array(out)


def fd_directional_derivative(t_start, dt, r, b, a, v_r, v_b, v_a, x_det, t0, omega, dS, charge=None, field_mask=1,
                              geom=0, h=1e-30):
    """Complex-step derivative of J = sum(dS * S_FD) along (v_r, v_b, v_a).  Returns (dJ, J)."""
    S = direct_fd_complex(t_start, dt, r + 1j * h * v_r, b + 1j * h * v_b, a + 1j * h * v_a, x_det, t0, omega,
                          charge, field_mask, geom)
    J = np.sum(np.asarray(dS) * S)
    return J.imag / h, J.real
