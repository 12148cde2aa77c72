"""torch.autograd Functions over the library's forward and adjoint entry points.

* ``LWSpectrum``: trajectory samples (r, beta, beta_dot) -> spectra S [n_pix][n_obs/2+1] through
  lw_deposit_td and lw_spectrum_fft; backward through lw_spectrum_fft_bwd and
  lw_deposit_td_bwd (FP64).  Pixels whose incoming gradient row is zero are left out of the
  backward (their contribution is exactly zero).
* ``BorisTrajectory``: (init [n_p][6], a0) -> samples through lw_trajectory_boris; backward
  through lw_trajectory_boris_bwd (forward-mode tangents of the FP64 pusher).
* ``LWSpectrumBoris``: (init [n_p][6], a0) -> spectra through lw_deposit_td with the trajectories
  recomputed inside the call (LW_TRAJ_BORIS) and lw_spectrum_fft; backward through
  lw_spectrum_fft_bwd and lw_deposit_td_bwd_boris, which pushes the trajectories again with
  their tangents.  No trajectory sample is stored at any point (only the trace E is kept).
* ``BunchInit``: gamma_mean -> the seeded bunch draw's initial conditions on the device, with
  d(init)/d(gamma_mean) of the recipe for the backward.

Chained, these give d(band-limited spectral energy)/d(gamma_mean, a0):

    init = bunch_init(w, rows, gamma)                  # gamma, a0: float64 CPU scalars
    r, b, bd = boris_trajectory(init, a0, w)
    S, diag = lw_spectrum(r, b, bd, w.t_start, w.dt, x_det, w.t0, w.dt_obs, w.n_obs)
    J = (weights * S).sum(); J.backward()

or, with no trajectory stored:

    S, diag = lw_spectrum_boris(bunch_init(w, rows, gamma), a0, w, x_det)
"""
from __future__ import annotations

import numpy as np
import torch

from . import inputs, lw


class LWSpectrum(torch.autograd.Function):
    @staticmethod
    def forward(ctx, r, beta, beta_dot, x_det, charge, t_start, dt, t0, dt_obs, n_obs, prec, field_mask, geom):
        E, diag = lw.deposit_td(r, beta, beta_dot, t_start, dt, x_det, t0, dt_obs, n_obs, prec=prec,
                                field_mask=field_mask, geom=geom, charge=charge)
        S = lw.spectrum_fft(E, dt_obs, prec)
        ctx.save_for_backward(r, beta, beta_dot, x_det, charge, E)
        ctx.args = (t_start, dt, t0, dt_obs, n_obs, prec, field_mask, geom)
        ctx.mark_non_differentiable(diag)
        return S, diag

    @staticmethod
    def backward(ctx, dS, _ddiag):
        r, beta, beta_dot, x_det, charge, E = ctx.saved_tensors
        t_start, dt, t0, dt_obs, n_obs, prec, field_mask, geom = ctx.args
        if prec != "fp64":
            raise RuntimeError("LWSpectrum: gradients are computed in FP64; run the forward with prec='fp64'")
        nones = (None,) * 10
        if dS is None or not any(ctx.needs_input_grad[:3]):
            return (None, None, None) + nones
        dS = dS.to(torch.float64).contiguous()
        live = torch.nonzero(torch.any(dS != 0, dim=1)).flatten()
        if live.numel() == 0:
            z = torch.zeros_like(r)
            return (z, z.clone(), z.clone()) + nones
        if live.numel() < dS.shape[0]:
            E, dS, x_det = E[live].contiguous(), dS[live].contiguous(), x_det[live].contiguous()
        dE = lw.spectrum_fft_bwd(E, dS, dt_obs, "fp64")
        d_r, d_b, d_bd = lw.deposit_td_bwd(r, beta, beta_dot, t_start, dt, x_det, t0, dt_obs, n_obs, dE,
                                           field_mask=field_mask, geom=geom, charge=charge)
        return (d_r, d_b, d_bd) + nones


def lw_spectrum(r, beta, beta_dot, t_start, dt, x_det, t0, dt_obs, n_obs, prec="fp64", field_mask=lw.FIELD_ACCEL,
                geom="exact", charge=None):
    """Differentiable S [n_pix][n_obs/2+1] (and diag) of trajectory samples on the device."""
    return LWSpectrum.apply(r, beta, beta_dot, x_det, charge, float(t_start), float(dt), float(t0), float(dt_obs),
                            int(n_obs), prec, int(field_mask), geom)


class LWSpectrumBoris(torch.autograd.Function):
    @staticmethod
    def forward(ctx, init, a0, x_det, charge, n_samples, t_start, dt, lam, w0, n_cycles, t0, dt_obs, n_obs, prec,
                field_mask, geom):
        a0v = _f64_scalar(a0, "a0")
        E, diag = lw.deposit_td_boris(init, n_samples, t_start, dt, a0v, lam, w0, n_cycles, x_det, t0, dt_obs, n_obs,
                                      prec=prec, field_mask=field_mask, geom=geom, charge=charge)
        S = lw.spectrum_fft(E, dt_obs, prec)
        ctx.save_for_backward(init, x_det, charge, E)
        ctx.args = (n_samples, t_start, dt, a0v, lam, w0, n_cycles, t0, dt_obs, n_obs, prec, field_mask, geom)
        ctx.a0_meta = (a0.dtype, a0.device) if isinstance(a0, torch.Tensor) else None
        ctx.mark_non_differentiable(diag)
        return S, diag

    @staticmethod
    def backward(ctx, dS, _ddiag):
        init, x_det, charge, E = ctx.saved_tensors
        n_samples, t_start, dt, a0v, lam, w0, n_cycles, t0, dt_obs, n_obs, prec, field_mask, geom = ctx.args
        nones = (None,) * 14
        if prec != "fp64":
            raise RuntimeError("LWSpectrumBoris: gradients are computed in FP64; run the forward with prec='fp64'")
        if dS is None or not (ctx.needs_input_grad[0] or ctx.needs_input_grad[1]):
            return (None, None) + nones
        dS = dS.to(torch.float64).contiguous()
        live = torch.nonzero(torch.any(dS != 0, dim=1)).flatten()
        if live.numel() == 0:
            g_a0 = None if ctx.a0_meta is None else torch.zeros((), dtype=ctx.a0_meta[0], device=ctx.a0_meta[1])
            return (torch.zeros_like(init), g_a0) + nones
        if live.numel() < dS.shape[0]:
            E, dS, x_det = E[live].contiguous(), dS[live].contiguous(), x_det[live].contiguous()
        dE = lw.spectrum_fft_bwd(E, dS, dt_obs, "fp64")
        grad_init, grad_a0 = lw.deposit_td_bwd_boris(init, n_samples, t_start, dt, a0v, lam, w0, n_cycles, x_det, t0,
                                                     dt_obs, n_obs, dE, field_mask=field_mask, geom=geom,
                                                     charge=charge)
        d_a0 = None
        if ctx.a0_meta is not None and ctx.needs_input_grad[1]:
            d_a0 = grad_a0.sum().to(dtype=ctx.a0_meta[0], device=ctx.a0_meta[1])
        return (grad_init, d_a0) + nones


def lw_spectrum_boris(init, a0, w: inputs.Workload, x_det, prec="fp64", field_mask=lw.FIELD_ACCEL, geom="exact",
                      charge=None):
    """Differentiable S [n_pix][n_obs/2+1] (and diag) of the bunch init [n_p][6] pushed through the
    laser of w with amplitude a0 (a float64 CPU scalar tensor, or a float), the trajectories
    recomputed inside the deposit and again inside its adjoint (never stored)."""
    L = w.laser
    return LWSpectrumBoris.apply(init, a0, x_det, charge, int(w.n_samples), float(w.t_start), float(w.dt),
                                 float(L.lam), float(L.w0), float(L.n_cycles), float(w.t0), float(w.dt_obs),
                                 int(w.n_obs), prec, int(field_mask), geom)


def _f64_scalar(x, name):
    """A Python float or a float64 scalar tensor (a float32 tensor would round the parameter)."""
    if isinstance(x, torch.Tensor):
        if x.dtype != torch.float64 or x.numel() != 1:
            raise TypeError(f"{name} must be a float64 scalar tensor, got {x.dtype} of shape {tuple(x.shape)}")
        return float(x)
    return float(x)


class BorisTrajectory(torch.autograd.Function):
    @staticmethod
    def forward(ctx, init, a0, n_samples, t_start, dt, lam, w0, n_cycles):
        a0v = _f64_scalar(a0, "a0")
        out = lw.trajectory_boris(init, n_samples, t_start, dt, a0v, lam, w0, n_cycles)
        ctx.save_for_backward(init)
        ctx.args = (n_samples, t_start, dt, a0v, lam, w0, n_cycles)
        ctx.a0_meta = (a0.dtype, a0.device) if isinstance(a0, torch.Tensor) else None
        return out

    @staticmethod
    def backward(ctx, g_r, g_b, g_bd):
        (init,) = ctx.saved_tensors
        n_samples, t_start, dt, a0v, lam, w0, n_cycles = ctx.args
        shape = (init.shape[0], n_samples, 3)
        g = [torch.zeros(shape, dtype=torch.float64, device=init.device) if x is None else x.contiguous()
             for x in (g_r, g_b, g_bd)]
        grad_init, grad_a0 = lw.trajectory_boris_bwd(init, n_samples, t_start, dt, a0v, lam, w0, n_cycles, *g)
        d_a0 = None
        if ctx.a0_meta is not None and ctx.needs_input_grad[1]:
            d_a0 = grad_a0.sum().to(dtype=ctx.a0_meta[0], device=ctx.a0_meta[1])
        return grad_init, d_a0, None, None, None, None, None, None


def boris_trajectory(init, a0, w: inputs.Workload):
    """Differentiable FP64 Boris samples (r, beta, beta_dot) of init [n_p][6] in the laser of w
    with amplitude a0 (a float64 CPU scalar tensor, or a float)."""
    L = w.laser
    return BorisTrajectory.apply(init, a0, w.n_samples, w.t_start, w.dt, L.lam, L.w0, L.n_cycles)


class BunchInit(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gamma, w, rows, device):
        g = _f64_scalar(gamma, "gamma")
        init = inputs.bunch_init(w, gamma=g)
        dinit = inputs.bunch_init_dgamma(w.scaled(gamma=g), rows)
        if rows is not None:
            init = init[np.asarray(rows)]
        ctx.save_for_backward(torch.as_tensor(np.ascontiguousarray(dinit), device=device))
        ctx.g_meta = (gamma.dtype, gamma.device) if isinstance(gamma, torch.Tensor) else None
        return torch.as_tensor(np.ascontiguousarray(init), device=device)

    @staticmethod
    def backward(ctx, grad_init):
        if ctx.g_meta is None or not ctx.needs_input_grad[0]:
            return None, None, None, None
        (dinit,) = ctx.saved_tensors
        d = torch.sum(grad_init * dinit).to(dtype=ctx.g_meta[0], device=ctx.g_meta[1])
        return d, None, None, None


def bunch_init(w: inputs.Workload, rows, gamma, device="cuda"):
    """Initial conditions of the seeded draw of w (rows of it, or all if None) at mean Lorentz
    factor gamma (a float64 CPU scalar tensor), as a float64 device tensor [n][6]."""
    return BunchInit.apply(gamma, w, rows, torch.device(device))
