#!/usr/bin/env python3
"""Benchmark of the time-domain Lienard-Wiechert hot path on one MI355X.

Headline workload ("precision"): 1e5 electrons (gamma = 200, sigma_gamma/gamma = 1e-3,
sigma_x,y = 2 um, sigma_z = 5 um, eps_n = 1 mm mrad, seeded draws) in a Gaussian laser pulse
(a0 = 1, w0 = 10 um, 20 cycles of 1 um), 2e4 FP64 Boris steps, 128 x 128 pixels over +-2/gamma
at 1 m, 2^18 observer grid points per pixel (16 per first-harmonic period), exact geometry,
acceleration field.  The initial conditions and pixels are resident in HBM before timing.

One step = lw_deposit_td with the trajectories recomputed inside the call by the FP64 Boris
pusher, span by span (LW_TRAJ_BORIS: the 144 GB of samples never exist whole), i.e. the arrival
time of every particle x sample x pixel, the field where the interpolation reads it and the
linear-interpolation deposit, + lw_spectrum_fft (|E(w)|^2), in mixed precision (arrival times in
FP64, fields/trace/FFT in FP32).  ``value`` counts particle * sample * pixel triples per second
of step time.

In the same line: the all-FP64 pass of the same workload (speedup of mixed over FP64) and the
band-L2 error of mixed against FP64 in the harmonic bands h = 1..5 of every pixel; the deposit
kernel against the roofline of the work it performs (an FP64 arrival time for every triple, the
field at both ends and the interpolation for every deposited grid point; kernel time from HIP
events the library records around its launches), with counter figures from committed rocprofv3
summaries while the deposit sources are unchanged; the culled variant (same spectra); the FFT
against HBM bandwidth; the Boris pusher's trajectory write rate; the observer-window
diagnostics; the bunch workload (1e4 e-, 64 x 64 px, stored trajectories) with its own
roofline; the direct frequency-domain sum on 64 of its pixels; the gradient of a band objective
on the differentiation workload; and the FP64 CPU oracle on a bounded sample (``cpu_baseline``).

Other modes (one JSON line each, not the headline): ``--workload bunch`` (the bunch workload as
the headline), ``--workload large`` (one full-size pass of that configuration, mixed against
FP64, with the full-size adjoint), ``--cost-model`` (refit of the wall-clock model constants and
the TD/FD crossover), ``--accuracy`` (the single-electron accuracy experiment against a
converged reference and the oracle) and ``--det`` (the order-independent FP64 deposit against the
atomics-order one on the bunch workload).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("particle·step·pixel LW evals/s; mixed vs FP64 speedup at ≤1e-4 spectral error")

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
CUS, CLOCK_GHZ, LANES = 256, 2.4, 64
PEAK_F32_TFLOPS = 157.3  # vector FP32 (256 CUs x 2.4 GHz x 128 lanes x 2 flops, packed)
PEAK_F64_TFLOPS = 78.6   # vector FP64
# Work the deposit performs (its roofline): the arrival time of every (particle, sample, pixel)
# triple, 6 FP64 flops (three fused multiply-adds: the sample's time base minus n.r/(c dt_obs)),
# and for every deposited grid point the field at the interval's two ends (68 FP32 flops each:
# n x ((n - b) x bd), the 1/kappa^3 factor and the prefactors) plus the interpolation (13 FP32
# flops: weight, its complement, three lerps).  Roofline time = F64/P64 + F32/P32.
TRIPLE_F64_FLOPS = 6
FIELD_F32_FLOPS = 68
HIT_F32_FLOPS = 2 * FIELD_F32_FLOPS + 13
# the per-evaluation figure of a method that forms the field for every triple (dense)
DENSE_F32_FLOPS, DENSE_F64_FLOPS = 68, 6
# Direct FD: ~18 FP32 flops per (particle, sample, pixel, frequency) term (phase, sin/cos,
# three complex multiply-accumulates)
FD_TERM_FLOPS = 18
# Deposit adjoint (all FP64): the arrival time of every triple (6 flops, as in the forward) and for
# every deposited grid point, at the interval's two ends, the field (68 flops) and its
# vector-Jacobian product (twice the field's), plus the interpolation's adjoint (~20 flops)
ADJ_TRIPLE_F64_FLOPS = 6
ADJ_POINT_F64_FLOPS = 2 * (FIELD_F32_FLOPS + 2 * FIELD_F32_FLOPS) + 20
DEPOSIT_SOURCES = ("paper_2206_03015_amd/csrc/deposit.hip", "paper_2206_03015_amd/csrc/lw_internal.h")
SUMMARIES = {
    "precision": {"traffic": "profiles/k_scan_precision_mixed_hbm_traffic.md",
                  "valu": "profiles/k_scan_precision_mixed_valu.md",
                  "types": "profiles/valu_fp32_fp64_precision.md"},
    "bunch": {"traffic": "profiles/k_scan_bunch_mixed_exact_hbm_traffic.md",
              "valu": "profiles/k_scan_bunch_mixed_exact_valu.md",
              "types": "profiles/valu_fp32_fp64_bunch.md"},
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--geom", default="exact", choices=["exact", "farfield"])
    p.add_argument("--particles", type=int, default=None, help="override particle count (testing only)")
    p.add_argument("--no-fp64", action="store_true")
    p.add_argument("--no-fd", action="store_true")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-grad", action="store_true")
    p.add_argument("--no-cull", action="store_true", help="skip the culled-variant leg")
    p.add_argument("--no-bunch", action="store_true", help="skip the bunch-workload leg of the headline line")
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--cost-model", action="store_true",
                   help="instead of the headline step: refit the wall-clock model constants C1_t, C2_t, C_w "
                        "by single-variate sweeps and time the TD/FD crossover in the particle count")
    p.add_argument("--workload", default="precision", choices=["precision", "bunch", "large"],
                   help="precision: the headline (trajectories pushed inside the deposit); bunch: the bunch "
                        "workload as the headline (stored trajectories); large: one full-size pass of that "
                        "configuration with its adjoint")
    p.add_argument("--accuracy", action="store_true",
                   help="instead of the headline step: the single-electron accuracy experiment (Eq. "
                        "spectra_error of TD and FD against a converged FP64 FD reference and the oracle)")
    p.add_argument("--det", action="store_true",
                   help="instead of the headline step: the bunch workload in FP64 through lw_deposit_td and "
                        "lw_deposit_td_det (times, run-to-run bit equality of each, their difference)")
    p.add_argument("--copy-calibration-gib", type=float, default=0.0,
                   help="run a plain device copy of this many GiB first (scale for HBM byte counters)")
    return p.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU pixel "
              "sharding is described as a design only and not implemented.", flush=True)
        return 2
    import torch
    from paper_2206_03015_amd import lw

    lw.load()
    dev = torch.device("cuda:0")
    if args.cost_model:
        print(json.dumps(cost_model(torch, dev)), flush=True)
        return 0
    if args.accuracy:
        print(json.dumps(accuracy(torch, dev)), flush=True)
        return 0
    if args.det:
        print(json.dumps(det_leg(torch, dev)), flush=True)
        return 0
    if args.copy_calibration_gib > 0:
        n = int(args.copy_calibration_gib * (1 << 30)) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)  # a plain elementwise copy (torch runs it as kernels of <= 2 GiB): n*4 bytes read, n*4 written
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: {n * 4} bytes read and written by an elementwise copy")
        del src, dst
    if args.workload == "large":
        print(json.dumps(full_size(torch, dev, "large")), flush=True)
        return 0
    rec = headline(torch, dev, args)
    print(json.dumps(rec), flush=True)
    return 0


def deposit_roofline(triples, hits, kernel_s, launches, summaries=None, profiled=False):
    """Roofline of the deposit kernel on the work it performs (TRIPLE_F64_FLOPS per triple,
    HIT_F32_FLOPS per deposited grid point) over its measured time (HIP events around its
    launches), with the dense per-evaluation figure and the committed counter figures beside it."""
    f64 = triples * TRIPLE_F64_FLOPS
    f32 = hits * HIT_F32_FLOPS
    t_roof = f64 / (PEAK_F64_TFLOPS * 1e12) + f32 / (PEAK_F32_TFLOPS * 1e12)
    work = f64 + f32
    peak = work / t_roof / 1e12
    achieved = work / kernel_s / 1e12
    roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": None, "kernel": "k_scan", "launches": launches, "kernel_ms": kernel_s * 1e3,
            "work": {"f64_flops": f64, "f32_flops": f32, "triples": triples, "deposited_points": hits,
                     "f64_flops_per_triple": TRIPLE_F64_FLOPS, "f32_flops_per_deposited_point": HIT_F32_FLOPS},
            "roofline_ms": t_roof * 1e3}
    dense_s = triples * (DENSE_F32_FLOPS / (PEAK_F32_TFLOPS * 1e12) + DENSE_F64_FLOPS / (PEAK_F64_TFLOPS * 1e12))
    roof["dense_per_eval_figure"] = {"note": "68 FP32 + 6 FP64 flops credited to every triple (a method "
                                             "that forms the field everywhere); not the work performed",
                                     "frac": dense_s / kernel_s}
    if profiled and summaries:
        roof["traffic"] = _summary_value(summaries["traffic"], "hbm_bytes_per_step")
        valu = _summary_value(summaries["valu"], "valu_insts_per_step")
        if valu is not None:
            roof["executed_valu_insts"] = valu
            roof["valu_issue_frac"] = valu * 4 / (CUS * 4 * CLOCK_GHZ * 1e9 * kernel_s)
        ex = (_summary_value(summaries["types"], "f64_flops_per_step"),
              _summary_value(summaries["types"], "f32_flops_per_step"))
        if ex[0] is not None and ex[1] is not None:
            a64, a32 = ex[0] / kernel_s / 1e12, ex[1] / kernel_s / 1e12
            roof["executed"] = {"f64_tflops": a64, "f64_frac": a64 / PEAK_F64_TFLOPS,
                                "f32_tflops": a32, "f32_frac": a32 / PEAK_F32_TFLOPS}
    return roof


def band_errors(torch, dev, W, S_a, S_b, harmonics, chunk=512):
    """Band-L2 error of S_a against S_b (both [n_pix][n_obs/2+1] on the device) in the harmonic bands
    [(h - 0.3) w1, (h + 0.1) w1] of every pixel (w1 at the pixel's polar angle): max and median."""
    from paper_2206_03015_amd import inputs
    tx, ty = inputs.pixel_angles(W.n_side, W.theta_max)
    w1 = torch.as_tensor(np.array([W.omega1(t) for t in np.hypot(tx, ty)]), device=dev)[:, None]
    wgrid = torch.as_tensor(2 * np.pi * np.arange(W.n_obs // 2 + 1) / (W.n_obs * W.dt_obs), device=dev)
    out = {}
    for h in harmonics:
        errs = []
        for m0 in range(0, W.n_pix, chunk):
            m1 = min(W.n_pix, m0 + chunk)
            band = (wgrid[None, :] >= (h - 0.3) * w1[m0:m1]) & (wgrid[None, :] <= (h + 0.1) * w1[m0:m1])
            a = S_a[m0:m1].double() * band
            b = S_b[m0:m1].double() * band
            den = torch.linalg.vector_norm(b, dim=1)
            ok = den > 0
            errs.append((torch.linalg.vector_norm(a - b, dim=1)[ok] / den[ok]).cpu().numpy())
        errs = np.concatenate(errs)
        out[f"h{h}"] = {"max": float(errs.max()), "median": float(np.median(errs)), "pixels": int(errs.size)}
        log(f"[bench] h={h}: band L2 mixed vs FP64 max {errs.max():.2e} median {np.median(errs):.2e} over "
            f"{errs.size} pixels")
    return out


def headline(torch, dev, args):
    """The headline line: the precision workload (default) with in-call Boris trajectories, or the
    bunch workload with stored trajectories (``--workload bunch``)."""
    from paper_2206_03015_amd import grid, inputs, lw
    name = args.workload
    W = inputs.workload(name)
    if args.particles:
        W = W.scaled(n_p=args.particles)
    L = W.laser
    log(f"[bench] workload {name}: n_p={W.n_p} n_samples={W.n_samples} n_pix={W.n_pix} n_obs={W.n_obs}")
    init = torch.as_tensor(inputs.bunch_init(W), device=dev)
    x_det = torch.as_tensor(inputs.pixel_positions(W.n_side, W.theta_max, W.D), device=dev)
    n_pix, n_obs = W.n_pix, W.n_obs
    triples = W.n_p * W.n_samples * n_pix
    in_call = name == "precision"

    # ---- trajectories pushed once (untimed for the step): the pusher's write rate, and the first
    # and last samples of every particle for the observer-window diagnostics
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    r, b, bd = lw.trajectory_boris(init, W.n_samples, W.t_start, W.dt, L.a0, L.lam, L.w0, L.n_cycles)
    e1.record()
    torch.cuda.synchronize()
    push_ms = e0.elapsed_time(e1)
    traj_bytes = 72 * W.n_p * W.n_samples
    stream_rec = {"kernel": "k_boris (lw_trajectory_boris)", "bytes_written": traj_bytes, "ms": push_ms,
                  "GBs": traj_bytes / (push_ms / 1e3) / 1e9, "frac_of_hbm_peak":
                  traj_bytes / (push_ms / 1e3) / 1e9 / PEAK_HBM_GBS}
    log(f"[bench] Boris trajectories {W.n_p} x {W.n_samples}: {push_ms:.0f} ms, {stream_rec['GBs']:.0f} GB/s")
    diag_rec = grid.window_diagnostics(W.t_start, W.t_start + (W.n_samples - 1) * W.dt, r[:, 0].cpu().numpy(),
                                       r[:, -1].cpu().numpy(), x_det.cpu().numpy(), W.t0, W.dt_obs, n_obs,
                                       W.gamma, L.lam)
    if in_call:
        del r, b, bd
        torch.cuda.empty_cache()
    ws_f = torch.empty(lw.workspace_bytes(lw.WS_FFT, n_pix, n_obs, "mixed"), dtype=torch.uint8, device=dev)

    def deposit(prec, E, diag, ws, cull=False):
        if in_call:
            lw.deposit_td_boris(init, W.n_samples, W.t_start, W.dt, L.a0, L.lam, L.w0, L.n_cycles, x_det, W.t0,
                                W.dt_obs, n_obs, prec=prec, geom=args.geom, out=E, diag=diag, ws=ws, cull=cull)
        else:
            lw.deposit_td(r, b, bd, W.t_start, W.dt, x_det, W.t0, W.dt_obs, n_obs, prec=prec, geom=args.geom,
                          out=E, diag=diag, ws=ws, cull=cull)

    def run(prec, steps, warmup, cull=False):
        dt = torch.float64 if prec == "fp64" else torch.float32
        E = torch.empty((n_pix, 3, n_obs), dtype=dt, device=dev)
        S = torch.empty((n_pix, n_obs // 2 + 1), dtype=dt, device=dev)
        which = lw.WS_DEPOSIT_BORIS if in_call else lw.WS_DEPOSIT
        ws_d = torch.empty(lw.workspace_bytes(which, W.n_p, W.n_samples, prec), dtype=torch.uint8, device=dev)
        wsf = ws_f if prec == "mixed" else torch.empty(lw.workspace_bytes(lw.WS_FFT, n_pix, n_obs, prec),
                                                       dtype=torch.uint8, device=dev)
        diag = torch.zeros(4, dtype=torch.int64, device=dev)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        dep_ms, fft_ms = [], []
        kern_ms, kern_n = 0.0, 0
        for it in range(warmup + steps):
            if it == warmup:
                torch.cuda.synchronize()
                lw.timing_enable(True)
                t_start = time.time()
            ev[0].record()
            deposit(prec, E, diag, ws_d, cull)
            ev[1].record()
            lw.spectrum_fft(E, W.dt_obs, prec, out=S, ws=wsf)
            ev[2].record()
            if it >= warmup:
                torch.cuda.synchronize()
                ms, n = lw.timing_read(lw.KERNEL_DEPOSIT)
                kern_ms += ms
                kern_n += n
                dep_ms.append(ev[0].elapsed_time(ev[1]))
                fft_ms.append(ev[1].elapsed_time(ev[2]))
                log(f"[bench] {prec}{' culled' if cull else ''} step {it - warmup}: deposit {dep_ms[-1]:.1f} ms "
                    f"(kernel {ms:.1f} ms in {n} launches), fft {fft_ms[-1]:.1f} ms")
        torch.cuda.synchronize()
        wall = (time.time() - t_start) / steps * 1e3
        lw.timing_enable(False)
        del E, ws_d
        torch.cuda.empty_cache()
        return dict(ms_per_step=wall, deposit_ms=float(np.mean(dep_ms)), fft_ms=float(np.mean(fft_ms)),
                    kernel_ms=kern_ms / steps, launches=kern_n // steps, diag=diag.cpu().tolist(), S=S)

    mixed = run("mixed", args.steps, args.warmup)
    S_mixed = mixed.pop("S")
    out = {}
    if not args.no_fp64:
        # one all-FP64 pass of the same workload
        res64 = run("fp64", 1, 0)
        S64 = res64.pop("S")
        harmonics = range(1, 6) if name == "precision" else range(1, 2)
        out["fp64"] = {"ms_per_step": res64["ms_per_step"], "deposit_ms": res64["deposit_ms"],
                       "kernel_ms": res64["kernel_ms"], "fft_ms": res64["fft_ms"],
                       "evals_per_s": triples / (res64["ms_per_step"] / 1e3)}
        out["mixed_vs_fp64_speedup"] = res64["ms_per_step"] / mixed["ms_per_step"]
        out["mixed_vs_fp64_deposit_speedup"] = res64["deposit_ms"] / mixed["deposit_ms"]
        out["mixed_vs_fp64_band_l2_err"] = band_errors(torch, dev, W, S_mixed, S64, harmonics)
        out["diag_fp64_equal"] = res64["diag"] == mixed["diag"]
        del S64
        torch.cuda.empty_cache()
    if not args.no_cull:
        # culled variant (LW_CULL): particles whose arrivals miss a wavefront's window are
        # skipped after two arrival-time evaluations; same spectra, reported separately
        cul = run("mixed", 1, 0, cull=True)
        S_c = cul.pop("S")
        diff = float(torch.max(torch.abs(S_c - S_mixed)) / torch.max(torch.abs(S_mixed)))
        out["culled"] = {"ms_per_step": cul["ms_per_step"], "deposit_ms": cul["deposit_ms"],
                         "fft_ms": cul["fft_ms"], "evals_per_s": triples / (cul["ms_per_step"] / 1e3),
                         "diag_equal": cul["diag"] == mixed["diag"], "max_rel_diff_vs_full": diff}
        del S_c
    del S_mixed
    if not in_call:
        del r, b, bd
    torch.cuda.empty_cache()

    profiled = args.geom == "exact" and args.particles is None
    roof = deposit_roofline(triples, mixed["diag"][3], mixed["kernel_ms"] / 1e3, mixed["launches"],
                            SUMMARIES.get(name), profiled)
    fft_bytes = n_pix * (3 * n_obs + n_obs // 2 + 1) * 4
    fft_gbs = fft_bytes / (mixed["fft_ms"] / 1e3) / 1e9

    bunch = None
    if name == "precision" and not args.no_bunch:
        bunch = bunch_leg(torch, dev, args)
    grad = None
    if not args.no_grad:
        grad = grad_leg(torch, dev)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(W, args.geom, args.cpu_seconds)

    value = triples / (mixed["ms_per_step"] / 1e3)
    desc = {"precision": "precision: 1e5 e-, gamma 200, a0 1, 2e4 Boris steps pushed inside the deposit, "
                         "128x128 px, 2^18 grid",
            "bunch": "bunch: 1e4 e-, gamma 50, a0 0.5, 2e4 Boris steps (stored), 64x64 px, 2^18 grid"}[name]
    rec = {
        "metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": mixed["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64 tau + f32 field/trace/FFT", "data": "synthetic",
        "config": {"workload": desc, "n_particles": W.n_p, "n_samples": W.n_samples, "n_pix": n_pix,
                   "n_obs": n_obs, "geom": args.geom, "field": "accel", "prec": "mixed",
                   "trajectories": "pushed inside the deposit (LW_TRAJ_BORIS spans)" if in_call else "stored"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "deposit_ms": mixed["deposit_ms"], "deposit_kernel_ms": mixed["kernel_ms"], "fft_ms": mixed["fft_ms"],
        "deposit_evals_per_s": triples / (mixed["deposit_ms"] / 1e3),
        "fft": {"bound": "hbm", "algorithmic_bytes": fft_bytes, "achieved_GBs": fft_gbs,
                "frac": fft_gbs / PEAK_HBM_GBS},
        "trajectory_streaming": stream_rec,
        "grid": diag_rec,
        "diag": mixed["diag"],
        "bunch": bunch,
        "grad": grad,
        "paper_serial_evals_per_s": 1.0 / 1.02e-7,
    }
    rec.update(out)
    return rec


def bunch_leg(torch, dev, args):
    """The bunch workload (1e4 e-, 2e4 stored Boris steps, 64 x 64 px, 2^18 grid) as an extra key:
    mixed steps (deposit + FFT) with the deposit's roofline, one FP64 pass (band-L2 error of
    mixed against it) and the direct frequency-domain sum on 64 of its pixels x 4096 frequencies."""
    from paper_2206_03015_amd import grid, inputs, lw
    W = inputs.workload("bunch")
    L = W.laser
    init = torch.as_tensor(inputs.bunch_init(W), device=dev)
    r, b, bd = lw.trajectory_boris(init, W.n_samples, W.t_start, W.dt, L.a0, L.lam, L.w0, L.n_cycles)
    x_det = torch.as_tensor(inputs.pixel_positions(W.n_side, W.theta_max, W.D), device=dev)
    n_pix, n_obs = W.n_pix, W.n_obs
    triples = W.n_p * W.n_samples * n_pix
    diag_rec = grid.window_diagnostics(W.t_start, W.t_start + (W.n_samples - 1) * W.dt, r[:, 0].cpu().numpy(),
                                       r[:, -1].cpu().numpy(), x_det.cpu().numpy(), W.t0, W.dt_obs, n_obs,
                                       W.gamma, L.lam)
    res = {}
    S = {}
    for prec, steps in (("mixed", max(1, min(args.steps, 5))), ("fp64", 1)):
        dt = torch.float64 if prec == "fp64" else torch.float32
        E = torch.empty((n_pix, 3, n_obs), dtype=dt, device=dev)
        S[prec] = torch.empty((n_pix, n_obs // 2 + 1), dtype=dt, device=dev)
        ws_d = torch.empty(lw.workspace_bytes(lw.WS_DEPOSIT, W.n_p, W.n_samples, prec), dtype=torch.uint8,
                           device=dev)
        ws_f = torch.empty(lw.workspace_bytes(lw.WS_FFT, n_pix, n_obs, prec), dtype=torch.uint8, device=dev)
        diag = torch.zeros(4, dtype=torch.int64, device=dev)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        dep, fft, kern, nl = [], [], 0.0, 0
        for it in range(steps + 1):
            if it == 1:
                torch.cuda.synchronize()
                lw.timing_enable(True)
                t0 = time.time()
            ev[0].record()
            lw.deposit_td(r, b, bd, W.t_start, W.dt, x_det, W.t0, W.dt_obs, n_obs, prec=prec, geom=args.geom,
                          out=E, diag=diag, ws=ws_d)
            ev[1].record()
            lw.spectrum_fft(E, W.dt_obs, prec, out=S[prec], ws=ws_f)
            ev[2].record()
            if it >= 1:
                torch.cuda.synchronize()
                ms, n = lw.timing_read(lw.KERNEL_DEPOSIT)
                kern += ms
                nl += n
                dep.append(ev[0].elapsed_time(ev[1]))
                fft.append(ev[1].elapsed_time(ev[2]))
        torch.cuda.synchronize()
        wall = (time.time() - t0) / steps * 1e3
        lw.timing_enable(False)
        res[prec] = {"ms_per_step": wall, "deposit_ms": float(np.mean(dep)), "kernel_ms": kern / steps,
                     "launches": nl // steps, "fft_ms": float(np.mean(fft)), "diag": diag.cpu().tolist(),
                     "evals_per_s": triples / (wall / 1e3)}
        log(f"[bench] bunch {prec}: {wall:.1f} ms per step (deposit kernel {kern / steps:.1f} ms), fft "
            f"{np.mean(fft):.1f} ms")
        del E, ws_d, ws_f
        torch.cuda.empty_cache()
    m = res["mixed"]
    profiled = args.geom == "exact" and args.particles is None
    out = {"workload": "bunch: 1e4 e-, gamma 50, a0 0.5, 2e4 Boris steps (stored), 64x64 px, 2^18 grid",
           "value": m["evals_per_s"], "unit": "evals/s", "ms_per_step": m["ms_per_step"],
           "deposit_ms": m["deposit_ms"], "deposit_kernel_ms": m["kernel_ms"], "fft_ms": m["fft_ms"],
           "diag": m["diag"],
           "roofline": deposit_roofline(triples, m["diag"][3], m["kernel_ms"] / 1e3, m["launches"],
                                        SUMMARIES["bunch"], profiled),
           "fp64": res["fp64"], "mixed_vs_fp64_speedup": res["fp64"]["ms_per_step"] / m["ms_per_step"],
           "mixed_vs_fp64_band_l2_err": band_errors(torch, dev, W, S["mixed"], S["fp64"], range(1, 2)),
           "grid": diag_rec}
    fft_bytes = n_pix * (3 * n_obs + n_obs // 2 + 1) * 4
    out["fft"] = {"achieved_GBs": fft_bytes / (m["fft_ms"] / 1e3) / 1e9,
                  "frac": fft_bytes / (m["fft_ms"] / 1e3) / 1e9 / PEAK_HBM_GBS}
    del S
    torch.cuda.empty_cache()
    if not args.no_fd:
        out["direct_fd"] = fd_leg(torch, dev, W, r, b, bd, x_det, m["ms_per_step"], args.geom)
    del r, b, bd
    torch.cuda.empty_cache()
    return out


def det_leg(torch, dev, reps=2):
    """The bunch workload (1e4 e-, 2e4 stored Boris steps, 64 x 64 px, 2^18 grid), FP64: the
    atomics-order deposit against the order-independent one.  Each is run `reps` times after a
    warm-up; reported: mean wall time of a call, whether its outputs are bit-identical across the
    runs (and how many elements differ), and max |E_det - E_fp64| / max |E_fp64|."""
    from paper_2206_03015_amd import inputs, lw
    W = inputs.workload("bunch")
    L = W.laser
    init = torch.as_tensor(inputs.bunch_init(W), device=dev)
    r, b, bd = lw.trajectory_boris(init, W.n_samples, W.t_start, W.dt, L.a0, L.lam, L.w0, L.n_cycles)
    x_det = torch.as_tensor(inputs.pixel_positions(W.n_side, W.theta_max, W.D), device=dev)
    n_pix, n_obs = W.n_pix, W.n_obs
    ws = torch.empty(lw.workspace_bytes(lw.WS_DEPOSIT, W.n_p, W.n_samples, "fp64"), dtype=torch.uint8, device=dev)
    acc = torch.empty(lw.workspace_bytes(lw.WS_DEPOSIT_DET_ACC, n_pix, n_obs, "fp64"), dtype=torch.uint8,
                      device=dev)
    E = [torch.empty((n_pix, 3, n_obs), dtype=torch.float64, device=dev) for _ in range(2)]
    calls = {
        "fp64": lambda o: lw.deposit_td(r, b, bd, W.t_start, W.dt, x_det, W.t0, W.dt_obs, n_obs, prec="fp64", out=o,
                                        ws=ws),
        "det": lambda o: lw.deposit_td_det(r, b, bd, W.t_start, W.dt, x_det, W.t0, W.dt_obs, n_obs, out=o, ws=ws,
                                           acc=acc),
    }
    res = {"workload": "bunch", "n_particles": W.n_p, "n_samples": W.n_samples, "n_pix": n_pix, "n_obs": n_obs}
    ref = None
    for name, fn in calls.items():
        fn(E[0])
        ms = []
        for i in range(reps):
            torch.cuda.synchronize()
            t0 = time.time()
            fn(E[i % 2])
            torch.cuda.synchronize()
            ms.append((time.time() - t0) * 1e3)
        a, c = E[0].view(torch.int64), E[1].view(torch.int64)
        res[name] = {"ms": float(np.mean(ms)), "bit_identical": bool(torch.equal(a, c)),
                     "elements_differing": int((a != c).sum())}
        log(f"[bench] det leg, {name}: {res[name]['ms']:.1f} ms per call, runs bit-identical "
            f"{res[name]['bit_identical']} ({res[name]['elements_differing']} of {a.numel()} elements differ)")
        if ref is None:
            ref = E[0].clone()
        else:
            res["max_rel_diff_det_vs_fp64"] = float((E[0] - ref).abs().max() / ref.abs().max())
    res["det_over_fp64"] = res["det"]["ms"] / res["fp64"]["ms"]
    return res


def fd_leg(torch, dev, W, r, b, bd, x_det, td_ms_per_step, geom, n_fd_pix=64, n_w=4096):
    """Direct frequency-domain sum (comparison path) on n_fd_pix evenly spaced pixels x n_w
    FFT-bin frequencies of the first-harmonic band, mixed precision."""
    from paper_2206_03015_amd import lw
    n_pix, n_obs = W.n_pix, W.n_obs
    sel = torch.arange(0, n_pix, n_pix // n_fd_pix, device=dev)[:n_fd_pix]
    w1 = W.omega1()
    dw = 2 * np.pi / (n_obs * W.dt_obs)
    j0 = int(0.7 * w1 / dw)
    jstep = max(1, int((0.4 * w1 / dw) / n_w))
    omega = torch.as_tensor((j0 + jstep * np.arange(n_w)) * dw, device=dev)
    xs = x_det[sel].contiguous()
    ws_fd = torch.empty(lw.workspace_bytes(lw.WS_DIRECT_FD, n_fd_pix, n_w, "mixed"), dtype=torch.uint8, device=dev)
    Sfd = torch.empty((n_fd_pix, n_w), dtype=torch.float64, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    lw.direct_fd(r[:64], b[:64], bd[:64], W.t_start, W.dt, xs, W.t0, omega, prec="mixed", geom=geom, out=Sfd,
                 ws=ws_fd)
    torch.cuda.synchronize()
    e0.record()
    lw.direct_fd(r, b, bd, W.t_start, W.dt, xs, W.t0, omega, prec="mixed", geom=geom, out=Sfd, ws=ws_fd)
    e1.record()
    torch.cuda.synchronize()
    fd_ms = e0.elapsed_time(e1)
    terms = W.n_p * W.n_samples * n_fd_pix * n_w
    fd_per_pix_bin = fd_ms / (n_fd_pix * n_w)
    td_per_pix_bin = td_ms_per_step / (n_pix * (n_obs // 2 + 1))
    fd_tflops = terms * FD_TERM_FLOPS / (fd_ms / 1e3) / 1e12
    log(f"[bench] direct FD {n_fd_pix} pix x {n_w} w: {fd_ms:.1f} ms")
    return {"pixels": n_fd_pix, "n_omega": n_w, "ms": fd_ms, "terms_per_s": terms / (fd_ms / 1e3),
            "td_speedup_per_pixel_bin": fd_per_pix_bin / td_per_pix_bin,
            "roofline": {"bound": "alu", "achieved": fd_tflops, "peak": PEAK_F32_TFLOPS, "unit": "TFLOP/s",
                         "frac": fd_tflops / PEAK_F32_TFLOPS, "flops_per_term": FD_TERM_FLOPS}}


def fit_leading_constant(sweeps):
    """The paper's fit of a wall-clock model t = C * x (x: the product of the sizes): one
    least-squares constant per single-variate sweep, C = sum(x t)/sum(x^2), then their mean.
    sweeps: {name: [(x, t), ...]}.  Returns (C, {name: C_name})."""
    per = {}
    for name, pts in sweeps.items():
        x = np.array([p[0] for p in pts], dtype=float)
        t = np.array([p[1] for p in pts], dtype=float)
        per[name] = float(np.dot(x, t) / np.dot(x, x))
    return float(np.mean(list(per.values()))), per


def crossover(n_p, t_td, t_fd):
    """Smallest particle count from which the time-domain method is faster than the
    frequency-domain one for every larger count measured (None if it never is)."""
    n_p, t_td, t_fd = (np.asarray(v, dtype=float) for v in (n_p, t_td, t_fd))
    order = np.argsort(n_p)
    n_p, faster = n_p[order], (t_td < t_fd)[order]
    for i in range(len(n_p)):
        if faster[i:].all():
            return float(n_p[i])
    return None


def _timed(torch, fn, reps=5, warmup=2):
    """Median wall time (s) of fn() on the current stream, HIP events around each call."""
    for _ in range(warmup):
        fn()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    return float(np.median(ts))


def cost_model(torch, dev):
    """GPU refit of the wall-clock model of Sec. "Performance" (time-domain W1_t = C1_t N_s N_p
    N_obs and W2_t = C2_t N_obs N_Tu log2 N_Tu, frequency-domain W_w = C_w N_s N_p N_obs N_w)
    by single-variate sweeps around a base point sized for the GPU, and the TD/FD crossover
    experiment (100 um uniform bunch, 5 periods of a 1 um plane wave, N_s = 100, one observer,
    N_Tu = 2^20, N_w = 100).  Mixed precision, exact geometry, acceleration field."""
    from paper_2206_03015_amd import inputs, lw
    out = {"metric": "wall-clock model constants (s per unit of the model)", "prec": "mixed", "geom": "exact"}
    base = inputs.workload("bunch")
    L = base.laser

    def bunch(n_p, n_steps, n_side):
        W = base.scaled(n_p=n_p, n_steps=n_steps, n_side=n_side)
        init = torch.as_tensor(inputs.bunch_init(W), device=dev)
        r, b, bd = lw.trajectory_boris(init, W.n_samples, W.t_start, W.dt, L.a0, L.lam, L.w0, L.n_cycles)
        x = torch.as_tensor(inputs.pixel_positions(W.n_side, W.theta_max, W.D), device=dev)
        return W, r, b, bd, x

    # ---- W1_t: deposit time; base 1000 particles x 20001 samples x 32 x 32 pixels, 2^18 grid
    sw1 = {"N_s": [], "N_p": [], "N_obs": []}
    pts = [("N_s", 1000, s_, 32) for s_ in (5000, 10000, 20000, 40000)] + \
          [("N_p", p_, 20000, 32) for p_ in (250, 500, 1000, 2000)] + \
          [("N_obs", 1000, 20000, n_) for n_ in (16, 23, 32, 45)]
    for name, n_p, n_steps, n_side in pts:
        W, r, b, bd, x = bunch(n_p, n_steps, n_side)
        E = torch.empty((W.n_pix, 3, W.n_obs), dtype=torch.float32, device=dev)
        ws = torch.empty(lw.workspace_bytes(lw.WS_DEPOSIT, W.n_p, W.n_samples, "mixed"), dtype=torch.uint8,
                         device=dev)
        t = _timed(torch, lambda: lw.deposit_td(r, b, bd, W.t_start, W.dt, x, W.t0, W.dt_obs, W.n_obs,
                                               prec="mixed", out=E, ws=ws))
        sw1[name].append((W.n_samples * W.n_p * W.n_pix, t))
        log(f"[cost] W1 {name}: N_s={W.n_samples} N_p={W.n_p} N_obs={W.n_pix}: {t * 1e3:.2f} ms")
        del E, ws, r, b, bd
    c1, c1_per = fit_leading_constant(sw1)

    # ---- W2_t: FFT time; base 1024 pixels x 2^18 points
    sw2 = {"N_obs": [], "N_Tu": []}
    for name, n_pix, lg in [("N_obs", n_, 18) for n_ in (256, 512, 1024, 2048)] + \
                           [("N_Tu", 1024, lg_) for lg_ in (16, 17, 18, 19, 20)]:
        n_obs = 1 << lg
        E = torch.randn((n_pix, 3, n_obs), dtype=torch.float32, device=dev)
        S = torch.empty((n_pix, n_obs // 2 + 1), dtype=torch.float32, device=dev)
        ws = torch.empty(lw.workspace_bytes(lw.WS_FFT, n_pix, n_obs, "mixed"), dtype=torch.uint8, device=dev)
        t = _timed(torch, lambda: lw.spectrum_fft(E, 1e-20, "mixed", out=S, ws=ws))
        sw2[name].append((n_pix * n_obs * math.log2(n_obs), t))
        log(f"[cost] W2 {name}: N_obs={n_pix} N_Tu=2^{lg}: {t * 1e3:.3f} ms")
        del E, S, ws
    c2, c2_per = fit_leading_constant(sw2)

    # ---- W_w: direct FD time; base 100 particles x 2001 samples x 8 pixels x 1024 frequencies
    sww = {"N_s": [], "N_p": [], "N_obs": [], "N_w": []}
    pts = [("N_s", 100, s_, 8, 1024) for s_ in (1000, 2000, 4000, 8000)] + \
          [("N_p", p_, 2000, 8, 1024) for p_ in (50, 100, 200, 400)] + \
          [("N_obs", 100, 2000, n_, 1024) for n_ in (4, 8, 16, 32)] + \
          [("N_w", 100, 2000, 8, w_) for w_ in (256, 512, 1024, 2048)]
    for name, n_p, n_steps, n_pix, n_w in pts:
        W, r, b, bd, x = bunch(n_p, n_steps, 8)
        xs = x[:n_pix].contiguous()
        w1 = W.omega1()
        omega = torch.as_tensor(np.linspace(0.7 * w1, 1.1 * w1, n_w), device=dev)
        ws = torch.empty(lw.workspace_bytes(lw.WS_DIRECT_FD, n_pix, n_w, "mixed"), dtype=torch.uint8, device=dev)
        Sfd = torch.empty((n_pix, n_w), dtype=torch.float64, device=dev)
        t = _timed(torch, lambda: lw.direct_fd(r, b, bd, W.t_start, W.dt, xs, W.t0, omega, prec="mixed",
                                              out=Sfd, ws=ws))
        sww[name].append((W.n_samples * W.n_p * n_pix * n_w, t))
        log(f"[cost] Ww {name}: N_s={W.n_samples} N_p={W.n_p} N_obs={n_pix} N_w={n_w}: {t * 1e3:.3f} ms")
        del ws, Sfd, r, b, bd
    cw, cw_per = fit_leading_constant(sww)
    out["constants"] = {"C1_t": c1, "C2_t": c2, "C_w": cw, "log": "log2",
                        "per_sweep": {"C1_t": c1_per, "C2_t": c2_per, "C_w": cw_per},
                        "paper_cpu_serial": {"C1_t": 1.02e-7, "C2_t": 8.61e-9, "C_w": 1.17e-7}}

    # ---- crossover: 100 um uniform line bunch, 5 periods of a 1 um plane wave, N_s = 100
    gamma, a0, n_cycles, lb = 5.0, 0.5, 5.0, 100e-6
    n_steps, n_obs, n_w = 100, 1 << 20, 100
    t_sim = (lb + n_cycles * L.lam) / (2.0 * inputs.C_LIGHT)
    t_start, dt = -0.5 * t_sim, t_sim / n_steps
    x1 = torch.as_tensor(np.array([[0.0, 0.0, base.D]]), device=dev)
    rows = []
    for n_p in (1, 2, 5, 10, 20, 40, 80, 160, 320, 640, 1280, 2560, 5120):
        init = torch.as_tensor(inputs.uniform_line_init(n_p, lb, gamma, t_start), device=dev)
        r, b, bd = lw.trajectory_boris(init, n_steps + 1, t_start, dt, a0, L.lam, 0.0, n_cycles)
        # observer window: the whole arrival-time span on axis, N_Tu points
        span = (t_sim * (1.0 + a0 * a0 / 2.0) / (4 * gamma * gamma) + lb / inputs.C_LIGHT)
        dt_obs = 1.2 * span / n_obs
        t0 = -0.6 * span
        E = torch.empty((1, 3, n_obs), dtype=torch.float32, device=dev)
        S = torch.empty((1, n_obs // 2 + 1), dtype=torch.float32, device=dev)
        ws_d = torch.empty(lw.workspace_bytes(lw.WS_DEPOSIT, n_p, n_steps + 1, "mixed"), dtype=torch.uint8,
                           device=dev)
        ws_f = torch.empty(lw.workspace_bytes(lw.WS_FFT, 1, n_obs, "mixed"), dtype=torch.uint8, device=dev)
        w1 = 4 * gamma ** 2 * 2 * np.pi * inputs.C_LIGHT / L.lam / (1 + a0 * a0 / 2)
        omega = torch.as_tensor(np.linspace(0.5 * w1, 1.5 * w1, n_w), device=dev)
        ws_w = torch.empty(lw.workspace_bytes(lw.WS_DIRECT_FD, 1, n_w, "mixed"), dtype=torch.uint8, device=dev)
        Sfd = torch.empty((1, n_w), dtype=torch.float64, device=dev)

        def td():
            lw.deposit_td(r, b, bd, t_start, dt, x1, t0, dt_obs, n_obs, prec="mixed", out=E, ws=ws_d)
            lw.spectrum_fft(E, dt_obs, "mixed", out=S, ws=ws_f)

        def fd():
            lw.direct_fd(r, b, bd, t_start, dt, x1, t0, omega, prec="mixed", out=Sfd, ws=ws_w)

        t_td, t_fd = _timed(torch, td, reps=21), _timed(torch, fd, reps=21)
        rows.append((n_p, t_td, t_fd))
        log(f"[cost] crossover N_p={n_p}: TD {t_td * 1e6:.1f} us, FD {t_fd * 1e6:.1f} us")
    out["crossover"] = {"setup": "100 um uniform line bunch, gamma 5, plane wave a0 0.5, 5 periods of 1 um, "
                                 "N_s 100, one on-axis observer, TD N_Tu 2^20, FD N_w 100",
                        "n_p": [x[0] for x in rows], "td_s": [x[1] for x in rows], "fd_s": [x[2] for x in rows],
                        "td_faster_from_n_p": crossover(*zip(*rows)), "paper_cpu_serial_td_faster_from_n_p": 41}
    return out


def full_size(torch, dev, name):
    """One full-size pass of the precision or large workload: deposit with the trajectories
    recomputed batch by batch inside the call (LW_TRAJ_BORIS: 1e5 electrons x 2e4 steps would
    need 144 GB stored), then FFT, in mixed precision and in FP64; the band-L2 error of mixed
    against FP64 in the harmonic bands [(h - 0.3) w1, (h + 0.1) w1] of every pixel (h = 1..5 for
    the precision workload, h = 1 otherwise).  Reports evaluations per second of each pass."""
    from paper_2206_03015_amd import inputs, lw
    W = inputs.workload(name)
    L = W.laser
    init = torch.as_tensor(inputs.bunch_init(W), device=dev)
    x = torch.as_tensor(inputs.pixel_positions(W.n_side, W.theta_max, W.D), device=dev)
    triples = W.n_p * W.n_samples * W.n_pix
    args = (W.n_samples, W.t_start, W.dt, L.a0, L.lam, L.w0, L.n_cycles, x, W.t0, W.dt_obs, W.n_obs)
    out = {"workload": name, "n_particles": W.n_p, "n_samples": W.n_samples, "n_pix": W.n_pix, "n_obs": W.n_obs}
    S = {}
    for prec in ("mixed", "fp64"):
        torch.cuda.synchronize()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        E, diag = lw.deposit_td_boris(init, *args, prec=prec)
        e[1].record()
        S[prec] = lw.spectrum_fft(E, W.dt_obs, prec)
        e[2].record()
        torch.cuda.synchronize()
        dep_ms, fft_ms = e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])
        out[prec] = {"deposit_ms": dep_ms, "fft_ms": fft_ms, "evals_per_s": triples / (dep_ms / 1e3),
                     "diag": diag.cpu().tolist()}
        log(f"[{name}] {prec}: deposit {dep_ms:.0f} ms ({triples / dep_ms * 1e3:.3e} evals/s), fft {fft_ms:.1f} ms")
        del E
        torch.cuda.empty_cache()
    tx, ty = inputs.pixel_angles(W.n_side, W.theta_max)
    th = torch.as_tensor(np.hypot(tx, ty), device=dev)
    w1 = torch.as_tensor(np.array([W.omega1(t) for t in np.hypot(tx, ty)]), device=dev)[:, None]
    wgrid = torch.as_tensor(2 * np.pi * np.arange(W.n_obs // 2 + 1) / (W.n_obs * W.dt_obs), device=dev)
    harmonics = range(1, 6) if name == "precision" else range(1, 2)
    out["band_l2_err"] = {}
    for h in harmonics:
        errs = []
        for m0 in range(0, W.n_pix, 512):
            m1 = min(W.n_pix, m0 + 512)
            band = (wgrid[None, :] >= (h - 0.3) * w1[m0:m1]) & (wgrid[None, :] <= (h + 0.1) * w1[m0:m1])
            a = S["mixed"][m0:m1].double() * band
            b = S["fp64"][m0:m1] * band
            den = torch.linalg.vector_norm(b, dim=1)
            ok = den > 0
            errs.append((torch.linalg.vector_norm(a - b, dim=1)[ok] / den[ok]).cpu().numpy())
        errs = np.concatenate(errs)
        out["band_l2_err"][f"h{h}"] = {"max": float(errs.max()), "median": float(np.median(errs)),
                                      "pixels": int(errs.size)}
        log(f"[{name}] h={h}: band L2 mixed vs FP64 max {errs.max():.2e} median {np.median(errs):.2e} "
            f"over {errs.size} pixels")
    del th
    out["mixed_vs_fp64_deposit_speedup"] = out["fp64"]["deposit_ms"] / out["mixed"]["deposit_ms"]
    del S
    torch.cuda.empty_cache()
    if name == "large":
        out["adjoint"] = full_size_adjoint(torch, dev, W, init)
    return out


def full_size_adjoint(torch, dev, W, init):
    """Adjoint of a band objective on the large workload at full size: J = sum over the central
    8 x 8 pixels of the first-harmonic band energy (+-2 % of w1, reading of the differentiation
    objective), dJ/d(init, a0) through the FFT adjoint, the deposit adjoint and the pusher's
    tangents with the trajectories recomputed in the call (FP64), checked against a central
    difference in a0 (step 1e-6 a0)."""
    from paper_2206_03015_amd import inputs, lw
    L = W.laser
    cen = inputs.central_pixels(W.n_side, 8)
    xc_np = inputs.pixel_positions(W.n_side, W.theta_max, W.D)[cen]
    xc = torch.as_tensor(np.ascontiguousarray(xc_np), device=dev)
    wts = torch.as_tensor(inputs.band_weights(W, xc_np), device=dev)

    def objective(a0):
        E, diag = lw.deposit_td_boris(init, W.n_samples, W.t_start, W.dt, a0, L.lam, L.w0, L.n_cycles, xc, W.t0,
                                      W.dt_obs, W.n_obs, prec="fp64")
        S = lw.spectrum_fft(E, W.dt_obs, "fp64")
        return E, float(torch.sum(wts * S)), diag

    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    e[0].record()
    E, J, diag = objective(L.a0)
    e[1].record()
    dE = lw.spectrum_fft_bwd(E, wts, W.dt_obs, "fp64")
    lw.timing_enable(True)
    e[2].record()
    g_init, g_a0 = lw.deposit_td_bwd_boris(init, W.n_samples, W.t_start, W.dt, L.a0, L.lam, L.w0, L.n_cycles, xc,
                                           W.t0, W.dt_obs, W.n_obs, dE)
    e[3].record()
    torch.cuda.synchronize()
    bwd_ms, bwd_n = lw.timing_read(lw.KERNEL_DEPOSIT_BWD)
    tan_ms, tan_n = lw.timing_read(lw.KERNEL_BORIS_TANGENT)
    lw.timing_enable(False)
    dj_da0 = float(torch.sum(g_a0))
    points = int(diag.cpu()[3])
    del E, dE
    h = 1e-6 * L.a0
    _, Jp, _ = objective(L.a0 + h)
    _, Jm, _ = objective(L.a0 - h)
    fd = (Jp - Jm) / (2 * h)
    # the sample-gradient kernel on the work it performs (FP64 only)
    triples = W.n_p * W.n_samples * len(cen)
    work = ADJ_TRIPLE_F64_FLOPS * triples + ADJ_POINT_F64_FLOPS * points
    t_roof = work / (PEAK_F64_TFLOPS * 1e12)
    roof = {"bound": "alu", "kernel": "k_deposit_bwd", "launches": bwd_n, "kernel_ms": bwd_ms,
            "achieved": work / (bwd_ms / 1e3) / 1e12, "peak": PEAK_F64_TFLOPS, "unit": "TFLOP/s",
            "frac": t_roof / (bwd_ms / 1e3),
            "work": {"f64_flops": work, "triples": triples, "deposited_points": points,
                     "f64_flops_per_triple": ADJ_TRIPLE_F64_FLOPS, "f64_flops_per_deposited_point": ADJ_POINT_F64_FLOPS}}
    rec = {"pixels": int(len(cen)), "J": J, "dJ_da0": dj_da0, "dJ_da0_central_difference": fd,
           "rel_diff": abs(dj_da0 - fd) / abs(fd), "forward_ms": e[0].elapsed_time(e[1]),
           "fft_bwd_ms": e[1].elapsed_time(e[2]), "deposit_boris_bwd_ms": e[2].elapsed_time(e[3]),
           "deposit_bwd_kernel_ms": bwd_ms, "boris_tangent_kernel_ms": tan_ms, "tangent_launches": tan_n,
           "deposit_bwd_roofline": roof, "grad_init_norm": float(torch.linalg.vector_norm(g_init))}
    log(f"[large] adjoint kernels: k_deposit_bwd {bwd_ms:.0f} ms in {bwd_n} launches (roofline fraction "
        f"{roof['frac']:.3f}), k_boris_tangent_span {tan_ms:.0f} ms in {tan_n} launches")
    log(f"[large] adjoint on {len(cen)} pixels: forward {rec['forward_ms']:.0f} ms, FFT adjoint "
        f"{rec['fft_bwd_ms']:.1f} ms, deposit+pusher adjoint {rec['deposit_boris_bwd_ms']:.0f} ms; dJ/da0 "
        f"{dj_da0:.6e} vs central difference {fd:.6e} (rel {rec['rel_diff']:.1e})")
    return rec


def spectra_error(S, S_ref):
    """Eq. spectra_error: |S - S_ref| / max(S_ref) over every (observer, frequency); returns its
    maximum and mean."""
    S, S_ref = np.asarray(S, dtype=float), np.asarray(S_ref, dtype=float)
    e = np.abs(S - S_ref) / np.max(S_ref)
    return float(e.max()), float(e.mean())


def accuracy_setup(torch, dev, n_theta=101, n_s=20000):
    """Inputs of the accuracy experiment (Sec. "Accuracy"): one electron (gamma 5) along +z
    through 7 periods of a counter-propagating 1 um plane wave (sin^2 envelope, a0 = 0.5), its
    FP64 Boris trajectory of n_s steps on the device, n_theta observers in the y-z plane over
    +-2/gamma at 1 m, w_max = 3 w1(0) and dt_obs = pi/w_max (N_Tu = 2 N_w: the FFT bins are
    j w_max/N_w), and an observer-window origin before the earliest arrival."""
    from paper_2206_03015_amd import inputs, lw
    c = inputs.C_LIGHT
    gamma, a0, lam, n_cycles = 5.0, 0.5, 1e-6, 7.0
    theta_max, D = 2.0 / gamma, 1.0
    t_sim = 1.05 * n_cycles * lam / (2.0 * c)
    t_start = -0.5 * t_sim
    uz = math.sqrt(gamma * gamma - 1.0)
    z0 = uz / gamma * c * t_start
    init = torch.as_tensor(np.array([[0.0, 0.0, z0, 0.0, 0.0, uz]]), device=dev)
    th = np.linspace(-theta_max, theta_max, n_theta)
    xd = np.stack([np.zeros_like(th), np.sin(th), np.cos(th)], axis=-1) * D
    w_l = 2.0 * np.pi * c / lam
    w1 = 4.0 * gamma ** 2 * w_l / (1.0 + 0.5 * a0 * a0)
    w_max = 3.0 * w1
    dt_obs = np.pi / w_max
    t_first = t_start - np.cos(th) * z0 / c
    t0 = float(np.min(t_first)) - 16.0 * dt_obs

    def traj(n):
        dt = t_sim / (n - 1)
        return dt, lw.trajectory_boris(init, n, t_start, dt, a0, lam, 0.0, n_cycles)

    return dict(gamma=gamma, a0=a0, lam=lam, n_cycles=n_cycles, t_start=t_start, t_sim=t_sim, theta=th,
                x_det=torch.as_tensor(xd, device=dev), w_max=w_max, dt_obs=dt_obs, t0=t0, traj=traj, n_s=n_s)


def accuracy(torch, dev):
    """The accuracy experiment of Sec. "Accuracy" (set-up of accuracy_setup): the time-domain
    spectra (FP64 Boris trajectory of 2e4 steps -> deposit on N_Tu = 2 N_w grid points -> FFT) and
    the direct frequency-domain sum at the same N_w + 1 bins (same trajectory) are compared with
    a converged reference: the FP64 direct sum over a 16x finer Boris trajectory (its distance to
    the 8x one is reported).  N_w in {4096, 8192, 16384} (the paper's 5e3, 1e4, 2e4 rounded to
    powers of two for the FFT).  At N_w = 4096 the time-domain spectra are also taken on 2x, 4x
    and 8x finer observer grids (the same bins)."""
    from paper_2206_03015_amd import lw
    A = accuracy_setup(torch, dev)
    gamma, a0, lam, n_cycles, t_start = A["gamma"], A["a0"], A["lam"], A["n_cycles"], A["t_start"]
    x, w_max, dt_obs, t0, n_s, fine = A["x_det"], A["w_max"], A["dt_obs"], A["t0"], A["n_s"], 16
    n_theta = x.shape[0]
    dt, (r, b, bd) = A["traj"](n_s + 1)
    dtf, (rf, bf, bdf) = A["traj"](fine * n_s + 1)
    dth, (rh, bh, bdh) = A["traj"](fine // 2 * n_s + 1)
    rows = []
    for n_w in (4096, 8192, 16384):
        n_obs = 2 * n_w
        omega = torch.as_tensor(np.arange(n_w + 1) * (w_max / n_w), device=dev)
        S_td = {}
        for prec in ("fp64", "mixed"):
            E, diag = lw.deposit_td(r, b, bd, t_start, dt, x, t0, dt_obs, n_obs, prec=prec)
            S_td[prec] = lw.spectrum_fft(E, dt_obs, prec).double().cpu().numpy()
            d = diag.cpu().numpy()
            assert d[0] == 0 and d[1] == 0 and d[2] == 0, d  # whole pulse inside the window
        S_fd = lw.direct_fd(r, b, bd, t_start, dt, x, t0, omega, prec="fp64").cpu().numpy()
        S_ref = lw.direct_fd(rf, bf, bdf, t_start, dtf, x, t0, omega, prec="fp64").cpu().numpy()
        S_half = lw.direct_fd(rh, bh, bdh, t_start, dth, x, t0, omega, prec="fp64").cpu().numpy()
        rec = {"n_omega": n_w, "n_tu": n_obs}
        for name, S in (("td", S_td["fp64"]), ("td_mixed", S_td["mixed"]), ("fd", S_fd), ("ref_8x", S_half)):
            mx, mean = spectra_error(S, S_ref)
            rec[name] = {"max": mx, "mean": mean}
        if n_w == 4096:
            # finer observer grids (the same bins): TD error against grid points per period
            rec["td_finer_grid"] = []
            for f in (2, 4, 8):
                E, _ = lw.deposit_td(r, b, bd, t_start, dt, x, t0, dt_obs / f, f * n_obs, prec="fp64")
                S = lw.spectrum_fft(E, dt_obs / f, "fp64").cpu().numpy()[:, : n_w + 1]
                mx, mean = spectra_error(S, S_ref)
                rec["td_finer_grid"].append({"factor": f, "n_tu": f * n_obs, "max": mx, "mean": mean})
                log(f"[accuracy] N_w={n_w}, grid x{f}: TD max {mx:.3e} mean {mean:.3e}")
        rows.append(rec)
        log(f"[accuracy] N_w={n_w}: TD max {rec['td']['max']:.3e} mean {rec['td']['mean']:.3e}; "
            f"FD max {rec['fd']['max']:.3e} mean {rec['fd']['mean']:.3e}; ref 8x vs 16x {rec['ref_8x']['max']:.1e}")
    return {"metric": "Eq. spectra_error against a converged FP64 FD reference",
            "setup": {"gamma": gamma, "a0": a0, "lambda_m": lam, "periods": n_cycles, "envelope": "sin^2",
                      "observers": f"{n_theta} in the y-z plane over +-2/gamma at 1 m", "n_steps": n_s,
                      "reference_steps": fine * n_s, "w_max_over_w1": 3.0, "dt_obs_s": dt_obs},
            "rows": rows,
            "paper_table_nw": {"td_max": [0.1287, 0.1290, 0.1291], "td_mean": [3.520e-3, 3.522e-3, 3.524e-3],
                               "fd_max": [5.366e-2] * 3, "fd_mean": [1.589e-3, 1.589e-3, 1.580e-3]}}


def grad_leg(torch, dev):
    """d(band energy)/d(gamma_mean, a0) on the differentiation workload (1e3 e-, 1e4 steps, 32 x 32
    pixels, 2^16 grid, objective over the central 8 x 8 pixels): seeded draw -> FP64 Boris ->
    deposit -> FFT forward, then the three adjoints, through torch.autograd."""
    from paper_2206_03015_amd import autograd as ag
    from paper_2206_03015_amd import inputs
    W = inputs.workload("grad")
    x = inputs.pixel_positions(W.n_side, W.theta_max, W.D)
    weights = torch.as_tensor(inputs.band_weights(W, x, inputs.central_pixels(W.n_side, 8)), device=dev)
    x_det = torch.as_tensor(x, device=dev)

    def once():
        gamma = torch.tensor(W.gamma, dtype=torch.float64, requires_grad=True)
        a0 = torch.tensor(W.laser.a0, dtype=torch.float64, requires_grad=True)
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        init = ag.bunch_init(W, None, gamma, device=dev)
        r, b, bd = ag.boris_trajectory(init, a0, W)
        S, _ = ag.lw_spectrum(r, b, bd, W.t_start, W.dt, x_det, W.t0, W.dt_obs, W.n_obs, prec="fp64")
        J = torch.sum(weights * S)
        e[1].record()
        J.backward()
        e[2].record()
        torch.cuda.synchronize()
        return float(J.detach()), float(gamma.grad), float(a0.grad), e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])

    once()
    J, dg, da, fwd_ms, bwd_ms = once()
    log(f"[bench] grad: forward {fwd_ms:.1f} ms, backward {bwd_ms:.1f} ms, dJ/dgamma {dg:.4e}, dJ/da0 {da:.4e}")
    return {"workload": "grad: 1e3 e-, 1e4 Boris steps, 32x32 px, 2^16 grid, band objective on the central 8x8",
            "J": J, "dJ_dgamma": dg, "dJ_da0": da, "forward_ms": fwd_ms, "backward_ms": bwd_ms,
            "forward_evals_per_s": W.n_p * W.n_samples * W.n_pix / (fwd_ms / 1e3), "prec": "fp64"}


def _deposit_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in DEPOSIT_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _profile_figures(path):
    """The "- key: `value`" figures of a committed rocprofv3 summary, or None when the deposit
    sources changed since its counters were taken."""
    path = os.path.join(ROOT, path)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.startswith("- "):
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha256") != _deposit_source_hash():
        return None
    return vals


def _summary_value(path, key):
    """One "- key: `value`" figure of a committed rocprofv3 summary (None when absent or when the
    deposit sources changed since its counters were taken)."""
    vals = _profile_figures(path)
    try:
        return float(vals[key]) if vals else None
    except (KeyError, ValueError):
        return None


def cpu_baseline(W, geom, seconds):
    """FP64 oracle (OpenMP over pixels) on a pixel subset x particle subset of the same workload,
    trajectories from the oracle's own Boris pusher.  Sized to ~``seconds`` of CPU work."""
    import oracle
    from paper_2206_03015_amd import inputs
    L = W.laser
    g = oracle.GEOM_EXACT if geom == "exact" else oracle.GEOM_FARFIELD
    init = inputs.bunch_init(W)
    x = inputs.pixel_positions(W.n_side, W.theta_max, W.D)
    n_pix = 64
    xs = np.ascontiguousarray(x[:: max(1, W.n_pix // n_pix)][:n_pix])

    def timed(n_p):
        rr, bb, aa = oracle.boris(init[:n_p], W.n_samples, W.t_start, W.dt, L.a0, L.lam, L.w0, L.n_cycles)
        t0 = time.time()
        oracle.deposit_td(W.t_start, W.dt, rr, bb, aa, xs, W.t0, W.dt_obs, W.n_obs, geom=g)
        return time.time() - t0

    # time = a + b n_p (the fixed part is the zeroed trace and thread start-up): two small
    # calibration runs fix a and b, then the sample is sized to `seconds`
    t4, t16 = timed(4), timed(16)
    b = max((t16 - t4) / 12.0, 1e-6)
    a = max(t4 - 4 * b, 0.0)
    n_p = int(max(16, min(W.n_p, (seconds - a) / b)))
    t = timed(n_p)
    triples = n_p * W.n_samples * n_pix
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    cores = min(cores, os.cpu_count() or cores, n_pix)
    log(f"[bench] cpu oracle: {n_p} particles x {W.n_samples} samples x {n_pix} pixels in {t:.1f} s")
    return {"value": triples / t, "unit": "evals/s", "cores": cores, "kind": "oracle",
            "sample": f"{n_p} particles x {W.n_samples} samples x {n_pix} pixels of the {W.name} workload "
                      f"(FP64 deposit only, trajectories from the oracle's pusher untimed, {t:.1f} s)"}


if __name__ == "__main__":
    sys.exit(main())
