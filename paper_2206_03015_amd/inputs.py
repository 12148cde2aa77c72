"""Seeded synthetic inputs for the time-domain Lienard-Wiechert path.

This module holds none of the method's arithmetic: it draws particle phase
space with a fixed seed, fixes laser pulse and detector parameters, and
chooses the simulation window and the observer grid.  Both the HIP path and the
CPU oracle take their inputs from here; neither is imported by it.

Workloads (sizes of the paper's inverse-Compton-scattering setting, Sec. 1 and
Table 2 ranges; electron along +z, laser along -z, collision at t = 0, z = 0):

* ``single``   one electron, gamma = 50, plane-wave pulse a0 = 0.1, lambda = 1 um,
               20 cycles, 2e4 steps, one on-axis pixel at 1 m, 2^16 grid points.
* ``bunch``    1e4 electrons, gamma = 50 (sigma_gamma/gamma = 1e-3), sigma_x,y = 2 um,
               sigma_z = 5 um, eps_n = 1 mm mrad; Gaussian pulse a0 = 0.5,
               w0 = 10 um, 20 cycles; 2e4 Boris steps; 64 x 64 pixels over +-1/gamma;
               2^18 grid points.
* ``precision`` gamma = 200, a0 = 1, 1e5 electrons, 128 x 128 pixels over +-2/gamma.
* ``grad``     1e3 electrons (bunch distributions), 1e4 steps, 32 x 32 pixels, 2^16.
* ``large``    1e5 electrons, gamma = 100, 64 x 64 pixels over +-1.5/gamma, 2^20.

Random draws: numpy PCG64 with seed 1000 + index, fixed order x, y, z, ux, uy,
g (standard normals), then x = sigma_x x^, u_x = (eps_n/sigma_x) u^_x (uncorrelated
at the waist), gamma = gamma_mean (1 + (sigma_gamma/gamma) g^),
u_z = sqrt(gamma^2 - 1 - u_x^2 - u_y^2).  The draws describe the bunch at t = 0;
particles are moved back ballistically to t_start.

Observer grid: dt_obs = T1 / s_p with T1 = lambda (1 + a0^2/2) / (4 gamma_max^2 c)
the first-harmonic period (gamma_max = gamma_mean (1 + 3 sigma_gamma/gamma)), s_p
samples per period, and the n_obs-point window centred on observer time 0
(the arrival of the bunch centre), i.e. t0 = -n_obs dt_obs / 2.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass, field

import numpy as np

C_LIGHT = 299792458.0


@dataclass
class Laser:
    a0: float
    lam: float = 1.0e-6
    w0: float = 0.0  # <= 0: plane wave
    n_cycles: float = 20.0


@dataclass
class Workload:
    name: str
    index: int
    n_p: int
    n_steps: int
    gamma: float
    laser: Laser
    n_side: int
    theta_max: float
    n_obs: int
    samples_per_period: float
    sig_gamma: float = 0.0
    sig_x: float = 0.0
    sig_y: float = 0.0
    sig_z: float = 0.0
    eps_n: float = 0.0
    D: float = 1.0
    trajectory: str = "boris"  # "analytic" (plane-wave closed form) or "boris"
    window_override: float | None = None  # observer window length (s), else n_obs * dt_obs from the policy
    extra: dict = field(default_factory=dict)

    # ---- derived ------------------------------------------------------------------------------
    @property
    def n_samples(self) -> int:
        return self.n_steps + 1

    @property
    def n_pix(self) -> int:
        return self.n_side * self.n_side

    @property
    def t_sim(self) -> float:
        """Simulation window: every particle within 4 sigma_z crosses the whole pulse."""
        if self.trajectory == "analytic":
            return 1.05 * self.laser.n_cycles * self.laser.lam / (2.0 * C_LIGHT)
        return (8.0 * self.sig_z + self.laser.n_cycles * self.laser.lam) / (2.0 * C_LIGHT)

    @property
    def t_start(self) -> float:
        return -0.5 * self.t_sim

    @property
    def dt(self) -> float:
        return self.t_sim / self.n_steps

    @property
    def dt_obs(self) -> float:
        if self.window_override is not None:
            return self.window_override / self.n_obs
        gmax = self.gamma * (1.0 + 3.0 * self.sig_gamma)
        T1 = self.laser.lam * (1.0 + 0.5 * self.laser.a0 ** 2) / (4.0 * gmax * gmax * C_LIGHT)
        return T1 / self.samples_per_period

    @property
    def t0(self) -> float:
        return -0.5 * self.n_obs * self.dt_obs

    def omega1(self, theta=0.0) -> float:
        """Nominal first-harmonic angular frequency at polar angle theta."""
        wl = 2.0 * np.pi * C_LIGHT / self.laser.lam
        return 4.0 * self.gamma ** 2 * wl / (1.0 + 0.5 * self.laser.a0 ** 2 + (self.gamma * theta) ** 2)

    def scaled(self, **kw) -> "Workload":
        """A copy with some sizes replaced (for tests)."""
        return dataclasses.replace(self, **kw)


def pixel_angles(n_side: int, theta_max: float):
    """Cell-centred (theta_x, theta_y) of an n_side x n_side grid over [-theta_max, theta_max]^2,
    pixel m = iy * n_side + ix."""
    c = -theta_max + (np.arange(n_side) + 0.5) * (2.0 * theta_max / n_side)
    ty, tx = np.meshgrid(c, c, indexing="ij")
    return tx.reshape(-1), ty.reshape(-1)


def pixel_positions(n_side: int, theta_max: float, D: float = 1.0) -> np.ndarray:
    """Detector positions on the sphere of radius D, x = D (sin tx, cos tx sin ty, cos tx cos ty)
    (the angle convention of the paper's Fig. on the normal vector)."""
    tx, ty = pixel_angles(n_side, theta_max)
    if n_side == 1:
        tx = np.zeros(1)
        ty = np.zeros(1)
    return np.stack([D * np.sin(tx), D * np.cos(tx) * np.sin(ty), D * np.cos(tx) * np.cos(ty)], axis=-1)


def bunch_init(w: Workload, n_p: int | None = None, gamma=None) -> np.ndarray:
    """Initial phase space [n_p][6] = x, y, z (m), u_x, u_y, u_z at t_start.  ``gamma`` replaces
    the mean Lorentz factor of the draw (the normal deviates stay the same); it may be complex,
    which carries a complex step through the recipe."""
    n = w.n_p if n_p is None else n_p
    gbar = w.gamma if gamma is None else gamma
    if w.trajectory == "analytic" or w.n_p == 1:
        uz = np.sqrt(gbar ** 2 - 1.0)
        bz = uz / gbar
        return np.array([[0.0, 0.0, bz * C_LIGHT * w.t_start, 0.0, 0.0, uz]])
    rng = np.random.Generator(np.random.PCG64(1000 + w.index))
    xh = rng.standard_normal(w.n_p)
    yh = rng.standard_normal(w.n_p)
    zh = rng.standard_normal(w.n_p)
    uxh = rng.standard_normal(w.n_p)
    uyh = rng.standard_normal(w.n_p)
    gh = rng.standard_normal(w.n_p)
    x = w.sig_x * xh
    y = w.sig_y * yh
    z = w.sig_z * zh
    ux = (w.eps_n / w.sig_x) * uxh if w.sig_x > 0 else 0.0 * uxh
    uy = (w.eps_n / w.sig_y) * uyh if w.sig_y > 0 else 0.0 * uyh
    g = gbar * (1.0 + w.sig_gamma * gh)
    uz = np.sqrt(g * g - 1.0 - ux * ux - uy * uy)
    t = w.t_start
    init = np.stack([x + C_LIGHT * ux / g * t, y + C_LIGHT * uy / g * t, z + C_LIGHT * uz / g * t,
                     ux + 0.0 * g, uy + 0.0 * g, uz], axis=-1)
    return np.ascontiguousarray(init[:n])


def uniform_line_init(n_p: int, length: float, gamma: float, t_start: float) -> np.ndarray:
    """Initial phase space [n_p][6] of a line bunch: n_p electrons evenly spaced over ``length``
    along z (cell centres, centred on z = 0 at t = 0), on axis, all with Lorentz factor gamma
    along +z, moved back ballistically to t_start (the crossover setting of Sec. "Performance")."""
    uz = np.sqrt(gamma * gamma - 1.0)
    bz = uz / gamma
    z = -0.5 * length + (np.arange(n_p) + 0.5) * (length / n_p) + bz * C_LIGHT * t_start
    init = np.zeros((n_p, 6))
    init[:, 2] = z
    init[:, 5] = uz
    return init


def bunch_init_dgamma(w: Workload, rows=None) -> np.ndarray:
    """d(init)/d(gamma_mean) of ``bunch_init`` [len(rows)][6] (rows: indices into the full draw,
    default all), exact to rounding by a complex step h = 1e-30 through the recipe."""
    h = 1e-30
    full = bunch_init(w, gamma=w.gamma + 1j * h)
    sel = full if rows is None else full[np.asarray(rows)]
    return np.ascontiguousarray(sel.imag / h)


def band_weights(w: Workload, x_det: np.ndarray, pixels=None, rel_width: float = 0.02) -> np.ndarray:
    """Weights W [n_pix][n_obs/2+1] of the band objective J = sum_m sum_j W[m][j] S[m][j]:
    W = d_omega on the bins with |omega_j - omega1(theta_m)| <= rel_width omega1(theta_m) of the
    selected pixels (all if None), 0 elsewhere; omega_j = 2 pi j/(n_obs dt_obs), theta_m the polar
    angle of pixel m, band edges at the nominal gamma and a0."""
    x_det = np.asarray(x_det, dtype=np.float64).reshape(-1, 3)
    n_pix = x_det.shape[0]
    d_omega = 2.0 * np.pi / (w.n_obs * w.dt_obs)
    omega = d_omega * np.arange(w.n_obs // 2 + 1)
    W = np.zeros((n_pix, w.n_obs // 2 + 1))
    sel = range(n_pix) if pixels is None else pixels
    for m in sel:
        th = np.arccos(np.clip(x_det[m, 2] / np.linalg.norm(x_det[m]), -1.0, 1.0))
        w1 = w.omega1(th)
        W[m, np.abs(omega - w1) <= rel_width * w1] = d_omega
    return W


def central_pixels(n_side: int, n_centre: int) -> np.ndarray:
    """Indices m = iy n_side + ix of the central n_centre x n_centre block of the pixel grid."""
    lo = (n_side - n_centre) // 2
    idx = np.arange(lo, lo + n_centre)
    return (idx[:, None] * n_side + idx[None, :]).reshape(-1)


_PAPER_WORKLOADS = {}


def _register(w: Workload):
    _PAPER_WORKLOADS[w.name] = w
    _PAPER_WORKLOADS[w.index] = w
    return w


_register(Workload(name="single", index=0, n_p=1, n_steps=20000, gamma=50.0, laser=Laser(a0=0.1),
                   n_side=1, theta_max=0.0, n_obs=1 << 16, samples_per_period=0.0, trajectory="analytic",
                   window_override=8.0 * (20.0 * 1.0e-6 / (2.0 * C_LIGHT)) / (2.0 * 50.0 ** 2)))
_register(Workload(name="bunch", index=1, n_p=10000, n_steps=20000, gamma=50.0,
                   laser=Laser(a0=0.5, w0=10e-6), n_side=64, theta_max=1.0 / 50.0, n_obs=1 << 18,
                   samples_per_period=8.0, sig_gamma=1e-3, sig_x=2e-6, sig_y=2e-6, sig_z=5e-6, eps_n=1e-6,
                   extra={"fd_pixels": 64, "fd_omega": 4096}))
_register(Workload(name="precision", index=2, n_p=100000, n_steps=20000, gamma=200.0,
                   laser=Laser(a0=1.0, w0=10e-6), n_side=128, theta_max=2.0 / 200.0, n_obs=1 << 18,
                   samples_per_period=16.0, sig_gamma=1e-3, sig_x=2e-6, sig_y=2e-6, sig_z=5e-6, eps_n=1e-6))
_register(Workload(name="grad", index=3, n_p=1000, n_steps=10000, gamma=50.0,
                   laser=Laser(a0=0.5, w0=10e-6), n_side=32, theta_max=1.0 / 50.0, n_obs=1 << 16,
                   samples_per_period=8.0, sig_gamma=1e-3, sig_x=2e-6, sig_y=2e-6, sig_z=5e-6, eps_n=1e-6))
_register(Workload(name="large", index=4, n_p=100000, n_steps=20000, gamma=100.0,
                   laser=Laser(a0=0.8, w0=10e-6), n_side=64, theta_max=1.5 / 100.0, n_obs=1 << 20,
                   samples_per_period=8.0, sig_gamma=5e-4, sig_x=3e-6, sig_y=3e-6, sig_z=10e-6, eps_n=1e-6))


def workload(key) -> Workload:
    """Workload by name ("single", "bunch", "precision", "grad", "large") or index 0..4."""
    return _PAPER_WORKLOADS[key]


def random_trajectory(n_p: int, n_samples: int, seed: int, dt: float = 1e-18, gamma: float = 20.0,
                      wiggle: float = 1e-3, spread: float = 1e-6):
    """Smooth synthetic trajectories for kernel tests that need no particular physics:
    r, beta, beta_dot [n_p][n_samples][3] with |beta| < 1 and |r_i - r_{i-1}| < c dt.
    Each particle moves along +z at speed ~ (1 - 1/(2 gamma^2)) c with a small sinusoidal
    transverse wiggle of seeded amplitude, phase and period, starting from a seeded offset
    of rms size ``spread`` (m).  beta_dot is the
    time derivative of the wiggle (consistent to the sampling)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = np.arange(n_samples) * dt
    amp = wiggle * (0.5 + rng.random((n_p, 2)))
    per = dt * n_samples / (3.0 + 5.0 * rng.random((n_p, 1)))
    ph = 2.0 * np.pi * rng.random((n_p, 2))
    off = spread * rng.standard_normal((n_p, 3))
    w = 2.0 * np.pi / per
    bx = amp[:, :1] * np.sin(w * t[None] + ph[:, :1])
    by = amp[:, 1:] * np.sin(w * t[None] + ph[:, 1:])
    btot = 1.0 - 0.5 / gamma ** 2
    bz = np.sqrt(btot ** 2 - bx ** 2 - by ** 2)
    beta = np.stack([bx, by, bz], axis=-1)
    bd = np.stack([amp[:, :1] * w * np.cos(w * t[None] + ph[:, :1]),
                   amp[:, 1:] * w * np.cos(w * t[None] + ph[:, 1:]),
                   np.zeros_like(bx)], axis=-1)
    # positions: cumulative trapezoid of c*beta (keeps |dr| < c dt since |beta| < 1)
    dr = 0.5 * (beta[:, 1:] + beta[:, :-1]) * C_LIGHT * dt
    r = np.concatenate([np.zeros((n_p, 1, 3)), np.cumsum(dr, axis=1)], axis=1) + off[:, None, :]
    return (np.ascontiguousarray(r), np.ascontiguousarray(beta), np.ascontiguousarray(bd))
