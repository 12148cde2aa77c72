// FP64 Boris trajectories of electrons in the laser pulse (the trajectory source of
// the time-domain method; the paper integrates the equations of motion with the
// Boris method).  One lane per particle; the samples are written as
// r, beta, beta_dot [n_particles][n_samples][3].
#include "lw_internal.h"

#include <algorithm>

namespace lw {
namespace {

struct LaserDev {
    double a0, wl, w0, nc, E0;  // wl = 2 pi c / lambda, E0 = a0 m_e c wl / e
};

// Pulse written through its normalised vector potential a_x = a0 g(phi) sin(phi),
// g = cos^2(phi/(2 nc)) on |phi| < pi nc, phi = wl (t + z/c):
// E_x = -E0 T(rho) d(g sin)/dphi, B_y = -E_x / c, T = exp(-rho^2/w0^2) (w0 > 0).
__device__ __forceinline__ void laser_eb(const LaserDev &L, double x, double y, double z, double t, double &Ex,
                                         double &By)
{
    const double phi = L.wl * (t + z / kC);
    Ex = 0.0;
    By = 0.0;
    if (!(fabs(phi) < kPi * L.nc)) return;
    double sh, ch, sp, cp, s2, c2;
    sincos(phi / (2.0 * L.nc), &sh, &ch);
    sincos(phi, &sp, &cp);
    sincos(phi / L.nc, &s2, &c2);
    const double g = ch * ch;
    const double gp = -s2 / (2.0 * L.nc);
    const double dS = gp * sp + g * cp;
    double T = 1.0;
    if (L.w0 > 0.0) T = exp(-(x * x + y * y) / (L.w0 * L.w0));
    Ex = -L.E0 * T * dS;
    By = -Ex / kC;
}

// Boris update of u = gamma beta over time h for an electron, with E = (Ex,0,0), B = (0,By,0).
__device__ __forceinline__ void kick(double &ux, double &uy, double &uz, double Ex, double By, double h)
{
    const double q = -kQe, m = kMe;
    const double a = q * h / (2.0 * m * kC);
    double mx = ux + a * Ex, my = uy, mz = uz;
    const double gm = sqrt(1.0 + mx * mx + my * my + mz * mz);
    const double ty = q * h * By / (2.0 * m * gm);  // rotation vector (0, ty, 0)
    const double sy = 2.0 * ty / (1.0 + ty * ty);
    // u' = u- + u- x t ;  u+ = u- + u' x s
    const double px = mx - mz * ty, py = my, pz = mz + mx * ty;
    const double nx = mx - pz * sy, ny = my, nz = mz + px * sy;
    ux = nx + a * Ex;
    uy = ny;
    uz = nz;
}

__global__ __launch_bounds__(256) void k_boris(const double *__restrict__ init, int64_t n_particles,
                                               int64_t n_samples, double t_start, double dt, LaserDev L,
                                               double *__restrict__ r, double *__restrict__ beta,
                                               double *__restrict__ beta_dot)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_particles) return;
    double x = init[6 * k], y = init[6 * k + 1], z = init[6 * k + 2];
    double usx = init[6 * k + 3], usy = init[6 * k + 4], usz = init[6 * k + 5];  // u at the sample time
    double uhx = usx, uhy = usy, uhz = usz;                                      // u half a step later
    double Ex, By;
    laser_eb(L, x, y, z, t_start, Ex, By);
    kick(uhx, uhy, uhz, Ex, By, 0.5 * dt);
    const double q = -kQe, m = kMe;
    for (int64_t i = 0; i < n_samples; ++i) {
        const double ti = t_start + (double)i * dt;
        const double g = sqrt(1.0 + usx * usx + usy * usy + usz * usz);
        const double bx = usx / g, by = usy / g, bz = usz / g;
        laser_eb(L, x, y, z, ti, Ex, By);
        // d beta/dt = q/(gamma m c) [E + c beta x B - beta (beta.E)],  E = (Ex,0,0), B = (0,By,0)
        const double f = q / (g * m * kC);
        const double be = bx * Ex;
        const double ax = f * (Ex - kC * bz * By - bx * be);
        const double ay = f * (-by * be);
        const double az = f * (kC * bx * By - bz * be);
        const size_t o = (size_t)(k * n_samples + i) * 3;
        r[o] = x;
        r[o + 1] = y;
        r[o + 2] = z;
        beta[o] = bx;
        beta[o + 1] = by;
        beta[o + 2] = bz;
        beta_dot[o] = ax;
        beta_dot[o + 1] = ay;
        beta_dot[o + 2] = az;
        if (i + 1 == n_samples) break;
        const double gh = sqrt(1.0 + uhx * uhx + uhy * uhy + uhz * uhz);
        x += kC * uhx / gh * dt;
        y += kC * uhy / gh * dt;
        z += kC * uhz / gh * dt;
        double nx = uhx, ny = uhy, nz = uhz;
        laser_eb(L, x, y, z, t_start + (double)(i + 1) * dt, Ex, By);
        kick(nx, ny, nz, Ex, By, dt);
        usx = 0.5 * (uhx + nx);
        usy = 0.5 * (uhy + ny);
        usz = 0.5 * (uhz + nz);
        uhx = nx;
        uhy = ny;
        uhz = nz;
    }
}

}  // namespace

lw_status launch_boris(const lw_traj_t *t, double *r, double *beta, double *beta_dot, hipStream_t s)
{
    if (t->n_particles == 0) return LW_OK;
    LaserDev L;
    L.a0 = t->laser.a0;
    L.wl = 2.0 * kPi * kC / t->laser.lambda;
    L.w0 = t->laser.w0;
    L.nc = t->laser.n_cycles;
    L.E0 = L.a0 * kMe * kC * L.wl / kQe;
    const int64_t blocks = (t->n_particles + 63) / 64;
    k_boris<<<(unsigned)blocks, 64, 0, s>>>(t->init, t->n_particles, t->n_samples, t->t_start, t->dt, L, r, beta,
                                           beta_dot);
    return check_launch("lw_trajectory_boris");
}

}  // namespace lw
