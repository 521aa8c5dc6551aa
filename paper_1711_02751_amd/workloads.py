"""Seeded synthetic workloads: initial conditions and run parameters.

This module holds no arithmetic of the numerical method.  It evaluates
closed-form initial states at node coordinates supplied by the caller and
lists the run parameters of each named workload; both the HIP library's
tests/benchmark and the CPU oracle consume it, and neither is imported here.

Variables are the user units (h, hu, hv): total depth and momenta.  Domains
are periodic [0, Lx) x [0, Ly).  Random draws use numpy's PCG64 with a fixed
draw order: bump centres, bump widths, then the velocity modes.
"""
import math
from dataclasses import dataclass, field

import numpy as np


def standing_wave(x, y, t, g, H, amp=0.01, Lx=1.0, Ly=1.0):
    """Exact solution of the linearized planar system (lemma of Sec. 3):
        eta = amp cos(2 pi x / Lx) cos(2 pi y / Ly) cos(omega t)
        (hu, hv) = (g H amp / omega) (kx sin cos, ky cos sin) sin(omega t)
    with kx = 2 pi / Lx, ky = 2 pi / Ly, omega^2 = g H (kx^2 + ky^2)."""
    kx, ky = 2.0 * math.pi / Lx, 2.0 * math.pi / Ly
    om = math.sqrt(g * H * (kx * kx + ky * ky))
    cx, sx = np.cos(kx * x), np.sin(kx * x)
    cy, sy = np.cos(ky * y), np.sin(ky * y)
    h = H + amp * cx * cy * math.cos(om * t)
    c = H * amp / om * math.sin(om * t)
    return h, c * kx * sx * cy, c * ky * cx * sy


def standing_wave_omega(g, H, Lx=1.0, Ly=1.0):
    kx, ky = 2.0 * math.pi / Lx, 2.0 * math.pi / Ly
    return math.sqrt(g * H * (kx * kx + ky * ky))


def bump_flow(x, y, seed, H=1.0, n_bumps=1, amp=0.01, sigma=(0.05, 0.10),
              n_modes=8, max_mode=4, umax=0.1, Lx=1.0, Ly=1.0):
    """Gaussian height bumps on a seeded divergence-free vortical flow.

    h = H + amp * sum_b exp(-d_b^2 / (2 sigma_b^2)), d_b the periodic
    minimum-image distance to centre b (centres ~ U[0,1)^2 of the domain,
    sigma_b ~ U[sigma] in domain units).  Stream function
    psi = sum_m a_m cos(2 pi (p_m x/Lx + q_m y/Ly) + theta_m) with distinct
    integer (p_m, q_m) in [-max_mode, max_mode]^2 minus the origin,
    a_m ~ N(0, 1) / (p_m^2 + q_m^2), theta_m ~ U[0, 2 pi); (u, v) =
    (d_y psi, -d_x psi), scaled so that max |u| over the given points is umax.
    Returns (h, hu, hv)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.random((n_bumps, 2))
    sigmas = rng.uniform(sigma[0], sigma[1], n_bumps)
    cand = [(p, q) for p in range(-max_mode, max_mode + 1)
            for q in range(-max_mode, max_mode + 1) if (p, q) != (0, 0)]
    pick = rng.choice(len(cand), size=n_modes, replace=False)
    modes = [cand[i] for i in pick]
    amps = rng.standard_normal(n_modes)
    theta = rng.uniform(0.0, 2.0 * math.pi, n_modes)

    xs, ys = np.asarray(x) / Lx, np.asarray(y) / Ly
    h = np.full(xs.shape, float(H))
    for b in range(n_bumps):
        dx = xs - centres[b, 0]
        dy = ys - centres[b, 1]
        dx -= np.round(dx)
        dy -= np.round(dy)
        h = h + amp * np.exp(-(dx * dx + dy * dy) / (2.0 * sigmas[b] ** 2))
    u = np.zeros(xs.shape)
    v = np.zeros(xs.shape)
    for m, (p, q) in enumerate(modes):
        a = amps[m] / (p * p + q * q)
        s = np.sin(2.0 * math.pi * (p * xs + q * ys) + theta[m])
        u += -a * s * 2.0 * math.pi * q / Ly
        v += a * s * 2.0 * math.pi * p / Lx
    speed = np.sqrt(u * u + v * v).max()
    if speed > 0:
        u *= umax / speed
        v *= umax / speed
    return h, h * u, h * v


@dataclass
class Workload:
    """One named run: mesh, degree, physics, time step and step count."""
    name: str
    n: int
    k: int
    g: float
    H: float
    dt: float
    steps: int
    nonlinear: bool
    ic: str
    seed: int = 0
    n_bumps: int = 1
    L: float = 1.0
    notes: str = ""

    @property
    def n_dof(self):
        return 3 * self.n * self.n * (self.k + 1) ** 2

    def initial_state(self, x, y):
        if self.ic == "standing_wave":
            return standing_wave(x, y, 0.0, self.g, self.H, Lx=self.L, Ly=self.L)
        return bump_flow(x, y, self.seed, H=self.H, n_bumps=self.n_bumps,
                         Lx=self.L, Ly=self.L)


# Time steps.  Courant reading: Cr = dt max(|u| + sqrt(phi)) / dx_min with
# dx_min the smallest LGL node spacing (h/2)(1 - xi_1):
#   k=4: 1 - xi_1 = 1 - sqrt(3/7);  k=6: 1 - xi_1 = 0.16977610372143...;
#   k=3: 1 - xi_1 = 1 - 1/sqrt(5).
# The bump workloads take dt = 2 dx_min: advective Courant 0.2 at |u| = 0.1
# and gravity Courant about 6.5 for g = 9.81, H = 1.  An advective Courant of
# 0.5 (dt = 5 dx_min) exceeds the stability limit of the explicit nonlinear
# part at k = 4 and k = 6 (growth within a few dozen steps); 2 dx_min runs
# the step counts below without growth.
ADVECTIVE_DT_FACTOR = 2.0
_XI1 = {3: 1.0 - 1.0 / math.sqrt(5.0), 4: 1.0 - math.sqrt(3.0 / 7.0),
        6: 0.16977610372143304}


def bump_dt(n, k, L=1.0):
    return ADVECTIVE_DT_FACTOR * _XI1[k] / 2.0 * L / n


WORKLOADS = {
    "standing_wave_8x8_k2": Workload(
        "standing_wave_8x8_k2", n=8, k=2, g=1.0, H=1.0, dt=0.01, steps=100,
        nonlinear=False, ic="standing_wave",
        notes="linearized, exact standing wave, FP64"),
    "bump_64x64_k4": Workload(
        "bump_64x64_k4", n=64, k=4, g=9.81, H=1.0, dt=bump_dt(64, 4), steps=500,
        nonlinear=True, ic="bump_flow", seed=2),
    "bump_256x256_k4": Workload(
        "bump_256x256_k4", n=256, k=4, g=9.81, H=1.0, dt=bump_dt(256, 4), steps=500,
        nonlinear=True, ic="bump_flow", seed=3),
    "bump_1024x1024_k6": Workload(
        "bump_1024x1024_k6", n=1024, k=6, g=9.81, H=1.0, dt=bump_dt(1024, 6), steps=200,
        nonlinear=True, ic="bump_flow", seed=5, n_bumps=16),
}


def ensemble_members(seed=4, count=64, k=3, g=9.81, H=1.0, steps=100):
    """Ensemble of `count` periodic runs on uneven meshes n_m in [32, 128];
    member m uses IC seed 4000 + m and dt_m = 2 dx_min(n_m), so dt_m / h_m
    is the same for every member."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(32, 129, size=count)
    return [Workload(f"member{m}", n=int(sizes[m]), k=k, g=g, H=H,
                     dt=bump_dt(int(sizes[m]), k), steps=steps, nonlinear=True,
                     ic="bump_flow", seed=4000 + m)
            for m in range(count)]


def moving_vortex(x, y, t, H_inf=1.0, u_inf=1.0, v_inf=0.0, beta=5.0,
                  xc=0.0, yc=0.0, g=2.0):
    """Exact translating vortex of Sec. 6.1 (eq. tc_vortex_ic), user units:
        H = H_inf - beta^2 / (32 pi^2) exp(-2 (r^2 - 1))
        u = u_inf - beta / (2 pi) exp(-(r^2 - 1)) y_t
        v = v_inf + beta / (2 pi) exp(-(r^2 - 1)) x_t
    with x_t = x - xc - u_inf t, y_t = y - yc - v_inf t, r^2 = x_t^2 + y_t^2.
    Returns (h, hu, hv).  (g is part of the test's definition, not of H.)"""
    xt = x - xc - u_inf * t
    yt = y - yc - v_inf * t
    r2 = xt * xt + yt * yt
    e = np.exp(-(r2 - 1.0))
    h = H_inf - beta * beta / (32.0 * math.pi ** 2) * e * e
    u = u_inf - beta / (2.0 * math.pi) * e * yt
    v = v_inf + beta / (2.0 * math.pi) * e * xt
    return h, h * u, h * v


def water_drop(x, y, H_inf=100.0, sigma=0.1, xc=1.0, yc=1.0):
    """Water-height perturbation of Sec. 6.2 on [0, 2]^2 (the paper's
    [-1, 1]^2 translated, centre (1, 1)): depth H_inf + exp(-r^2 / (2
    sigma^2)), r the distance to the centre, at rest.  The paper does not
    print sigma; 0.1 is the reading taken (a bump resolved by the 20 x 20,
    degree-8 mesh: about 9 nodes across one sigma).  Returns (h, hu, hv)."""
    r2 = (x - xc) ** 2 + (y - yc) ** 2
    h = H_inf + np.exp(-r2 / (2.0 * sigma * sigma))
    z = np.zeros_like(h)
    return h, z, z.copy()
