"""Pins of the closed-basin oracle (oracle/basin.py: reflecting walls over a
variable depth):

  * a constant depth reproduces the walled box of `box` (residuals, steps);
  * method of images: the basin equals the periodic variable-depth oracle
    of `bathy` on the mirror-doubled domain (state mirrored with the normal
    momentum negated, depth mirrored), restricted to the basin, for the
    residuals and for whole ARS2 / ARS3 steps;
  * a lake at rest over an uneven bottom stays at rest (the source term
    balances the pressure term, the walls pass no flux);
  * mass is conserved to round-off over nonlinear steps.
"""
import math

import numpy as np
import pytest

from oracle import basin, bathy, box, imex, swe
from test_oracle_bathy import smooth_state
from test_oracle_wall import drop_state, mirror_extend


def bottom(mesh, H=1.0, amp=0.2):
    """An uneven depth with no symmetry of the basin."""
    x, y = mesh.coords()
    return H * (1.0 + amp * np.sin(2.3 * x / mesh.Lx + 0.4) * np.cos(1.7 * y / mesh.Ly)
                + 0.5 * amp * np.cos(3.1 * y / mesh.Ly - 0.2) * x / mesh.Lx)


def mirror_depth(B):
    """(ny, nx, K, K) -> (2 ny, 2 nx, K, K): the depth mirrored like the
    state, without a sign change."""
    row = np.concatenate([B, B[:, ::-1, :, ::-1]], axis=1)
    return np.concatenate([row, row[::-1, :, ::-1, :]], axis=0)


def basin_state(mesh, g, H, seed=3):
    """A water-height perturbation plus a smooth flow whose normal momentum
    does not vanish on the walls (so the reflection is exercised)."""
    q = drop_state(mesh, g, H, sigma=0.2, xc=0.35 * mesh.Lx, yc=0.6 * mesh.Ly, umax=0.02,
                   seed=seed)
    x, y = mesh.coords()
    q += 0.02 * g * H * smooth_state(x, y, mesh.Lx, mesh.Ly, a=1.0)
    return q


def test_constant_depth_is_the_walled_box():
    n, k, g, H, dt = 5, 3, 9.81, 1.0, 0.004
    m = swe.Mesh(n, n, 1.0, 1.0, k)
    q = basin_state(m, g, H)
    B = np.full((n, n, m.K, m.K), H)
    ref = box.reflect_exterior(m, q)
    for a, b in [(basin.nl_residual(m, q, g * B), box.nl_residual(m, q, g * H, ref)),
                 (basin.linear_residual(m, q, g * B), box.linear_residual(m, q, g * H, ref))]:
        assert np.abs(a - b).max() < 1e-12 * np.abs(b).max()
    P = basin.BasinProblem(n, n, 1.0, 1.0, k, g, B, dt)
    Pw = box.BoxProblem(n, n, 1.0, 1.0, k, g, H, dt, "wall", tableau=imex.ars232())
    assert np.abs(P.run(q, 3) - Pw.run(q, 3)).max() < 1e-12 * np.abs(q).max()


def test_residuals_equal_the_periodic_mirror_image():
    nx, ny, k, g = 4, 3, 3, 9.81
    m = swe.Mesh(nx, ny, 1.2, 1.0, k)
    B = bottom(m)
    q = basin_state(m, g, 1.0)
    m2 = swe.Mesh(2 * nx, 2 * ny, 2.4, 2.0, k)
    q2, B2 = mirror_extend(q), mirror_depth(B)
    for fb, fp in [(basin.nl_residual, bathy.nl_residual),
                   (basin.linear_residual, bathy.linear_residual)]:
        a = mirror_extend(fb(m, q, g * B))
        b = fp(m2, q2, g * B2)
        assert np.abs(a - b).max() < 1e-11 * np.abs(b).max()


@pytest.mark.parametrize("tab,k,steps", [(imex.ars232(), 3, 5), (imex.ars443(), 2, 3)])
def test_steps_equal_the_periodic_mirror_image(tab, k, steps):
    n, g, dt = 3, 9.81, 0.004
    m = swe.Mesh(n, n, 1.0, 1.0, k)
    B = bottom(m, amp=0.3)
    q0 = basin_state(m, g, 1.0, seed=5)
    a = basin.BasinProblem(n, n, 1.0, 1.0, k, g, B, dt, tableau=tab).run(q0, steps)
    Pp = bathy.BathyProblem(2 * n, 2 * n, 2.0, 2.0, k, g, mirror_depth(B), dt, tableau=tab)
    b = Pp.run(mirror_extend(q0), steps)
    assert np.abs(mirror_extend(a) - b).max() < 1e-10 * np.abs(b).max()
    assert np.abs(a - q0).max() > 1e-3 * np.abs(q0).max()     # the state did move


def test_lake_at_rest_stays_at_rest():
    n, k, g = 4, 4, 9.81
    m = swe.Mesh(n, n, 1.0, 1.0, k)
    B = bottom(m, amp=0.3)
    q = np.zeros(m.shape)
    q[0] = 0.05 * g      # a flat surface 0.05 above the reference plane
    assert np.abs(basin.nl_residual(m, q, g * B)).max() < 1e-12
    lin = basin.linear_residual(m, q, g * B)
    # without the source term the pressure gradient phi_eta grad phi_B remains
    raw = basin.dg_residual(m, q, g * B, bathy.flux_linear, bathy.rusanov_linear)
    assert np.abs(raw).max() > 0.1
    assert np.abs(lin).max() < 1e-10 * np.abs(raw).max()
    P = basin.BasinProblem(n, n, 1.0, 1.0, k, g, B, 0.01)
    q1 = P.run(q, 3)
    assert np.abs(q1 - q).max() < 1e-10 * np.abs(q).max()


def test_mass_is_conserved():
    n, k, g = 5, 3, 9.81
    m = swe.Mesh(n, n, 1.0, 1.0, k)
    B = bottom(m, amp=0.3)
    q = basin_state(m, g, 1.0, seed=7)
    P = basin.BasinProblem(n, n, 1.0, 1.0, k, g, B, 0.006)
    m0 = swe.mass(m, q)[0]
    q1 = P.run(q, 8)
    assert np.abs(q1 - q).max() > 1e-3 * np.abs(q).max()
    assert abs(swe.mass(m, q1)[0] - m0) < 1e-13 * np.sum(m.mass() * np.abs(q[0]))
