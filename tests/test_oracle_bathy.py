"""Pins of the oracle with variable bathymetry (oracle/bathy.py):

  * a constant depth reproduces the flat-bottom oracle (residuals and steps);
  * on smooth periodic data the DG residuals converge to the analytic
    operators: the linear part with its source term to
    (-div U, -phi_B grad phi_eta) (the phi_eta grad phi_B of the flux and of
    the source cancel), the nonlinear part to -div F_NL, at a rate near k;
  * the source term is what keeps a lake at rest over an uneven bottom at
    rest in the continuous operator: dropping it leaves a residual;
  * mass is conserved to round-off over nonlinear steps.
"""
import math

import numpy as np
import pytest

from oracle import bathy, imex, swe


def bottom(mesh, H=1.0, amp=0.2):
    x, y = mesh.coords()
    return H * (1.0 + amp * np.sin(2 * math.pi * x / mesh.Lx) * np.cos(2 * math.pi * y / mesh.Ly)
                + 0.5 * amp * np.cos(4 * math.pi * y / mesh.Ly))


def smooth_state(x, y, Lx, Ly, a=0.05):
    kx, ky = 2 * math.pi / Lx, 2 * math.pi / Ly
    p = a * np.sin(kx * x + 0.3) * np.cos(ky * y)
    U = a * np.cos(kx * x) * np.sin(2 * ky * y + 0.1)
    V = a * np.sin(2 * kx * x - 0.2) * np.cos(ky * y)
    return np.stack([p, U, V])


def test_constant_depth_is_the_flat_bottom_oracle():
    m = swe.Mesh(6, 5, 1.2, 1.0, 3)
    rng = np.random.default_rng(4)
    g, H = 9.81, 1.0
    q = 0.05 * rng.standard_normal(m.shape)
    B = np.full((m.ny, m.nx, m.K, m.K), H)
    for a, b in [(bathy.nl_residual(m, q, g * B), swe.nl_residual(m, q, g * H)),
                 (bathy.linear_residual(m, q, g * B), swe.linear_dglf_residual(m, q, g * H))]:
        assert np.abs(a - b).max() < 1e-13 * np.abs(b).max()
    P = bathy.BathyProblem(6, 5, 1.2, 1.0, 3, g, B, 0.004)
    Pf = imex.Problem(6, 5, 1.2, 1.0, 3, g, H, 0.004)
    assert np.abs(P.run(q, 3) - Pf.run(q, 3)).max() < 1e-12 * np.abs(q).max()


def _fd(f, x, y, d, h=1e-5):
    if d == 0:
        return (f(x + h, y) - f(x - h, y)) / (2 * h)
    return (f(x, y + h) - f(x, y - h)) / (2 * h)


@pytest.mark.parametrize("which", ["linear", "nonlinear"])
def test_residuals_converge_to_the_analytic_operators(which):
    g, k, L = 2.0, 3, 1.0
    errs = []
    for n in (4, 8, 16):
        m = swe.Mesh(n, n, L, L, k)
        x, y = m.coords()
        B = bottom(m)
        phiB = g * B
        q = smooth_state(x, y, L, L)

        def phiB_fn(xx, yy):
            return g * (1.0 + 0.2 * np.sin(2 * math.pi * xx) * np.cos(2 * math.pi * yy)
                        + 0.1 * np.cos(4 * math.pi * yy))

        if which == "linear":
            got = bathy.linear_residual(m, q, phiB)
            ref = np.stack([
                -(_fd(lambda a, b: smooth_state(a, b, L, L)[1], x, y, 0)
                  + _fd(lambda a, b: smooth_state(a, b, L, L)[2], x, y, 1)),
                -phiB * _fd(lambda a, b: smooth_state(a, b, L, L)[0], x, y, 0),
                -phiB * _fd(lambda a, b: smooth_state(a, b, L, L)[0], x, y, 1)])
        else:
            got = bathy.nl_residual(m, q, phiB)

            def fnl(a, b, d):
                s = smooth_state(a, b, L, L)
                Fx, Fy = bathy.flux_nonlinear(s, phiB_fn(a, b))
                return Fx if d == 0 else Fy
            ref = -(_fd(lambda a, b: fnl(a, b, 0), x, y, 0) + _fd(lambda a, b: fnl(a, b, 1), x, y, 1))
        errs.append(np.sqrt(np.sum(m.mass()[None] * (got - ref) ** 2)))
    rates = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    print(which, errs, rates)
    assert min(rates) > k - 0.6


def test_source_term_balances_the_bottom_in_the_linear_operator():
    """phi_eta constant, U = V = 0 over an uneven bottom: -phi_B grad phi_eta
    = 0, so the linear residual vanishes up to the discrete error; without
    the source term it is O(phi_eta grad phi_B)."""
    g, k, n = 2.0, 4, 8
    m = swe.Mesh(n, n, 1.0, 1.0, k)
    phiB = g * bottom(m)
    q = np.zeros(m.shape)
    q[0] = 0.05
    with_src = bathy.linear_residual(m, q, phiB)
    without = bathy.dg_residual(m, q, phiB, bathy.flux_linear, bathy.rusanov_linear)
    assert np.abs(with_src).max() < 1e-10 * np.abs(without).max() + 1e-12
    assert np.abs(without).max() > 0.05


def test_mass_is_conserved():
    g, k, n = 9.81, 3, 6
    m = swe.Mesh(n, n, 1.0, 1.0, k)
    B = bottom(m, amp=0.3)
    x, y = m.coords()
    q = smooth_state(x, y, 1.0, 1.0, a=0.2)
    P = bathy.BathyProblem(n, n, 1.0, 1.0, k, g, B, 0.006)
    m0 = swe.mass(m, q)[0]
    q1 = P.run(q, 10)
    assert np.abs(q1 - q).max() > 1e-3
    assert abs(swe.mass(m, q1)[0] - m0) < 1e-13 * np.sum(m.mass() * np.abs(q[0]))
