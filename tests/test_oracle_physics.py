"""Pins of the oracle's fluxes and DG operators against the PDE itself."""
import math

import numpy as np
import pytest

from oracle import swe
from paper_1711_02751_amd import workloads as W


def _rand_state(shape, rng, phi_B):
    q = np.empty((3,) + shape)
    q[0] = 0.05 * phi_B * rng.standard_normal(shape)
    q[1] = 0.3 * rng.standard_normal(shape)
    q[2] = 0.3 * rng.standard_normal(shape)
    return q


def test_flux_matches_original_equations():
    """F(q) for (phi_eta, U, V) = (g(H-B), gHu, gHv) is g times the flux of
    the conservative SWE in (H, Hu) (eq. governingeq) up to the constant
    g^2 B^2 / 2 on the momentum diagonal (zero divergence on a flat bottom)."""
    rng = np.random.default_rng(1)
    g, B = 9.81, 1.3
    H = B + 0.2 * rng.random(50)
    u, v = rng.standard_normal(50), rng.standard_normal(50)
    q = np.stack([g * (H - B), g * H * u, g * H * v])
    Fx, Fy = swe.flux_full(q, g * B)
    c = g * g * B * B / 2
    np.testing.assert_allclose(Fx[0], g * H * u, rtol=1e-13)
    np.testing.assert_allclose(Fx[1], g * (H * u * u + g * H * H / 2) - c, rtol=1e-12)
    np.testing.assert_allclose(Fx[2], g * H * u * v, rtol=1e-13)
    np.testing.assert_allclose(Fy[1], g * H * u * v, rtol=1e-13)
    np.testing.assert_allclose(Fy[2], g * (H * v * v + g * H * H / 2) - c, rtol=1e-12)


def test_nonlinear_flux_is_quadratic_remainder():
    """F_NL vanishes to second order about the lake at rest: F_L is the
    linearisation of F (Sec. 3.1)."""
    rng = np.random.default_rng(2)
    q = _rand_state((40,), rng, 2.0)
    n1 = np.abs(np.stack(swe.flux_nonlinear(1e-3 * q, 2.0))).max()
    n2 = np.abs(np.stack(swe.flux_nonlinear(1e-4 * q, 2.0))).max()
    assert 90 < n1 / n2 < 110
    assert np.all(np.stack(swe.flux_nonlinear(q, 2.0))[:, 0] == 0.0)


@pytest.mark.parametrize("nvec", [(1.0, 0.0), (0.0, -1.0), (0.6, 0.8)])
def test_rusanov_consistency(nvec):
    rng = np.random.default_rng(3)
    q = _rand_state((30,), rng, 1.5)
    nx, ny = nvec
    Fx, Fy = swe.flux_full(q, 1.5)
    np.testing.assert_allclose(swe.rusanov_full(q, q, nx, ny, 1.5), Fx * nx + Fy * ny, atol=1e-14)
    Lx, Ly = swe.flux_linear(q, 1.5)
    np.testing.assert_allclose(swe.rusanov_linear(q, q, nx, ny, 1.5), Lx * nx + Ly * ny, atol=1e-14)


def test_free_stream_preserved():
    m = swe.Mesh(5, 4, 1.0, 0.8, 3)
    q = np.zeros(m.shape)
    q[0], q[1], q[2] = 0.02, 0.3, -0.2
    assert np.abs(swe.nl_residual(m, q, 9.81)).max() < 1e-12
    assert np.abs(swe.linear_dglf_residual(m, q, 9.81)).max() < 1e-12


def _smooth(x, y, Lx, Ly):
    a = 2 * math.pi / Lx
    b = 2 * math.pi / Ly
    p = 0.1 * np.sin(a * x) * np.cos(b * y) + 0.05 * np.cos(2 * b * y)
    U = 0.4 * np.cos(a * x + 0.3) * np.sin(b * y) + 0.2
    V = -0.3 * np.sin(a * x) * np.sin(2 * b * y + 1.0) - 0.1
    dp = (0.1 * a * np.cos(a * x) * np.cos(b * y),
          -0.1 * b * np.sin(a * x) * np.sin(b * y) - 0.1 * b * np.sin(2 * b * y))
    dU = (-0.4 * a * np.sin(a * x + 0.3) * np.sin(b * y), 0.4 * b * np.cos(a * x + 0.3) * np.cos(b * y))
    dV = (-0.3 * a * np.cos(a * x) * np.sin(2 * b * y + 1.0),
          -0.6 * b * np.sin(a * x) * np.cos(2 * b * y + 1.0))
    return np.stack([p, U, V]), dp, dU, dV


def _exact_divergence(q, dp, dU, dV, phi_B, part):
    """-div F_part(q) from the analytic derivatives (chain rule)."""
    p, U, V = q
    phi = p + phi_B
    if part == "linear":
        return np.stack([-(dU[0] + dV[1]), -phi_B * dp[0], -phi_B * dp[1]])
    # F_NL x: (0, U^2/phi + p^2/2, UV/phi); y: (0, UV/phi, V^2/phi + p^2/2)
    dphi = dp
    dx_uu = 2 * U * dU[0] / phi - U * U * dphi[0] / phi ** 2 + p * dp[0]
    dy_uv = (dU[1] * V + U * dV[1]) / phi - U * V * dphi[1] / phi ** 2
    dx_uv = (dU[0] * V + U * dV[0]) / phi - U * V * dphi[0] / phi ** 2
    dy_vv = 2 * V * dV[1] / phi - V * V * dphi[1] / phi ** 2 + p * dp[1]
    return np.stack([np.zeros_like(p), -(dx_uu + dy_uv), -(dx_uv + dy_vv)])


@pytest.mark.parametrize("part", ["linear", "nonlinear"])
@pytest.mark.parametrize("k", [2, 3])
def test_dg_residual_converges_to_divergence(part, k):
    """M^-1 L_DG(q) -> -div F_L(q) and M^-1 NL(q) -> -div F_NL(q) for a smooth
    periodic field: the observed rate rises towards k (last rate >= k - 0.35).  A dropped face
    term, a sign or a transposed derivative stalls the rate at 0 or -1."""
    phi_B = 2.0
    errs = []
    for n in [8, 16, 32]:
        m = swe.Mesh(n, n + 2, 1.0, 1.3, k)
        x, y = m.coords()
        q, dp, dU, dV = _smooth(x, y, 1.0, 1.3)
        if part == "linear":
            r = swe.linear_dglf_residual(m, q, phi_B)
        else:
            r = swe.nl_residual(m, q, phi_B)
        ex = _exact_divergence(q, dp, dU, dV, phi_B, part)
        mm = m.mass()
        errs.append(math.sqrt(sum(np.sum(mm * (r[c] - ex[c]) ** 2) for c in range(3))))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > k - 0.35 and rates.min() > k - 1.0, (errs, rates)


def test_hdg_trace_closed_form_is_conservative():
    """qhat from hdg_trace makes the hybridized flux single valued:
    Fhat.n- (from K-) + Fhat.n+ (from K+) = 0 at every face node."""
    from oracle import hdg_dense
    rng = np.random.default_rng(4)
    m = swe.Mesh(4, 3, 1.0, 1.0, 2)
    q = _rand_state(m.shape[1:], rng, 3.0)
    qx, qy = swe.hdg_trace(m, q, 3.0)
    jx, jy = hdg_dense.hdg_conservation(m, q, qx, qy, 3.0)
    assert np.abs(jx).max() < 1e-13 and np.abs(jy).max() < 1e-13
