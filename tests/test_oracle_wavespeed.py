"""Pins of the Rusanov wave speeds tau* and tau_L* (Sec. 4.3, eqs.
Full_russanov and Linear_russanov).

The paper calls tau* the advection plus gravity wave speed: the largest
characteristic speed of the flux in the direction n, i.e. the spectral
radius of the flux Jacobian d(F(q) . n)/dq.  These tests form that Jacobian
by complex-step differentiation of the (separately pinned) flux, take its
eigenvalues with numpy, and check the oracle's wave speed and the
dissipation of its Rusanov fluxes against them.  A wave speed built from the
wrong geopotential (phi_B in place of phi), from u = U / phi_B, or without
the maximum over the two sides fails here; the pins on continuous data
cannot see it, because there the jump q- - q+ is zero.
"""
import numpy as np
import pytest

from oracle import swe


def _subcritical_states(rng, n, phi_B):
    """States (phi_eta, U, V) with phi = phi_eta + phi_B > 0 and |u| well
    below sqrt(phi) (the subcritical regime of Sec. 3)."""
    p = phi_B * rng.uniform(-0.4, 0.6, n)
    phi = p + phi_B
    speed = np.sqrt(phi) * rng.uniform(0.0, 0.9, n)
    ang = rng.uniform(0.0, 2.0 * np.pi, n)
    U = phi * speed * np.cos(ang)
    V = phi * speed * np.sin(ang)
    return np.stack([p, U, V])


def _normals(rng, n):
    a = rng.uniform(0.0, 2.0 * np.pi, n)
    return np.cos(a), np.sin(a)


def _jacobian_n(flux, q, nx, ny, phi_B):
    """d(F(q) . n)/dq at one state by complex steps (exact to rounding)."""
    h = 1e-30
    J = np.zeros((3, 3))
    for j in range(3):
        qc = q.astype(np.complex128)
        qc[j] += 1j * h
        Fx, Fy = flux(qc, phi_B)
        J[:, j] = (Fx * nx + Fy * ny).imag / h
    return J


def _spectral_radius(J):
    return float(np.max(np.abs(np.linalg.eigvals(J))))


@pytest.mark.parametrize("phi_B", [1.0, 9.81, 100.0])
def test_wave_speed_is_spectral_radius_of_flux_jacobian(phi_B):
    rng = np.random.default_rng(11)
    n = 120
    q = _subcritical_states(rng, n, phi_B)
    nx, ny = _normals(rng, n)
    got = swe.wave_speed(q, phi_B, nx, ny)
    for i in range(n):
        J = _jacobian_n(swe.flux_full, q[:, i], nx[i], ny[i], phi_B)
        rho = _spectral_radius(J)
        assert abs(got[i] - rho) <= 1e-8 * rho, (i, got[i], rho)


def test_linear_flux_speed_is_sqrt_phi_B():
    """tau_L* = sqrt(phi_B): the spectral radius of the linearised flux
    Jacobian, the same at every state and unit normal."""
    rng = np.random.default_rng(12)
    for phi_B in (0.5, 9.81, 100.0):
        q = _subcritical_states(rng, 20, phi_B)
        nx, ny = _normals(rng, 20)
        for i in range(20):
            J = _jacobian_n(swe.flux_linear, q[:, i], nx[i], ny[i], phi_B)
            assert abs(_spectral_radius(J) - np.sqrt(phi_B)) <= 1e-12 * np.sqrt(phi_B)


def _central(flux, qm, qp, nx, ny, phi_B):
    Fxm, Fym = flux(qm, phi_B)
    Fxp, Fyp = flux(qp, phi_B)
    return 0.5 * ((Fxm + Fxp) * nx + (Fym + Fyp) * ny)


@pytest.mark.parametrize("phi_B", [1.0, 9.81])
def test_rusanov_dissipation_uses_the_larger_side(phi_B):
    """F*(q-, q+) . n- minus the central flux is tau*/2 (q- - q+) with tau*
    the larger of the two sides' spectral radii; for the linear flux the
    coefficient is sqrt(phi_B)/2; the nonlinear remainder F*_NL carries
    (tau* - tau_L*)/2 (Sec. 4.3)."""
    rng = np.random.default_rng(13)
    n = 100
    qm = _subcritical_states(rng, n, phi_B)
    qp = _subcritical_states(rng, n, phi_B)
    nx, ny = _normals(rng, n)
    full = swe.rusanov_full(qm, qp, nx, ny, phi_B) - _central(swe.flux_full, qm, qp, nx, ny, phi_B)
    lin = swe.rusanov_linear(qm, qp, nx, ny, phi_B) - _central(swe.flux_linear, qm, qp, nx, ny,
                                                               phi_B)
    nl = (swe.rusanov_nonlinear(qm, qp, nx, ny, phi_B)
          - _central(swe.flux_nonlinear, qm, qp, nx, ny, phi_B))
    for i in range(n):
        rm = _spectral_radius(_jacobian_n(swe.flux_full, qm[:, i], nx[i], ny[i], phi_B))
        rp = _spectral_radius(_jacobian_n(swe.flux_full, qp[:, i], nx[i], ny[i], phi_B))
        tau = max(rm, rp)
        jump = qm[:, i] - qp[:, i]
        scale = np.abs(jump).max() * tau
        np.testing.assert_allclose(full[:, i], 0.5 * tau * jump, rtol=0, atol=1e-10 * scale)
        np.testing.assert_allclose(lin[:, i], 0.5 * np.sqrt(phi_B) * jump, rtol=0,
                                   atol=1e-12 * scale)
        np.testing.assert_allclose(nl[:, i], 0.5 * (tau - np.sqrt(phi_B)) * jump, rtol=0,
                                   atol=1e-10 * scale)


def test_nl_residual_face_term_on_a_jump():
    """The face term of the assembled NL residual on discontinuous data.

    The state is constant on each element and varies with the element
    column only, so the y faces see no jump and the x faces of element
    column ex see q- (own) and q+ (east neighbour).  For a constant
    element state the weak volume term at the east face nodes is
    (2/hx) F_x(q-) / w_k (summation by parts: sum_i w_i D_ia = delta_ak -
    delta_a0), hence at a middle-row east face node
        Phi_E = F_x,NL(q-) - (hx/2) w_k M^-1 NL,
    which must equal {F_NL} . n + (tau* - tau_L*)/2 (q- - q+) with tau* the
    larger spectral radius of the two sides' flux Jacobians."""
    rng = np.random.default_rng(14)
    phi_B, k = 9.81, 3
    mesh = swe.Mesh(4, 3, 1.0, 0.9, k)
    cols = _subcritical_states(rng, mesh.nx, phi_B)      # one state per element column
    q = np.zeros(mesh.shape)
    for ex in range(mesh.nx):
        q[:, :, ex] = cols[:, ex][:, None, None, None]
    r = swe.nl_residual(mesh, q, phi_B)
    w = mesh.ref.w
    jm = k // 2 if k % 2 == 0 else 1                      # a middle row (not 0, not k)
    for ex in range(mesh.nx):
        qm = cols[:, ex]
        qp = cols[:, (ex + 1) % mesh.nx]
        FxNL, _ = swe.flux_nonlinear(qm, phi_B)
        phi_e = FxNL - (mesh.hx / 2.0) * w[k] * r[:, 0, ex, jm, k]
        rm = _spectral_radius(_jacobian_n(swe.flux_full, qm, 1.0, 0.0, phi_B))
        rp = _spectral_radius(_jacobian_n(swe.flux_full, qp, 1.0, 0.0, phi_B))
        FxNLp, _ = swe.flux_nonlinear(qp, phi_B)
        want = 0.5 * (FxNL + FxNLp) + 0.5 * (max(rm, rp) - np.sqrt(phi_B)) * (qm - qp)
        np.testing.assert_allclose(phi_e, want, rtol=0, atol=1e-11 * (1 + np.abs(want).max()))
