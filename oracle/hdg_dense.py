"""Brute-force dense HDG stage system for tiny meshes (oracle, FP64).

Assembles, column by column, the full block system of Sec. 5 (eq.
linearizedHDGsystem)
    [A B; C D] (Q, Qhat) = (R1, 0)
from the two residuals that define it (eq. linearizedHDGsystem_Res_Flx):
    Res(Q, Qhat) = Q - dt a~_ii M^-1 L(Q, Qhat) - Res0
    Flx(Q, Qhat) = < [[Fhat_L(Q, Qhat) . n]], mu >   on every face
with the hybridized Lax-Friedrichs flux of eq. linear_hdgflux3.  The edge
inner product uses LGL quadrature, which is nondegenerate on P_k, so Flx = 0
for all mu in P_k is the vanishing of [[Fhat_L . n]] at every edge node.

Used by the tests to pin the oracle's stage solve: the dense block solve,
the explicit Schur complement of eq. linearizedHDGsystem_schur with the
recovery of eq. recover_volume_unknowns, and the DG-LF solve must agree.
"""
import numpy as np

from . import swe


def _lift(mesh, fe, fw, fn, fs):
    """M^-1 of <Phi, v>_dK for face fluxes given on the four edges."""
    w, k = mesh.ref.w, mesh.k
    sx, sy = 2.0 / mesh.hx, 2.0 / mesh.hy
    out = np.zeros(mesh.shape)
    out[..., :, k] += sx * fe / w[k]
    out[..., :, 0] += sx * fw / w[0]
    out[..., k, :] += sy * fn / w[k]
    out[..., 0, :] += sy * fs / w[0]
    return out


def _edge_states(mesh, Q, qx, qy):
    """Interior state and trace on the E, W, N, S edges of every element.

    x-face e is the west face of element e; its east face is the x-face of
    the east neighbour.  Likewise for y-faces (south / north)."""
    k = mesh.k
    qx_east = np.roll(qx, -1, axis=2)
    qy_north = np.roll(qy, -1, axis=1)
    return {
        'E': (Q[..., :, k], qx_east, 1.0, 0.0),
        'W': (Q[..., :, 0], qx, -1.0, 0.0),
        'N': (Q[..., k, :], qy_north, 0.0, 1.0),
        'S': (Q[..., 0, :], qy, 0.0, -1.0),
    }


def hdg_flux_n(q, qhat, nx, ny, phi_B):
    """n . Fhat_L(q, qhat) of eq. linear_hdgflux3."""
    t = np.sqrt(phi_B)
    p, U, V = q[0], q[1], q[2]
    return np.stack([nx * U + ny * V + t * (p - qhat[0]),
                     nx * phi_B * p + t * (U - qhat[1]),
                     ny * phi_B * p + t * (V - qhat[2])])


def hdg_L(mesh, Q, qx, qy, phi_B):
    """M^-1 L(Q, Qhat) = M^-1 [ (F_L(Q), grad v) - <Fhat_L . n, v> ]."""
    w, D = mesh.ref.w, mesh.ref.D
    sx, sy = 2.0 / mesh.hx, 2.0 / mesh.hy
    Fx, Fy = swe.flux_linear(Q, phi_B)
    Wd = (w[:, None] * D) / w[None, :]
    vol = (sx * np.einsum('cyxji,ia->cyxja', Fx, Wd)
           + sy * np.einsum('cyxji,jb->cyxbi', Fy, Wd))
    ed = _edge_states(mesh, Q, qx, qy)
    f = {s: hdg_flux_n(q, qh, nx, ny, phi_B) for s, (q, qh, nx, ny) in ed.items()}
    return vol - _lift(mesh, f['E'], f['W'], f['N'], f['S'])


def hdg_conservation(mesh, Q, qx, qy, phi_B):
    """[[Fhat_L . n]] at every face node: x-faces then y-faces."""
    k = mesh.k
    west = np.roll(Q, 1, axis=2)
    south = np.roll(Q, 1, axis=1)
    # x-face e: element e sees it as its W edge (n = (-1, 0)), the west
    # neighbour as its E edge (n = (1, 0)).
    jx = (hdg_flux_n(Q[..., :, 0], qx, -1.0, 0.0, phi_B)
          + hdg_flux_n(west[..., :, k], qx, 1.0, 0.0, phi_B))
    jy = (hdg_flux_n(Q[..., 0, :], qy, 0.0, -1.0, phi_B)
          + hdg_flux_n(south[..., k, :], qy, 0.0, 1.0, phi_B))
    return jx, jy


class DenseHDG:
    """Dense [A B; C D] of one implicit stage with coefficient dt*a_ii."""

    def __init__(self, mesh, phi_B, dt_aii):
        self.mesh, self.phi_B, self.c = mesh, phi_B, float(dt_aii)
        ny, nx, K = mesh.ny, mesh.nx, mesh.K
        self.nQ = 3 * ny * nx * K * K
        self.nT = 2 * 3 * ny * nx * K
        n = self.nQ + self.nT
        M = np.zeros((n, n))
        for col in range(n):
            x = np.zeros(n)
            x[col] = 1.0
            M[:, col] = self._apply(x)
        self.M = M

    def split(self, x):
        ny, nx, K = self.mesh.ny, self.mesh.nx, self.mesh.K
        Q = x[:self.nQ].reshape(3, ny, nx, K, K)
        t = x[self.nQ:].reshape(2, 3, ny, nx, K)
        return Q, t[0], t[1]

    def join(self, Q, qx, qy):
        return np.concatenate([Q.ravel(), qx.ravel(), qy.ravel()])

    def _apply(self, x):
        """Linear part of (Res, Flx); the Res0 term is moved to the RHS."""
        Q, qx, qy = self.split(x)
        r1 = Q - self.c * hdg_L(self.mesh, Q, qx, qy, self.phi_B)
        jx, jy = hdg_conservation(self.mesh, Q, qx, qy, self.phi_B)
        return np.concatenate([r1.ravel(), jx.ravel(), jy.ravel()])

    def solve_full(self, res0):
        rhs = np.concatenate([res0.ravel(), np.zeros(self.nT)])
        return self.split(np.linalg.solve(self.M, rhs))

    def solve_schur(self, res0):
        """Static condensation: (D - C A^-1 B) Qhat = R2 - C A^-1 R1, then
        Q = A^-1 (R1 - B Qhat)."""
        nQ = self.nQ
        A, B = self.M[:nQ, :nQ], self.M[:nQ, nQ:]
        C, D = self.M[nQ:, :nQ], self.M[nQ:, nQ:]
        R1 = res0.ravel()
        AiB = np.linalg.solve(A, B)
        AiR = np.linalg.solve(A, R1)
        qhat = np.linalg.solve(D - C @ AiB, -C @ AiR)
        Q = AiR - AiB @ qhat
        return self.split(np.concatenate([Q, qhat]))
