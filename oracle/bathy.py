"""Variable bathymetry on the periodic grid (oracle, FP64).  TEST
INFRASTRUCTURE ONLY, like the rest of this package.

With a depth B(x) below the reference plane, phi_B = g B varies in space
(Sec. 3.1, eq. psweGov).  The flux tensor keeps its form (eq.
psweFluxTensor) with phi_B at each node, the linear flux is F_L = (U,
phi_B phi_eta I) (eq. psweLinearFluxTensor), and the source
s = (0, phi_eta d_x phi_B, phi_eta d_y phi_B) belongs to the linear part L
(the semi-discrete form of Sec. 4.3).  Readings taken here:

  * phi_B is given by its nodal values; d_x phi_B, d_y phi_B are the
    derivatives of the element's nodal interpolant (the LGL derivative
    matrix), and (s, v)_K uses the collocated LGL quadrature like every
    other volume term;
  * at a face node both sides use their own nodal phi_B: tau* = max over the
    two sides of |u . n| + sqrt(phi), tau_L* = max(sqrt(phi_B-),
    sqrt(phi_B+)) (Sec. 4.3), and the HDG flux takes tau = tau_L*; the
    conservation condition then gives the same closed-form trace as with a
    constant phi_B, so the HDG stage equals the DG-LF stage of the linear
    part with this tau (the footnote to eq. linear_hdgflux3), which is what
    this module solves (a sparse LU of the assembled stage matrix).

Layout as in `swe`: q[c, ey, ex, j, i]; phiB[ey, ex, j, i].
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import imex, swe


def flux_full(q, phiB):
    """F of eq. psweFluxTensor with nodal phi_B."""
    p, U, V = q[0], q[1], q[2]
    phi = p + phiB
    Fx = np.stack([U, U * U / phi + 0.5 * p * p + p * phiB, U * V / phi])
    Fy = np.stack([V, V * U / phi, V * V / phi + 0.5 * p * p + p * phiB])
    return Fx, Fy


def flux_linear(q, phiB):
    """F_L of eq. psweLinearFluxTensor with nodal phi_B."""
    p, U, V = q[0], q[1], q[2]
    z = np.zeros_like(p)
    return np.stack([U, phiB * p, z]), np.stack([V, z, phiB * p])


def flux_nonlinear(q, phiB):
    Fx, Fy = flux_full(q, phiB)
    Lx, Ly = flux_linear(q, phiB)
    return Fx - Lx, Fy - Ly


def rusanov_full(qm, qp, bm, bp, nx, ny):
    Fxm, Fym = flux_full(qm, bm)
    Fxp, Fyp = flux_full(qp, bp)
    sm = np.abs((qm[1] * nx + qm[2] * ny) / (qm[0] + bm)) + np.sqrt(qm[0] + bm)
    sp_ = np.abs((qp[1] * nx + qp[2] * ny) / (qp[0] + bp)) + np.sqrt(qp[0] + bp)
    tau = np.maximum(sm, sp_)
    return 0.5 * ((Fxm + Fxp) * nx + (Fym + Fyp) * ny) + 0.5 * tau * (qm - qp)


def rusanov_linear(qm, qp, bm, bp, nx, ny):
    Fxm, Fym = flux_linear(qm, bm)
    Fxp, Fyp = flux_linear(qp, bp)
    tau = np.maximum(np.sqrt(bm), np.sqrt(bp))
    return 0.5 * ((Fxm + Fxp) * nx + (Fym + Fyp) * ny) + 0.5 * tau * (qm - qp)


def rusanov_nonlinear(qm, qp, bm, bp, nx, ny):
    return rusanov_full(qm, qp, bm, bp, nx, ny) - rusanov_linear(qm, qp, bm, bp, nx, ny)


def grad_phiB(mesh, phiB):
    """Nodal derivatives of each element's interpolant of phi_B."""
    D = mesh.ref.D
    dx = (2.0 / mesh.hx) * np.einsum('ai,yxji->yxja', D, phiB)
    dy = (2.0 / mesh.hy) * np.einsum('bj,yxji->yxbi', D, phiB)
    return dx, dy


def dg_residual(mesh, q, phiB, flux, numflux, source=False):
    """M^-1 [ (F(q), grad v)_K + (s(q), v)_K - <F*(q-, q+) . n-, v>_dK ]
    with nodal phi_B on both sides of every face (periodic grid); the
    source term only with source=True (the linear part)."""
    w, D, k = mesh.ref.w, mesh.ref.D, mesh.k
    sx, sy = 2.0 / mesh.hx, 2.0 / mesh.hy
    Fx, Fy = flux(q, phiB)
    Wd = (w[:, None] * D) / w[None, :]
    out = (sx * np.einsum('cyxji,ia->cyxja', Fx, Wd)
           + sy * np.einsum('cyxji,jb->cyxbi', Fy, Wd))
    if source:
        gx, gy = grad_phiB(mesh, phiB)
        out[1] += q[0] * gx
        out[2] += q[0] * gy
    east, west = np.roll(q, -1, axis=2), np.roll(q, 1, axis=2)
    north, south = np.roll(q, -1, axis=1), np.roll(q, 1, axis=1)
    bE, bW = np.roll(phiB, -1, axis=1), np.roll(phiB, 1, axis=1)
    bN, bS = np.roll(phiB, -1, axis=0), np.roll(phiB, 1, axis=0)
    phi_e = numflux(q[..., :, k], east[..., :, 0], phiB[..., :, k], bE[..., :, 0], 1.0, 0.0)
    phi_w = numflux(q[..., :, 0], west[..., :, k], phiB[..., :, 0], bW[..., :, k], -1.0, 0.0)
    phi_n = numflux(q[..., k, :], north[..., 0, :], phiB[..., k, :], bN[..., 0, :], 0.0, 1.0)
    phi_s = numflux(q[..., 0, :], south[..., k, :], phiB[..., 0, :], bS[..., k, :], 0.0, -1.0)
    out[..., :, k] -= sx * phi_e / w[k]
    out[..., :, 0] -= sx * phi_w / w[0]
    out[..., k, :] -= sy * phi_n / w[k]
    out[..., 0, :] -= sy * phi_s / w[0]
    return out


def nl_residual(mesh, q, phiB):
    return dg_residual(mesh, q, phiB, flux_nonlinear, rusanov_nonlinear)


def linear_residual(mesh, q, phiB):
    """M^-1 L(q): linear flux, Lax-Friedrichs flux with tau_L*, source."""
    return dg_residual(mesh, q, phiB, flux_linear, rusanov_linear, source=True)


def _period(n):
    """Smallest m >= 3 dividing n: elements whose indices agree mod m are at
    least 3 apart, also across the periodic wrap."""
    return next(m for m in range(3, n + 1) if n % m == 0)


def assemble_linear(mesh, phiB):
    """Sparse matrix of q -> M^-1 L(q), element-major ordering
    [ey][ex][c][j][i].  The operator couples an element only to itself and
    its four face neighbours, so the column of local unit vector d of
    element e is the residual of that vector, read at e and its neighbours.
    Elements of one colour (indices equal modulo `_period`) have disjoint
    neighbourhoods, so one residual evaluation serves the whole colour.
    Needs nx, ny >= 3."""
    ny, nx, K = mesh.ny, mesh.nx, mesh.K
    if nx < 3 or ny < 3:
        raise ValueError("needs at least 3 x 3 elements")
    nloc = 3 * K * K
    my, mx = _period(ny), _period(nx)
    offsets = [(0, 0), (0, 1), (0, -1), (1, 0), (-1, 0)]
    rows, cols, vals = [], [], []
    for cy in range(my):
        for cx in range(mx):
            for d in range(nloc):
                e = np.zeros((ny, nx, nloc))
                e[cy::my, cx::mx, d] = 1.0
                q = e.reshape(ny, nx, 3, K, K).transpose(2, 0, 1, 3, 4)
                out = linear_residual(mesh, q, phiB).transpose(1, 2, 0, 3, 4)
                out = out.reshape(ny, nx, nloc)
                for ey in range(cy, ny, my):
                    for ex in range(cx, nx, mx):
                        for dy, dx in offsets:
                            ty, tx = (ey + dy) % ny, (ex + dx) % nx
                            v = out[ty, tx]
                            nz = np.nonzero(v)[0]
                            rows.extend((ty * nx + tx) * nloc + nz)
                            cols.extend([(ey * nx + ex) * nloc + d] * len(nz))
                            vals.extend(v[nz])
    n = nx * ny * nloc
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


class BathyProblem:
    """Periodic planar SWE over nodal phi_B = g B (Algorithm 1 as in
    `imex.Problem`; the stage system solved by an LU of I - dt a~_ii L)."""

    def __init__(self, nx, ny, Lx, Ly, k, g, B, dt, tableau=None, nonlinear=True):
        """B: nodal depth, shape (ny, nx, K, K), positive."""
        self.mesh = swe.Mesh(nx, ny, Lx, Ly, k)
        self.g = float(g)
        self.phiB = self.g * np.asarray(B, dtype=np.float64)
        self.dt = float(dt)
        self.tab = tableau if tableau is not None else imex.ars232()
        self.nonlinear = bool(nonlinear)
        self.Lmat = assemble_linear(self.mesh, self.phiB)
        diag = np.unique(np.diag(self.tab.At)[np.diag(self.tab.At) != 0])
        if len(diag) != 1:
            raise ValueError("oracle stage solve expects an SDIRK tableau")
        self.a_ii = float(diag[0])
        n = self.Lmat.shape[0]
        stage = sp.identity(n, format='csc') - self.dt * self.a_ii * self.Lmat.tocsc()
        self.lu = spla.splu(stage.tocsc())

    def NL(self, q):
        if not self.nonlinear:
            return np.zeros_like(q)
        return nl_residual(self.mesh, q, self.phiB)

    def L(self, q):
        return swe.from_vec(self.Lmat @ swe.to_vec(q), self.mesh)

    def stage_solve(self, res0):
        return swe.from_vec(self.lu.solve(swe.to_vec(res0)), self.mesh)

    def step(self, qn):
        tab, dt = self.tab, self.dt
        NLs, Ls = [], []
        for i in range(tab.s):
            if tab.At[i, i] == 0.0:
                Q = qn
            else:
                res0 = qn.copy()
                for j in range(i):
                    res0 += dt * (tab.A[i, j] * NLs[j] + tab.At[i, j] * Ls[j])
                Q = self.stage_solve(res0)
            Ls.append(self.L(Q))
            NLs.append(self.NL(Q))
        qn1 = qn.copy()
        for i in range(tab.s):
            qn1 += dt * (tab.b[i] * NLs[i] + tab.bt[i] * Ls[i])
        return qn1

    def run(self, q0, nsteps):
        q = q0.copy()
        for _ in range(nsteps):
            q = self.step(q)
        return q
