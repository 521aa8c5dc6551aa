"""Closed basin: reflecting walls on the four sides of the rectangle over a
variable depth (oracle, FP64).  TEST INFRASTRUCTURE ONLY, like the rest of
this package.

The two bounded-domain ingredients are those of `box` (walls) and `bathy`
(nodal phi_B with its source term), taken together:

  * at a wall face the imaginary neighbour K+ carries the reflected state
    (Sec. 4.3, eq. reflection: phi_eta and the tangential momentum kept, the
    normal momentum negated) in the explicit Rusanov flux and in the
    hybridized flux of the implicit part;
  * the neighbour's phi_B at the face node is the element's own (the depth
    mirrored across the wall), so tau* and tau_L* of the wall face use one
    depth, and the conservation condition keeps the closed form of `box`;
    by the footnote to eq. linear_hdgflux3 the HDG stage is again the DG-LF
    stage with the reflected exterior state, which this module solves (a
    sparse LU of the assembled stage matrix).

Layout as in `swe`: q[c, ey, ex, j, i]; phiB[ey, ex, j, i].
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import bathy, box, imex, swe


def neighbour_depths(mesh, phiB):
    """The four neighbour phi_B arrays of the residual: the grid neighbour's
    inside the basin, the element's own face values across a wall."""
    k = mesh.k
    east, west = np.roll(phiB, -1, axis=1), np.roll(phiB, 1, axis=1)
    north, south = np.roll(phiB, -1, axis=0), np.roll(phiB, 1, axis=0)
    east[:, -1, :, 0] = phiB[:, -1, :, k]
    west[:, 0, :, k] = phiB[:, 0, :, 0]
    north[-1, :, 0, :] = phiB[-1, :, k, :]
    south[0, :, k, :] = phiB[0, :, 0, :]
    return east, west, north, south


def dg_residual(mesh, q, phiB, flux, numflux, source=False):
    """M^-1 [ (F(q), grad v)_K + (s(q), v)_K - <F*(q-, q+) . n-, v>_dK ] in
    the basin: `bathy.dg_residual` with the reflected state and the mirrored
    depth as the wall faces' exterior; the source term only with
    source=True (the linear part)."""
    w, D, k = mesh.ref.w, mesh.ref.D, mesh.k
    sx, sy = 2.0 / mesh.hx, 2.0 / mesh.hy
    Fx, Fy = flux(q, phiB)
    Wd = (w[:, None] * D) / w[None, :]
    out = (sx * np.einsum('cyxji,ia->cyxja', Fx, Wd)
           + sy * np.einsum('cyxji,jb->cyxbi', Fy, Wd))
    if source:
        gx, gy = bathy.grad_phiB(mesh, phiB)
        out[1] += q[0] * gx
        out[2] += q[0] * gy
    east, west, north, south = box.neighbour_states(mesh, q, box.reflect_exterior(mesh, q))
    bE, bW, bN, bS = neighbour_depths(mesh, phiB)
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
    return dg_residual(mesh, q, phiB, bathy.flux_nonlinear, bathy.rusanov_nonlinear)


def linear_residual(mesh, q, phiB):
    """M^-1 L(q) in the basin: linear flux, Lax-Friedrichs flux with tau_L*,
    source; linear in q (the reflection is linear)."""
    return dg_residual(mesh, q, phiB, bathy.flux_linear, bathy.rusanov_linear, source=True)


def assemble_linear(mesh, phiB):
    """Sparse matrix of q -> M^-1 L(q), element-major ordering
    [ey][ex][c][j][i].  An element couples to itself and its face
    neighbours only (the wall terms to itself), so elements whose indices
    agree modulo 3 in both directions have disjoint neighbourhoods (no wrap
    in a basin) and one residual evaluation per local unit vector serves
    the whole colour."""
    ny, nx, K = mesh.ny, mesh.nx, mesh.K
    nloc = 3 * K * K
    offsets = [(0, 0), (0, 1), (0, -1), (1, 0), (-1, 0)]
    rows, cols, vals = [], [], []
    for cy in range(3):
        for cx in range(3):
            for d in range(nloc):
                e = np.zeros((ny, nx, nloc))
                e[cy::3, cx::3, d] = 1.0
                if not e.any():
                    continue
                q = e.reshape(ny, nx, 3, K, K).transpose(2, 0, 1, 3, 4)
                out = linear_residual(mesh, q, phiB).transpose(1, 2, 0, 3, 4)
                out = out.reshape(ny, nx, nloc)
                for ey in range(cy, ny, 3):
                    for ex in range(cx, nx, 3):
                        for dy, dx in offsets:
                            ty, tx = ey + dy, ex + dx
                            if not (0 <= ty < ny and 0 <= tx < nx):
                                continue
                            v = out[ty, tx]
                            nz = np.nonzero(v)[0]
                            rows.extend((ty * nx + tx) * nloc + nz)
                            cols.extend([(ey * nx + ex) * nloc + d] * len(nz))
                            vals.extend(v[nz])
    n = nx * ny * nloc
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n))


class BasinProblem:
    """Planar SWE in the walled rectangle [0, Lx] x [0, Ly] over nodal
    phi_B = g B (Algorithm 1 as in `imex.Problem`; the stage system solved
    by an LU of I - dt a~_ii L)."""

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
