"""Bounded rectangle with boundary states from an imaginary neighbour
(oracle, FP64).  TEST INFRASTRUCTURE ONLY, like the rest of this package.

The periodic operators of `swe` take every face neighbour from the grid.
On a bounded rectangle the faces on the domain boundary have one element
only.  Sec. 4.3 imposes the wall condition there through an imaginary
neighbour K+ whose state q+ is set from the condition, used in the numerical
fluxes and in the conservation condition of the boundary face (eqs.
reflection, reflectionBC).  Sec. 6.1 imposes the exact solution as the
boundary condition of the moving vortex without saying how; the reading
taken here follows the same principle: the imaginary neighbour's state is
the exact solution at the stage time, in both the explicit Rusanov flux
F*_NL and the hybridized flux of the implicit part.  With q+ given, the
conservation condition on a boundary face has the same closed form as on an
interior face,
    qhat = {q} + (F_L(q-) - F_L(q+)) . n- / (2 tau),
so, by the footnote to eq. linear_hdgflux3, the HDG stage equals a DG-LF
stage whose boundary flux takes q+ as its exterior state (pinned against
the dense HDG block system in the tests, and against the paper's printed
errors of Tables 1 and 2).

Layout as in `swe`: q[c, ey, ex, j, i] on an nx-by-ny grid of [0, Lx] x
[0, Ly].  Exterior states on the four sides: ext['W'], ext['E'] of shape
(3, ny, K) indexed [c, ey, j]; ext['S'], ext['N'] of shape (3, nx, K)
indexed [c, ex, i].  Traces: qx (3, ny, nx + 1, K), x-face i of row ey at
x = i hx; qy (3, ny + 1, nx, K), y-face j of column ex at y = j hy.
"""
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import imex, swe
from .hdg_dense import hdg_flux_n


def boundary_points(mesh):
    """Coordinates of the face nodes on the four sides, shaped like ext."""
    x, y = mesh.coords()
    return {'W': (x[:, 0, :, 0], y[:, 0, :, 0]),
            'E': (x[:, -1, :, -1], y[:, -1, :, -1]),
            'S': (x[0, :, 0, :], y[0, :, 0, :]),
            'N': (x[-1, :, -1, :], y[-1, :, -1, :])}


def exterior_states(mesh, state_fn, t):
    """ext[side] = state_fn(x, y, t) at the boundary face nodes."""
    return {s: np.asarray(state_fn(px, py, t), dtype=np.float64)
            for s, (px, py) in boundary_points(mesh).items()}


def reflect_exterior(mesh, q):
    """The imaginary neighbour of a wall (Sec. 4.3, eq. reflection): at every
    boundary face node phi+ = phi- and U+ = U- - 2 (U- . n) n, i.e. the
    normal momentum changes sign.  Shaped like ext."""
    k = mesh.k
    e = q[:, :, -1, :, k].copy()
    w = q[:, :, 0, :, 0].copy()
    n = q[:, -1, :, k, :].copy()
    s = q[:, 0, :, 0, :].copy()
    e[1] *= -1.0
    w[1] *= -1.0
    n[2] *= -1.0
    s[2] *= -1.0
    return {'W': w, 'E': e, 'S': s, 'N': n}


def zero_exterior(mesh):
    K = mesh.K
    return {'W': np.zeros((3, mesh.ny, K)), 'E': np.zeros((3, mesh.ny, K)),
            'S': np.zeros((3, mesh.nx, K)), 'N': np.zeros((3, mesh.nx, K))}


def neighbour_states(mesh, q, ext):
    """The four face-neighbour arrays of `swe.dg_residual`, with the
    imaginary neighbours' states on the boundary: only the neighbour's nodes
    on the shared face are read, so those are the ones replaced."""
    k = mesh.k
    east = np.roll(q, -1, axis=2)
    west = np.roll(q, 1, axis=2)
    north = np.roll(q, -1, axis=1)
    south = np.roll(q, 1, axis=1)
    east[:, :, -1, :, 0] = ext['E']
    west[:, :, 0, :, k] = ext['W']
    north[:, -1, :, 0, :] = ext['N']
    south[:, 0, :, k, :] = ext['S']
    return east, west, north, south


def dg_residual(mesh, q, phi_B, flux, numflux, ext):
    """M^-1 [ (F(q), grad v)_K - <F*(q-, q+) . n-, v>_dK ] on the bounded
    grid: `swe.dg_residual` with q+ from the imaginary neighbour on the
    boundary faces."""
    w, D, k = mesh.ref.w, mesh.ref.D, mesh.k
    sx, sy = 2.0 / mesh.hx, 2.0 / mesh.hy
    Fx, Fy = flux(q, phi_B)
    Wd = (w[:, None] * D) / w[None, :]
    out = (sx * np.einsum('cyxji,ia->cyxja', Fx, Wd)
           + sy * np.einsum('cyxji,jb->cyxbi', Fy, Wd))
    east, west, north, south = neighbour_states(mesh, q, ext)
    phi_e = numflux(q[..., :, k], east[..., :, 0], 1.0, 0.0, phi_B)
    phi_w = numflux(q[..., :, 0], west[..., :, k], -1.0, 0.0, phi_B)
    phi_n = numflux(q[..., k, :], north[..., 0, :], 0.0, 1.0, phi_B)
    phi_s = numflux(q[..., 0, :], south[..., k, :], 0.0, -1.0, phi_B)
    out[..., :, k] -= sx * phi_e / w[k]
    out[..., :, 0] -= sx * phi_w / w[0]
    out[..., k, :] -= sy * phi_n / w[k]
    out[..., 0, :] -= sy * phi_s / w[0]
    return out


def nl_residual(mesh, q, phi_B, ext):
    """M^-1 NL(q) with F*_NL = F* - F*_L (Sec. 4.3) on the bounded grid."""
    return dg_residual(mesh, q, phi_B, swe.flux_nonlinear, swe.rusanov_nonlinear, ext)


def linear_residual(mesh, q, phi_B, ext):
    """M^-1 L_DG(q) with the linear Rusanov flux on the bounded grid; equal
    to M^-1 L(q, qhat) at the HDG trace (module docstring)."""
    return dg_residual(mesh, q, phi_B, swe.flux_linear, swe.rusanov_linear, ext)


def _shift_open(n, d):
    """P[r, s] = 1 iff r = s + d with both inside [0, n) (no wrap)."""
    s = np.arange(n)
    r = s + d
    ok = (r >= 0) & (r < n)
    return sp.csr_matrix((np.ones(ok.sum()), (r[ok], s[ok])), shape=(n, n))


def assemble_linear(mesh, phi_B):
    """Sparse matrix of q -> M^-1 L_DG(q) with zero exterior states.

    The linear Rusanov flux is linear in (q-, q+), so a boundary face keeps
    the q- part of an interior face (the element's own block is unchanged)
    and its q+ part becomes data: L_DG(q; ext) = L q + L_DG(0; ext).  The
    blocks are those of the periodic grid; only the shifts stop at the
    boundary."""
    L = None
    for (dy, dx), blk in swe.linear_blocks(mesh, phi_B).items():
        P = sp.kron(_shift_open(mesh.ny, dy), _shift_open(mesh.nx, dx), format='csr')
        term = sp.kron(P, sp.csr_matrix(blk), format='csr')
        L = term if L is None else L + term
    L.eliminate_zeros()
    return L.tocsr()


def assemble_wall(mesh, phi_B):
    """Sparse matrix of q -> M^-1 L_DG(q) with walls on all four sides: the
    open-grid operator plus q -> L_DG(0; reflect_exterior(q)).  The latter
    maps an element's own face nodes to its own residual, so it is block
    diagonal; its blocks are read off by applying it to one local unit
    vector in every element at once."""
    K = mesh.K
    nloc = 3 * K * K
    nel = mesh.nx * mesh.ny
    rows, cols, vals = [], [], []
    for d in range(nloc):
        e = np.zeros((mesh.ny, mesh.nx, nloc))
        e[:, :, d] = 1.0
        q = e.reshape(mesh.ny, mesh.nx, 3, K, K).transpose(2, 0, 1, 3, 4)
        out = linear_residual(mesh, np.zeros(mesh.shape), phi_B, reflect_exterior(mesh, q))
        o = out.transpose(1, 2, 0, 3, 4).reshape(nel, nloc)
        r, c = np.nonzero(o)
        rows.extend(r * nloc + c)
        cols.extend(r * nloc + d)
        vals.extend(o[r, c])
    B = sp.csr_matrix((vals, (rows, cols)), shape=(nel * nloc, nel * nloc))
    return (assemble_linear(mesh, phi_B) + B).tocsr()


def hdg_trace(mesh, q, phi_B, ext):
    """HDG trace on every face of the bounded grid (closed form of the
    conservation condition, with the imaginary neighbour's state on the
    boundary).  Returns qx (3, ny, nx + 1, K) and qy (3, ny + 1, nx, K)."""
    k = mesh.k
    tau = math.sqrt(phi_B)

    def trace(qm, qp, nx, ny):
        Fxm, Fym = swe.flux_linear(qm, phi_B)
        Fxp, Fyp = swe.flux_linear(qp, phi_B)
        return 0.5 * (qm + qp) + ((Fxm - Fxp) * nx + (Fym - Fyp) * ny) / (2.0 * tau)

    # left / right states of every x-face, lower / upper of every y-face
    left = np.concatenate([ext['W'][:, :, None, :], q[:, :, :, :, k]], axis=2)
    right = np.concatenate([q[:, :, :, :, 0], ext['E'][:, :, None, :]], axis=2)
    low = np.concatenate([ext['S'][:, None, :, :], q[:, :, :, k, :]], axis=1)
    up = np.concatenate([q[:, :, :, 0, :], ext['N'][:, None, :, :]], axis=1)
    return trace(left, right, 1.0, 0.0), trace(low, up, 0.0, 1.0)


class BoxProblem:
    """Planar SWE with flat bottom phi_B = g H on the bounded rectangle
    [0, Lx] x [0, Ly], boundary states from `state_fn(x, y, t)` (in
    (phi_eta, U, V)) at the stage times, or walls on all four sides with
    state_fn = "wall".  The step is Algorithm 1 with the implicit stage
    system of `imex.Problem`, now affine in Q:
        (I - dt a~_ii L) Q_i = Res0_i + dt a~_ii L_DG(0; ext(t_i)),
    t_i = t_n + c~_i dt (c = c~ for the ARS schemes); NL_i uses ext(t_i).
    With walls the imaginary neighbour reflects the element's own state, so
    L is linear (the reflection is part of the matrix, no data term) and
    NL_i takes the reflection of Q_i."""

    def __init__(self, nx, ny, Lx, Ly, k, g, H, dt, state_fn, tableau=None,
                 nonlinear=True):
        self.mesh = swe.Mesh(nx, ny, Lx, Ly, k)
        self.g, self.H = float(g), float(H)
        self.phi_B = self.g * self.H
        self.dt = float(dt)
        self.state_fn = state_fn
        self.tab = tableau if tableau is not None else imex.ars443()
        if not np.allclose(self.tab.c, self.tab.ct):
            raise ValueError("boundary data at the stage times needs c = c~")
        self.nonlinear = bool(nonlinear)
        self.wall = isinstance(state_fn, str) and state_fn == "wall"
        self.Lmat = (assemble_wall(self.mesh, self.phi_B) if self.wall
                     else assemble_linear(self.mesh, self.phi_B))
        diag = np.unique(np.diag(self.tab.At)[np.diag(self.tab.At) != 0])
        if len(diag) != 1:
            raise ValueError("oracle stage solve expects an SDIRK tableau")
        self.a_ii = float(diag[0])
        n = self.Lmat.shape[0]
        stage = sp.identity(n, format='csc') - self.dt * self.a_ii * self.Lmat.tocsc()
        self.lu = spla.splu(stage.tocsc())

    def ext(self, t):
        """Boundary data at time t (None with walls: no data)."""
        if self.wall:
            return None
        return exterior_states(self.mesh, self.state_fn, t)

    def exterior(self, q, t):
        """The imaginary neighbours' states for the state q at time t."""
        return reflect_exterior(self.mesh, q) if self.wall else self.ext(t)

    def NL(self, q, ext):
        if not self.nonlinear:
            return np.zeros_like(q)
        return nl_residual(self.mesh, q, self.phi_B, ext)

    def data(self, ext):
        """L_DG(0; ext): the boundary data's part of the linear residual."""
        if ext is None:
            return np.zeros(self.mesh.shape)
        return linear_residual(self.mesh, np.zeros(self.mesh.shape), self.phi_B, ext)

    def L(self, q, ext):
        return swe.from_vec(self.Lmat @ swe.to_vec(q), self.mesh) + self.data(ext)

    def stage_solve(self, res0, ext):
        rhs = res0 + self.dt * self.a_ii * self.data(ext)
        return swe.from_vec(self.lu.solve(swe.to_vec(rhs)), self.mesh)

    def step(self, qn, t, record=None):
        tab, dt = self.tab, self.dt
        NLs, Ls = [], []
        for i in range(tab.s):
            ti = t + tab.c[i] * dt
            ext = self.ext(ti)
            if tab.At[i, i] == 0.0:
                if i != 0:
                    raise ValueError("explicit-only stage after the first")
                Q = qn
            else:
                res0 = qn.copy()
                for j in range(i):
                    res0 += dt * (tab.A[i, j] * NLs[j] + tab.At[i, j] * Ls[j])
                Q = self.stage_solve(res0, ext)
            Ls.append(self.L(Q, ext))
            NLs.append(self.NL(Q, self.exterior(Q, ti)))
            if record is not None:
                qx, qy = hdg_trace(self.mesh, Q, self.phi_B, self.exterior(Q, ti))
                record.append(dict(Q=Q, qhat_x=qx, qhat_y=qy, NL=NLs[-1], L=Ls[-1]))
        qn1 = qn.copy()
        for i in range(tab.s):
            qn1 += dt * (tab.b[i] * NLs[i] + tab.bt[i] * Ls[i])
        return qn1

    def run(self, q0, nsteps, t0=0.0):
        q = q0.copy()
        for s in range(nsteps):
            q = self.step(q, t0 + s * self.dt)
        return q


def error_norms(mesh, q, q_exact, g, H):
    """Errors of Sec. 6.1 at the final time, LGL quadrature: L1 and L2 of
    eta = h - H, L2 of u and v, and sqrt(E) with E = (||eta||^2 +
    ||u||^2) / 2 in the error (Table 2's energy norm); u = U / phi with
    phi = phi_eta + g H.  Also the largest nodal error of eta.  Returns a
    dict."""
    m = mesh.mass()
    phi_B = g * H
    eta, eta_t = q[0] / g, q_exact[0] / g
    phi, phi_t = q[0] + phi_B, q_exact[0] + phi_B
    du = q[1] / phi - q_exact[1] / phi_t
    dv = q[2] / phi - q_exact[2] / phi_t
    de = eta - eta_t
    l2 = math.sqrt(np.sum(m * de * de))
    eu = math.sqrt(np.sum(m * du * du))
    ev = math.sqrt(np.sum(m * dv * dv))
    return dict(eta_L1=float(np.sum(m * np.abs(de))), eta_L2=l2,
                eta_Linf_nodes=float(np.max(np.abs(de))), u_L2=eu, v_L2=ev,
                sqrtE=math.sqrt(0.5 * (l2 * l2 + eu * eu + ev * ev)))


# ------------------------------------------- dense HDG with boundary faces
class DenseHDGBox:
    """Dense HDG stage system on the bounded grid, assembled column by
    column from its residuals (Sec. 5, eqs. linearizedHDGsystem and
    linearizedHDGsystem_Res_Flx), with the conservation condition of a
    boundary face taken between the element and its imaginary neighbour
    (Sec. 4.3): the system is affine in (Q, qhat), its constant part comes
    from the boundary states.  Used to pin the module's reading against
    the DG-LF stage solve on tiny meshes."""

    def __init__(self, mesh, phi_B, dt_aii, ext):
        """ext: boundary data, or "wall" (the neighbour reflects the
        element's own face values, eq. reflection)."""
        self.mesh, self.phi_B, self.c, self.ext = mesh, phi_B, float(dt_aii), ext
        ny, nx, K = mesh.ny, mesh.nx, mesh.K
        self.nQ = 3 * ny * nx * K * K
        self.nX = 3 * ny * (nx + 1) * K
        self.nY = 3 * (ny + 1) * nx * K
        n = self.nQ + self.nX + self.nY
        self.b0 = self._apply(np.zeros(n), ext)
        zero = ext if isinstance(ext, str) else zero_exterior(mesh)
        M = np.zeros((n, n))
        for col in range(n):
            x = np.zeros(n)
            x[col] = 1.0
            M[:, col] = self._apply(x, zero)
        self.M = M

    def split(self, x):
        ny, nx, K = self.mesh.ny, self.mesh.nx, self.mesh.K
        Q = x[:self.nQ].reshape(3, ny, nx, K, K)
        qx = x[self.nQ:self.nQ + self.nX].reshape(3, ny, nx + 1, K)
        qy = x[self.nQ + self.nX:].reshape(3, ny + 1, nx, K)
        return Q, qx, qy

    def _L(self, Q, qx, qy):
        """M^-1 L(Q, qhat) with the hybridized flux of eq. linear_hdgflux3."""
        m, phi_B = self.mesh, self.phi_B
        w, D, k = m.ref.w, m.ref.D, m.k
        sx, sy = 2.0 / m.hx, 2.0 / m.hy
        Fx, Fy = swe.flux_linear(Q, phi_B)
        Wd = (w[:, None] * D) / w[None, :]
        out = (sx * np.einsum('cyxji,ia->cyxja', Fx, Wd)
               + sy * np.einsum('cyxji,jb->cyxbi', Fy, Wd))
        fe = hdg_flux_n(Q[..., :, k], qx[:, :, 1:], 1.0, 0.0, phi_B)
        fw = hdg_flux_n(Q[..., :, 0], qx[:, :, :-1], -1.0, 0.0, phi_B)
        fn = hdg_flux_n(Q[..., k, :], qy[:, 1:], 0.0, 1.0, phi_B)
        fs = hdg_flux_n(Q[..., 0, :], qy[:, :-1], 0.0, -1.0, phi_B)
        out[..., :, k] -= sx * fe / w[k]
        out[..., :, 0] -= sx * fw / w[0]
        out[..., k, :] -= sy * fn / w[k]
        out[..., 0, :] -= sy * fs / w[0]
        return out

    def _apply(self, x, ext):
        m, phi_B, k = self.mesh, self.phi_B, self.mesh.k
        Q, qx, qy = self.split(x)
        if isinstance(ext, str):
            ext = reflect_exterior(m, Q)
        r1 = Q - self.c * self._L(Q, qx, qy)
        # x-faces: the element on the right sees the face as its W edge
        # (n = (-1, 0)), the one on the left as its E edge (n = (1, 0));
        # beyond the boundary the imaginary neighbour takes that role
        left = np.concatenate([ext['W'][:, :, None, :], Q[:, :, :, :, k]], axis=2)
        right = np.concatenate([Q[:, :, :, :, 0], ext['E'][:, :, None, :]], axis=2)
        jx = hdg_flux_n(right, qx, -1.0, 0.0, phi_B) + hdg_flux_n(left, qx, 1.0, 0.0, phi_B)
        low = np.concatenate([ext['S'][:, None, :, :], Q[:, :, :, k, :]], axis=1)
        up = np.concatenate([Q[:, :, :, 0, :], ext['N'][:, None, :, :]], axis=1)
        jy = hdg_flux_n(up, qy, 0.0, -1.0, phi_B) + hdg_flux_n(low, qy, 0.0, 1.0, phi_B)
        return np.concatenate([r1.ravel(), jx.ravel(), jy.ravel()])

    def solve(self, res0):
        """(Q, qx, qy) with Res = 0 and Flx = 0 for Res0 = res0."""
        rhs = -self.b0
        rhs[:self.nQ] += res0.ravel()
        return self.split(np.linalg.solve(self.M, rhs))
