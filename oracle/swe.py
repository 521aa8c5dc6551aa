"""Planar shallow-water DG operators (oracle, FP64, NumPy/SciPy).

State layout: q[c, ey, ex, j, i] with c in (phi_eta, U, V) (Sec. 3.1: the
conservative variables are (g eta, phi u, phi v)), (ey, ex) the element row
and column of a periodic nx-by-ny grid of hx-by-hy rectangles on
[0, Lx) x [0, Ly), and (j, i) the LGL node indices along y and x.

Semi-discrete form (Sec. 4.3, eq. SemiDiscretizedForm_ode):
    (dq/dt, v)_K = NL(q) + L(q, qhat)
    NL(q) = (F_NL(q), grad v)_K - <F*_NL(q+-) . n, v>_dK
    L(q)  = (F_L(q),  grad v)_K - <Fhat_L(q, qhat) . n, v>_dK
with F_NL = F - F_L and F*_NL = F* - F*_L (Sec. 4.3, eqs. Full_russanov and
Linear_russanov).  Inner products use LGL quadrature on the element and on
its edges, so the mass matrix is diagonal, (hx/2)(hy/2) w_i w_j.

Flat bottom everywhere: phi_B = g H is a constant and the source term
s = (0, phi_eta d_x phi_B, phi_eta d_y phi_B) of eq. psweGov vanishes.
"""
import numpy as np
import scipy.sparse as sp

from .lgl import RefElement


class Mesh:
    """Periodic nx-by-ny grid of affine rectangles with degree-k LGL nodes."""

    def __init__(self, nx, ny, Lx, Ly, k):
        self.nx, self.ny = int(nx), int(ny)
        self.Lx, self.Ly = float(Lx), float(Ly)
        self.ref = RefElement(k)
        self.k, self.K = k, k + 1
        self.hx = self.Lx / self.nx
        self.hy = self.Ly / self.ny

    @property
    def shape(self):
        return (3, self.ny, self.nx, self.K, self.K)

    @property
    def n_nodes(self):
        return self.nx * self.ny * self.K * self.K

    def coords(self):
        """Node coordinates x[ey, ex, j, i], y[ey, ex, j, i]."""
        xi = self.ref.x
        ex = np.arange(self.nx)[None, :, None, None]
        ey = np.arange(self.ny)[:, None, None, None]
        x = (ex + (xi[None, None, None, :] + 1.0) / 2.0) * self.hx
        y = (ey + (xi[None, None, :, None] + 1.0) / 2.0) * self.hy
        x = np.broadcast_to(x, (self.ny, self.nx, self.K, self.K)).copy()
        y = np.broadcast_to(y, (self.ny, self.nx, self.K, self.K)).copy()
        return x, y

    def mass(self):
        """Diagonal LGL mass (hx/2)(hy/2) w_i w_j, shape (ny, nx, K, K)."""
        w = self.ref.w
        m = (self.hx / 2.0) * (self.hy / 2.0) * w[:, None] * w[None, :]
        return np.broadcast_to(m, (self.ny, self.nx, self.K, self.K))

    def min_node_spacing(self):
        dxi = np.min(np.diff(self.ref.x))
        return min(dxi * self.hx / 2.0, dxi * self.hy / 2.0)


# ---------------------------------------------------------------- fluxes
def flux_full(q, phi_B):
    """Flux tensor F = (F_x, F_y) of eq. psweFluxTensor."""
    p, U, V = q[0], q[1], q[2]
    phi = p + phi_B
    Fx = np.stack([U, U * U / phi + 0.5 * p * p + p * phi_B, U * V / phi])
    Fy = np.stack([V, V * U / phi, V * V / phi + 0.5 * p * p + p * phi_B])
    return Fx, Fy


def flux_linear(q, phi_B):
    """Flux linearised about the lake at rest, eq. psweLinearFluxTensor."""
    p, U, V = q[0], q[1], q[2]
    z = np.zeros_like(p)
    Fx = np.stack([U, phi_B * p, z])
    Fy = np.stack([V, z, phi_B * p])
    return Fx, Fy


def flux_nonlinear(q, phi_B):
    """F_NL := F - F_L (Sec. 4.3)."""
    Fx, Fy = flux_full(q, phi_B)
    Lx, Ly = flux_linear(q, phi_B)
    return Fx - Lx, Fy - Ly


def wave_speed(q, phi_B, nx, ny):
    """|u . n| + sqrt(phi) with phi the total geopotential and u = U / phi."""
    phi = q[0] + phi_B
    un = (q[1] * nx + q[2] * ny) / phi
    return np.abs(un) + np.sqrt(phi)


def rusanov_full(qm, qp, nx, ny, phi_B):
    """F*(q-, q+) . n-  (eq. Full_russanov), jump [[q (x) n]] = (q- - q+) n-."""
    Fxm, Fym = flux_full(qm, phi_B)
    Fxp, Fyp = flux_full(qp, phi_B)
    tau = np.maximum(wave_speed(qm, phi_B, nx, ny), wave_speed(qp, phi_B, nx, ny))
    return 0.5 * ((Fxm + Fxp) * nx + (Fym + Fyp) * ny) + 0.5 * tau * (qm - qp)


def rusanov_linear(qm, qp, nx, ny, phi_B):
    """F*_L(q-, q+) . n-  (eq. Linear_russanov), tau_L* = max(sqrt(phi_B+-))."""
    Fxm, Fym = flux_linear(qm, phi_B)
    Fxp, Fyp = flux_linear(qp, phi_B)
    tau_L = np.sqrt(phi_B)
    return 0.5 * ((Fxm + Fxp) * nx + (Fym + Fyp) * ny) + 0.5 * tau_L * (qm - qp)


def rusanov_nonlinear(qm, qp, nx, ny, phi_B):
    """F*_NL := F* - F*_L, the nonlinear DG numerical flux (Sec. 4.3)."""
    return (rusanov_full(qm, qp, nx, ny, phi_B)
            - rusanov_linear(qm, qp, nx, ny, phi_B))


# ------------------------------------------------------ DG weak residual
def dg_residual(mesh, q, phi_B, flux, numflux):
    """M^-1 [ (F(q), grad v)_K - <F*(q-, q+) . n-, v>_dK ] at every node.

    v = l_a(xi) l_b(eta).  With LGL quadrature on the element
      (F_x, d_x v)_K / M_ab = (2/hx) sum_i (w_i / w_a) D[i, a] F_x(i, b)
    and on the east edge (xi = 1), for example,
      <Phi, v>_E / M_ab = (2/hx) delta_{a k} Phi_b / w_k.
    The exterior state q+ is the coincident node of the periodic neighbour.
    """
    w, D, k = mesh.ref.w, mesh.ref.D, mesh.k
    sx, sy = 2.0 / mesh.hx, 2.0 / mesh.hy
    Fx, Fy = flux(q, phi_B)
    Wd = (w[:, None] * D) / w[None, :]          # Wd[i, a] = w_i D_ia / w_a
    out = (sx * np.einsum('cyxji,ia->cyxja', Fx, Wd)
           + sy * np.einsum('cyxji,jb->cyxbi', Fy, Wd))

    east = np.roll(q, -1, axis=2)    # element (ey, ex + 1)
    west = np.roll(q, 1, axis=2)     # element (ey, ex - 1)
    north = np.roll(q, -1, axis=1)   # element (ey + 1, ex)
    south = np.roll(q, 1, axis=1)    # element (ey - 1, ex)

    phi_e = numflux(q[..., :, k], east[..., :, 0], 1.0, 0.0, phi_B)
    phi_w = numflux(q[..., :, 0], west[..., :, k], -1.0, 0.0, phi_B)
    phi_n = numflux(q[..., k, :], north[..., 0, :], 0.0, 1.0, phi_B)
    phi_s = numflux(q[..., 0, :], south[..., k, :], 0.0, -1.0, phi_B)

    out[..., :, k] -= sx * phi_e / w[k]
    out[..., :, 0] -= sx * phi_w / w[0]
    out[..., k, :] -= sy * phi_n / w[k]
    out[..., 0, :] -= sy * phi_s / w[0]
    return out


def nl_residual(mesh, q, phi_B):
    """M^-1 NL(q): DG residual of the nonlinear part with F*_NL."""
    return dg_residual(mesh, q, phi_B, flux_nonlinear, rusanov_nonlinear)


def linear_dglf_residual(mesh, q, phi_B):
    """M^-1 L_DG(q): DG residual of the linear part with the linear Rusanov
    (Lax-Friedrichs) flux.  On a polygonal mesh the hybridized flux
    Fhat_L and F*_L coincide once qhat is eliminated (footnote to eq.
    linear_hdgflux3), so this equals M^-1 L(q, qhat) at the HDG trace."""
    return dg_residual(mesh, q, phi_B, flux_linear, rusanov_linear)


# ------------------------------------------------ sparse linear operator
def to_vec(q):
    """(3, ny, nx, K, K) -> element-major vector [ey][ex][c][j][i]."""
    return np.ascontiguousarray(q.transpose(1, 2, 0, 3, 4)).ravel()


def from_vec(v, mesh):
    ny, nx, K = mesh.ny, mesh.nx, mesh.K
    return np.ascontiguousarray(v.reshape(ny, nx, 3, K, K).transpose(2, 0, 1, 3, 4))


def _shift(n, d):
    """P[r, s] = 1 iff r = s + d (mod n)."""
    r = (np.arange(n) + d) % n
    return sp.csr_matrix((np.ones(n), (r, np.arange(n))), shape=(n, n))


def linear_blocks(mesh, phi_B):
    """Blocks of q -> M^-1 L_DG(q) between an element and itself or a face
    neighbour: blocks[(dy, dx)] maps the local vector of element s to the
    contribution at element s + (dy, dx), local order [c][j][i].

    The operator is linear and couples an element only to itself and its
    four face neighbours, with the same blocks for every element of the
    uniform grid; each block is read off by applying the residual to unit
    vectors at the centre of a 3x3 periodic grid of the same element size.
    """
    K = mesh.K
    nloc = 3 * K * K
    probe = Mesh(3, 3, 3 * mesh.hx, 3 * mesh.hy, mesh.k)
    offsets = [(0, 0), (0, 1), (0, -1), (1, 0), (-1, 0)]
    blocks = {o: np.zeros((nloc, nloc)) for o in offsets}
    for d in range(nloc):
        e = np.zeros((3, 3, 3, K, K))           # [ey][ex][c][j][i]
        e[1, 1].reshape(-1)[d] = 1.0
        out = linear_dglf_residual(probe, e.transpose(2, 0, 1, 3, 4), phi_B)
        out = out.transpose(1, 2, 0, 3, 4)
        for (dy, dx) in offsets:
            blocks[(dy, dx)][:, d] = out[1 + dy, 1 + dx].ravel()
    return blocks


def assemble_linear(mesh, phi_B):
    """Sparse matrix of q -> M^-1 L_DG(q) in element-major ordering:
    sum over neighbour offsets o of kron(P_o, B_o), P_o the periodic shift."""
    L = None
    for (dy, dx), blk in linear_blocks(mesh, phi_B).items():
        P = sp.kron(_shift(mesh.ny, dy), _shift(mesh.nx, dx), format='csr')
        term = sp.kron(P, sp.csr_matrix(blk), format='csr')
        L = term if L is None else L + term
    L.eliminate_zeros()
    return L.tocsr()


class CirculantSolver:
    """Direct solve of (I - c M^-1 L_DG) Q = R on the uniform periodic grid.

    The matrix is block circulant over the element grid, so the 2-D DFT over
    (ey, ex) turns it into one dense (3K^2)-square system per wavenumber:
    S(kappa) = sum_o B_o exp(-2 pi i (kappa_y dy / ny + kappa_x dx / nx)).
    Each system is inverted once and reused, the analogue of factoring once.
    """

    def __init__(self, mesh, phi_B, c):
        self.mesh = mesh
        ny, nx, K = mesh.ny, mesh.nx, mesh.K
        nloc = 3 * K * K
        ky = np.fft.fftfreq(ny) * ny
        kx = np.fft.fftfreq(nx) * nx
        S = np.zeros((ny, nx, nloc, nloc), dtype=np.complex128)
        for (dy, dx), blk in linear_blocks(mesh, phi_B).items():
            ph = np.exp(-2j * np.pi * (ky[:, None] * dy / ny + kx[None, :] * dx / nx))
            S += ph[:, :, None, None] * blk[None, None]
        A = np.eye(nloc)[None, None] - c * S
        self.Ainv = np.linalg.inv(A)

    def solve(self, R):
        """R, Q: (3, ny, nx, K, K)."""
        ny, nx, K = self.mesh.ny, self.mesh.nx, self.mesh.K
        r = R.transpose(1, 2, 0, 3, 4).reshape(ny, nx, -1)
        rh = np.fft.fft2(r, axes=(0, 1))
        qh = np.einsum('yxab,yxb->yxa', self.Ainv, rh)
        q = np.fft.ifft2(qh, axes=(0, 1)).real
        return np.ascontiguousarray(q.reshape(ny, nx, 3, K, K).transpose(2, 0, 1, 3, 4))


# ---------------------------------------------------------- HDG traces
def hdg_trace(mesh, q, phi_B):
    """Single-valued HDG trace qhat on every face node.

    The conservation condition (eq. HDGcont) tested with LGL edge quadrature
    holds at each edge node, so with Fhat_L . n = F_L(q) . n + tau (q - qhat)
    (eq. linear_hdgflux3), tau = sqrt(phi_B):
        qhat = {q} + (F_L(q-) - F_L(q+)) . n- / (2 tau).
    Returns (qhat_x, qhat_y): x-face e is the west face of element e (left
    state from the west neighbour, n = (1, 0)); y-face e is the south face of
    element e (n = (0, 1)).  Shapes (3, ny, nx, K), last index along the face.
    """
    k = mesh.k
    tau = np.sqrt(phi_B)
    west = np.roll(q, 1, axis=2)
    south = np.roll(q, 1, axis=1)

    def trace(qm, qp, nx, ny):
        Fxm, Fym = flux_linear(qm, phi_B)
        Fxp, Fyp = flux_linear(qp, phi_B)
        jump = (Fxm - Fxp) * nx + (Fym - Fyp) * ny
        return 0.5 * (qm + qp) + jump / (2.0 * tau)

    qx = trace(west[..., :, k], q[..., :, 0], 1.0, 0.0)
    qy = trace(south[..., k, :], q[..., 0, :], 0.0, 1.0)
    return qx, qy


# ----------------------------------------------------------- diagnostics
def mass(mesh, q):
    """Discrete integral of each component (LGL quadrature)."""
    m = mesh.mass()
    return np.array([np.sum(m * q[c]) for c in range(3)])


def energy(mesh, q, phi_B):
    """E^h = ||phi_eta||^2 + ||U||^2_{phi_B^-1} (Lemma sdStability)."""
    m = mesh.mass()
    return float(np.sum(m * (q[0] ** 2 + (q[1] ** 2 + q[2] ** 2) / phi_B)))


def rel_l2(mesh, a, b):
    """Per-component ||a_c - b_c||_M / ||b_c||_M with the LGL mass."""
    m = mesh.mass()
    out = []
    for c in range(3):
        num = np.sqrt(np.sum(m * (a[c] - b[c]) ** 2))
        den = np.sqrt(np.sum(m * b[c] ** 2))
        out.append(num / den if den > 0 else num)
    return np.array(out)


def from_user(h, hu, hv, g, H):
    """(h, hu, hv) -> (phi_eta, U, V) = (g (h - H), g hu, g hv) (Sec. 3.1)."""
    return np.stack([g * (h - H), g * hu, g * hv])
