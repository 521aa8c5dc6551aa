"""IMEX Runge-Kutta stepping of the coupled HDG-DG system (oracle, FP64).

Stage and update formulas follow Sec. 5 (eqs. hdgIMEXRK_qi and
hdgIMEXRK_qn) and the loop of Algorithm 1.  The implicit stage system
(eq. IMEXRKDiscretizedForm) is solved through its plain definition: by the
flux identity of the footnote to eq. linear_hdgflux3 the HDG stage solution
is the solution of (I - dt a~_ii M^-1 L_DG) Q = Res0, a sparse linear system
that is factored once (SDIRK: a~_ii is the same for every implicit stage) and
reused for every stage and step, as the paper does with its LU (Sec. 6.1).
Larger grids may use the exact block-circulant (DFT) solve of the same
matrix instead; the tests pin the two against each other.
"""
import math
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import swe


@dataclass
class Tableau:
    name: str
    A: np.ndarray    # explicit a_ij (strictly lower triangular)
    b: np.ndarray
    At: np.ndarray   # implicit a~_ij (lower triangular)
    bt: np.ndarray

    @property
    def s(self):
        return len(self.b)

    @property
    def c(self):
        return self.A.sum(axis=1)

    @property
    def ct(self):
        return self.At.sum(axis=1)


def ars232():
    """ARS(2,3,2) of Ascher, Ruuth & Spiteri (1997), named in Sec. 5.

    gamma = 1 - 1/sqrt(2), delta = -2 sqrt(2)/3.  Implicit rows (0,0,0),
    (0,gamma,0), (0,1-gamma,gamma); explicit rows (0,0,0), (gamma,0,0),
    (delta,1-delta,0); b = b~ = (0, 1-gamma, gamma)."""
    g = 1.0 - 1.0 / math.sqrt(2.0)
    d = -2.0 * math.sqrt(2.0) / 3.0
    A = np.array([[0.0, 0.0, 0.0], [g, 0.0, 0.0], [d, 1.0 - d, 0.0]])
    At = np.array([[0.0, 0.0, 0.0], [0.0, g, 0.0], [0.0, 1.0 - g, g]])
    b = np.array([0.0, 1.0 - g, g])
    return Tableau("ARS232", A, b, At, b.copy())


def ars443():
    """ARS(4,4,3) of Ascher, Ruuth & Spiteri (1997), named in Sec. 5.

    Implicit rows (0), (0,1/2), (0,1/6,1/2), (0,-1/2,1/2,1/2),
    (0,3/2,-3/2,1/2,1/2); explicit rows (1/2), (11/18,1/18),
    (5/6,-5/6,1/2), (1/4,7/4,3/4,-7/4); both stiffly accurate."""
    At = np.zeros((5, 5))
    At[1, 1] = 0.5
    At[2, 1:3] = [1 / 6, 0.5]
    At[3, 1:4] = [-0.5, 0.5, 0.5]
    At[4, 1:5] = [1.5, -1.5, 0.5, 0.5]
    A = np.zeros((5, 5))
    A[1, 0] = 0.5
    A[2, 0:2] = [11 / 18, 1 / 18]
    A[3, 0:3] = [5 / 6, -5 / 6, 0.5]
    A[4, 0:4] = [0.25, 1.75, 0.75, -1.75]
    b = A[4].copy()
    bt = At[4].copy()
    return Tableau("ARS443", A, b, At, bt)


class Problem:
    """Periodic planar SWE with flat bottom phi_B = g H."""

    def __init__(self, nx, ny, Lx, Ly, k, g, H, dt, tableau=None,
                 nonlinear=True, solver="lu"):
        self.mesh = swe.Mesh(nx, ny, Lx, Ly, k)
        self.g, self.H = float(g), float(H)
        self.phi_B = self.g * self.H
        self.dt = float(dt)
        self.tab = tableau if tableau is not None else ars232()
        self.nonlinear = bool(nonlinear)
        self.Lmat = swe.assemble_linear(self.mesh, self.phi_B)
        diag = np.unique(np.diag(self.tab.At)[np.diag(self.tab.At) != 0])
        if len(diag) != 1:
            raise ValueError("oracle stage solve expects an SDIRK tableau")
        self.a_ii = float(diag[0])
        self.solver = solver
        if solver == "lu":
            n = self.Lmat.shape[0]
            stage = sp.identity(n, format='csc') - self.dt * self.a_ii * self.Lmat.tocsc()
            self.lu = spla.splu(stage.tocsc())
        elif solver == "circulant":
            self.circ = swe.CirculantSolver(self.mesh, self.phi_B, self.dt * self.a_ii)
        else:
            raise ValueError("solver must be 'lu' or 'circulant'")

    # operators on (3, ny, nx, K, K) arrays
    def NL(self, q):
        if not self.nonlinear:
            return np.zeros_like(q)
        return swe.nl_residual(self.mesh, q, self.phi_B)

    def L(self, q):
        return swe.from_vec(self.Lmat @ swe.to_vec(q), self.mesh)

    def stage_solve(self, res0):
        """Q with (I - dt a~_ii M^-1 L) Q = Res0 (eq.
        IMEXRKDiscretizedForm_localSolver with the conservation condition)."""
        if self.solver == "circulant":
            return self.circ.solve(res0)
        return swe.from_vec(self.lu.solve(swe.to_vec(res0)), self.mesh)

    def step(self, qn, record=None):
        """One step of Algorithm 1.  If `record` is a list, the stage
        states Q_i, their traces and NL_i, L_i are appended to it."""
        tab, dt = self.tab, self.dt
        NLs, Ls = [], []
        for i in range(tab.s):
            if tab.At[i, i] == 0.0:
                if i != 0:
                    raise ValueError("explicit-only stage after the first")
                Q = qn
            else:
                res0 = qn.copy()
                for j in range(i):
                    res0 += dt * (tab.A[i, j] * NLs[j] + tab.At[i, j] * Ls[j])
                Q = self.stage_solve(res0)
            Ls.append(self.L(Q))
            NLs.append(self.NL(Q))
            if record is not None:
                qx, qy = swe.hdg_trace(self.mesh, Q, self.phi_B)
                record.append(dict(Q=Q, qhat_x=qx, qhat_y=qy,
                                   NL=NLs[-1], L=Ls[-1]))
        qn1 = qn.copy()
        for i in range(tab.s):
            qn1 += dt * (tab.b[i] * NLs[i] + tab.bt[i] * Ls[i])
        return qn1

    def run(self, q0, nsteps):
        q = q0.copy()
        for _ in range(nsteps):
            q = self.step(q)
        return q
