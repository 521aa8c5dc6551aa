"""Shared set-up of GPU parity tests: the same seeded inputs go to the HIP
library (through its C ABI) and to the CPU oracle."""
import numpy as np

from oracle import imex, swe
from paper_1711_02751_amd import imexhdg as m
from paper_1711_02751_amd import workloads as W


def make_pair(nx, ny, k, g, H, dt, Lx=1.0, Ly=1.0, nonlinear=True, solver="lu",
              scheme=m.SCHEME_ARS232, **cfgkw):
    tab = imex.ars232() if scheme == m.SCHEME_ARS232 else imex.ars443()
    P = imex.Problem(nx, ny, Lx, Ly, k, g, H, dt, tableau=tab, nonlinear=nonlinear,
                     solver=solver)
    cfg = m.default_config(nx=nx, ny=ny, Lx=Lx, Ly=Ly, degree=k, g=g, H=H, dt=dt,
                           scheme=scheme,
                           physics=m.PHYSICS_NONLINEAR if nonlinear else m.PHYSICS_LINEARIZED,
                           **cfgkw)
    S = m.Solver(cfg)
    return P, S


def oracle_to_host(q):
    """(3, ny, nx, K, K) -> (3, n_nodes) in the C ABI host ordering."""
    return q.reshape(3, -1)


def host_to_oracle(a, mesh):
    return np.asarray(a).reshape(mesh.shape)


def to_dev(q, S):
    import torch
    v = m.volume_to_device_layout(oracle_to_host(q), S.nel, S.K)
    return torch.from_numpy(v).to(S.device)


def from_dev(t, S, mesh):
    v = m.volume_from_device_layout(t.cpu().numpy(), S.nel, S.K)
    return host_to_oracle(v, mesh)


def traces_from_dev(t, S, mesh):
    """device trace [d][c][j][e] -> oracle (qhat_x, qhat_y), (3, ny, nx, K)."""
    a = t.cpu().numpy().reshape(2, 3, S.K, mesh.ny, mesh.nx)
    return a[0].transpose(0, 2, 3, 1), a[1].transpose(0, 2, 3, 1)


def bump_state(P, seed=5, umax=0.1):
    x, y = P.mesh.coords()
    h, hu, hv = W.bump_flow(x, y, seed, H=P.H, Lx=P.mesh.Lx, Ly=P.mesh.Ly, umax=umax)
    return swe.from_user(h, hu, hv, P.g, P.H)


def rel_err(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)
