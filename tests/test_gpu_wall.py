"""Reflecting walls (IMEXHDG_BOUNDARY_WALL; Sec. 4.3, eqs. reflection and
reflectionBC) through the C ABI, against the oracle (oracle/box.py):

  * whole ARS2 / ARS3 steps on square, non-square, ragged-tile and
    one-element-wide meshes, host-driven and on the captured schedule,
    every node within 1e-11 of the oracle (FP64) and 1e-8 (MIXED);
  * the water-height perturbation of Sec. 6.2 at its full size (20 x 20
    elements, degree 8, H_inf = 100, g = 1, sigma = 0.1) to T = 0.16 with
    both of the paper's ARS2 time steps (0.002 and 0.02), every node against
    the oracle; mass conserved to round-off and the mirror symmetries of the
    centred drop kept.
"""
import numpy as np
import pytest

from oracle import box, imex
from paper_1711_02751_amd import imexhdg as m
from test_oracle_wall import drop_state

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def make_wall(nx, ny, k, dt, L=(2.0, 2.0), g=1.0, H=100.0, scheme=m.SCHEME_ARS232, **kw):
    tab = imex.ars232() if scheme == m.SCHEME_ARS232 else imex.ars443()
    cfg = m.default_config(nx=nx, ny=ny, Lx=L[0], Ly=L[1], degree=k, g=g, H=H, dt=dt,
                           scheme=scheme, physics=m.PHYSICS_NONLINEAR,
                           boundary=m.BOUNDARY_WALL, **kw)
    S = m.Solver(cfg)
    P = box.BoxProblem(nx, ny, L[0], L[1], k, g, H, dt, "wall", tableau=tab)
    return P, S


def state(S, P):
    return np.stack(S.get_state(vars=m.VARS_GEOPOTENTIAL)).reshape(P.mesh.shape)


def rel_max(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("nx,ny,k,L,scheme,launch,steps", [
    (4, 4, 3, (2.0, 2.0), m.SCHEME_ARS232, m.LAUNCH_HOST, 5),
    (6, 5, 2, (1.5, 1.0), m.SCHEME_ARS232, m.LAUNCH_GRAPH, 12),
    (21, 6, 2, (2.0, 0.6), m.SCHEME_ARS443, m.LAUNCH_GRAPH, 6),
    (1, 3, 4, (0.4, 1.2), m.SCHEME_ARS232, m.LAUNCH_HOST, 4),
    (5, 17, 3, (1.0, 2.0), m.SCHEME_ARS443, m.LAUNCH_HOST, 3),
])
def test_wall_steps_match_oracle(nx, ny, k, L, scheme, launch, steps):
    print(f"wall steps {nx}x{ny} k={k} scheme={scheme} launch={launch}", flush=True)
    P, S = make_wall(nx, ny, k, 0.004, L=L, scheme=scheme, launch=launch)
    q0 = drop_state(P.mesh, 1.0, 100.0, sigma=0.15, xc=0.37 * L[0], yc=0.58 * L[1],
                    umax=0.02, seed=nx + ny)
    S.set_state(*q0.reshape(3, -1), vars=m.VARS_GEOPOTENTIAL)
    S.step(steps)
    ref = P.run(q0, steps)
    err = rel_max(state(S, P), ref)
    print("  rel max err", err, flush=True)
    assert err < 1e-11
    assert rel_max(ref, q0) > 1e-4          # the state moved


def test_wall_mixed_precision_matches_oracle():
    P, S = make_wall(8, 8, 3, 0.004, precision=m.PREC_MIXED, krylov_rtol=1e-6,
                     refine_rtol=1e-9, refine_max=8)
    q0 = drop_state(P.mesh, 1.0, 100.0, sigma=0.2, xc=0.8, yc=1.1, umax=0.02, seed=2)
    S.set_state(*q0.reshape(3, -1), vars=m.VARS_GEOPOTENTIAL)
    S.step(10)
    err = rel_max(state(S, P), P.run(q0, 10))
    print("mixed rel max err", err, flush=True)
    assert err < 1e-8


@pytest.mark.parametrize("prec", [m.PREC_FP32, m.PREC_BF16])
def test_wall_reduced_precision_modes_match_oracle(prec):
    """The FP32 / BF16 local solves and FP32 DG residual with walls, on the
    captured schedule: within 1e-6 of the FP64 oracle."""
    P, S = make_wall(8, 8, 3, 0.004, precision=prec, krylov_rtol=1e-6, refine_rtol=1e-9,
                     refine_max=8, launch=m.LAUNCH_GRAPH)
    q0 = drop_state(P.mesh, 1.0, 100.0, sigma=0.2, xc=0.8, yc=1.1, umax=0.02, seed=2)
    S.set_state(*q0.reshape(3, -1), vars=m.VARS_GEOPOTENTIAL)
    S.step(10)
    err = rel_max(state(S, P), P.run(q0, 10))
    print(f"wall precision={prec}: rel max err {err}", flush=True)
    assert err < 1e-6


@pytest.mark.parametrize("dt", [0.002, 0.02])
def test_water_height_perturbation_full_size(dt):
    """Sec. 6.2: 20 x 20 elements of degree 8 on [0, 2]^2, H_inf = 100,
    g = 1, ARS2, T = 0.16 (80 or 8 steps): every node against the oracle,
    mass to round-off, and the drop's mirror symmetries."""
    print(f"water drop dt={dt}", flush=True)
    P, S = make_wall(20, 20, 8, dt)
    q0 = drop_state(P.mesh, 1.0, 100.0, sigma=0.1)
    S.set_state(*q0.reshape(3, -1), vars=m.VARS_GEOPOTENTIAL)
    steps = int(round(0.16 / dt))
    m0 = S.diag()["mass"][0]
    S.step(steps)
    got = state(S, P)
    d = S.diag()
    print("  mass drift", d["mass"][0] - m0, "graph steps", d["graph_steps"], flush=True)
    ref = P.run(q0, steps)
    err = rel_max(got, ref)
    print("  rel max err vs oracle", err, flush=True)
    assert err < 1e-10
    scale = np.sum(P.mesh.mass() * np.abs(q0[0]))          # integral of |phi_eta|
    assert abs(d["mass"][0] - m0) < 1e-12 * scale
    fx = got[:, :, ::-1, :, ::-1].copy()
    fx[1] *= -1.0
    assert rel_max(fx, got) < 1e-11
    assert rel_max(got[0], q0[0]) > 0.1      # the waves have left the centre
