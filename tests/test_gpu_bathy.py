"""Variable bathymetry (config variable_depth, imexhdg_set_depth; Sec. 3.1
eq. psweGov, Sec. 4.3) through the C ABI, against the oracle
(oracle/bathy.py):

  * whole ARS2 / ARS3 steps over a bottom varying by +-30 %, square and
    ragged-tile meshes, every node within 1e-10 of the oracle (FP64) and
    1e-8 (MIXED); the stage solves' defect corrections are counted and
    bounded;
  * a constant depth given through set_depth reproduces the flat-bottom
    path; mass is conserved; bad depths and flat-bottom contexts are
    rejected.
"""
import numpy as np
import pytest

from oracle import bathy, imex, swe
from paper_1711_02751_amd import imexhdg as m
from test_oracle_bathy import bottom, smooth_state

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def make_bathy(nx, ny, k, dt, amp=0.2, L=(1.0, 1.0), g=9.81, scheme=m.SCHEME_ARS232, **kw):
    tab = imex.ars232() if scheme == m.SCHEME_ARS232 else imex.ars443()
    mesh = swe.Mesh(nx, ny, L[0], L[1], k)
    B = bottom(mesh, amp=amp)
    cfg = m.default_config(nx=nx, ny=ny, Lx=L[0], Ly=L[1], degree=k, g=g, H=1.0, dt=dt,
                           scheme=scheme, physics=m.PHYSICS_NONLINEAR, variable_depth=1, **kw)
    S = m.Solver(cfg)
    S.set_depth(B.ravel())
    P = bathy.BathyProblem(nx, ny, L[0], L[1], k, g, B, dt, tableau=tab)
    return P, S, B


def state(S, P):
    return np.stack(S.get_state(vars=m.VARS_GEOPOTENTIAL)).reshape(P.mesh.shape)


def rel_max(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("nx,ny,k,scheme,amp,steps", [
    (6, 6, 3, m.SCHEME_ARS232, 0.2, 5),
    (20, 6, 2, m.SCHEME_ARS443, 0.3, 4),
    (9, 7, 4, m.SCHEME_ARS232, 0.1, 4),
])
def test_variable_depth_steps_match_oracle(nx, ny, k, scheme, amp, steps):
    print(f"bathy steps {nx}x{ny} k={k} scheme={scheme} amp={amp}", flush=True)
    P, S, _ = make_bathy(nx, ny, k, 0.004, amp=amp, scheme=scheme)
    x, y = P.mesh.coords()
    q0 = smooth_state(x, y, 1.0, 1.0, a=0.2)
    S.set_state(*q0.reshape(3, -1), vars=m.VARS_GEOPOTENTIAL)
    S.step(steps)
    d = S.diag()
    ref = P.run(q0, steps)
    err = rel_max(state(S, P), ref)
    # stage_solves counts every constant-depth solve, the corrections included
    stages = d["stage_solves"] - d["depth_corrections"]
    per_stage = d["depth_corrections"] / max(stages, 1)
    print("  rel max err", err, "corrections per stage", per_stage, flush=True)
    assert err < 1e-10
    assert rel_max(ref, q0) > 1e-3
    assert 1 <= per_stage <= 20


def test_variable_depth_mixed_precision():
    P, S, _ = make_bathy(6, 6, 3, 0.004, precision=m.PREC_MIXED, krylov_rtol=1e-6,
                         refine_rtol=1e-9, refine_max=8)
    x, y = P.mesh.coords()
    q0 = smooth_state(x, y, 1.0, 1.0, a=0.2)
    S.set_state(*q0.reshape(3, -1), vars=m.VARS_GEOPOTENTIAL)
    S.step(5)
    err = rel_max(state(S, P), P.run(q0, 5))
    print("mixed rel max err", err, flush=True)
    assert err < 1e-8


def test_constant_depth_is_the_flat_bottom_path_and_mass_is_kept():
    nx, ny, k, g, dt = 8, 6, 3, 9.81, 0.004
    flat = m.Solver(m.default_config(nx=nx, ny=ny, degree=k, g=g, H=1.0, dt=dt,
                                     launch=m.LAUNCH_HOST))
    var = m.Solver(m.default_config(nx=nx, ny=ny, degree=k, g=g, H=1.0, dt=dt,
                                    variable_depth=1))
    var.set_depth(np.full(var.n_nodes, 1.0))
    mesh = swe.Mesh(nx, ny, 1.0, 1.0, k)
    x, y = mesh.coords()
    q0 = smooth_state(x, y, 1.0, 1.0, a=0.2).reshape(3, -1)
    for S in (flat, var):
        S.set_state(*q0, vars=m.VARS_GEOPOTENTIAL)
        S.step(4)
    a = np.stack(flat.get_state(vars=m.VARS_GEOPOTENTIAL))
    b = np.stack(var.get_state(vars=m.VARS_GEOPOTENTIAL))
    assert rel_max(b, a) < 1e-12
    P, S, _ = make_bathy(nx, ny, k, dt, amp=0.3)
    S.set_state(*q0, vars=m.VARS_GEOPOTENTIAL)
    m0 = S.diag()["mass"][0]
    S.step(6)
    scale = np.sum(mesh.mass() * np.abs(q0[0].reshape(mesh.shape[1:])))
    assert abs(S.diag()["mass"][0] - m0) < 1e-12 * scale


def test_set_depth_rejects():
    P, S, B = make_bathy(6, 6, 2, 0.004)
    bad = B.ravel().copy()
    bad[3] = -0.1
    with pytest.raises(m.ImexError) as e:
        S.set_depth(bad)
    assert e.value.code == m.E_INVAL
    bad[3] = np.nan
    with pytest.raises(m.ImexError):
        S.set_depth(bad)
    flat = m.Solver(m.default_config(nx=4, ny=4, degree=2))
    with pytest.raises(m.ImexError):
        flat.set_depth(np.ones(flat.n_nodes))
