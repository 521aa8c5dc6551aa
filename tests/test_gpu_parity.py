"""Parity of the HIP path (through the C ABI) with the CPU oracle."""
import numpy as np
import pytest

from oracle import hdg_dense, imex, swe
from paper_1711_02751_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1711_02751_amd import imexhdg as m  # noqa: E402
from tests.gpu_helpers import (bump_state, from_dev, make_pair, rel_err, to_dev,  # noqa: E402
                               traces_from_dev)

# mesh cases: several 64-element tiles with a ragged tail, degenerate
# periodic neighbours (n = 1, 2), non-square elements, lowest and highest degree
MESHES = [(10, 7, 3, 1.0, 0.8), (16, 16, 4, 1.0, 1.0), (9, 11, 2, 1.3, 1.0),
          (1, 3, 2, 1.0, 1.0), (2, 2, 1, 1.0, 1.0), (5, 4, 8, 1.0, 1.0), (13, 5, 6, 0.7, 1.1)]


@pytest.mark.parametrize("nx,ny,k,Lx,Ly", MESHES)
def test_nl_residual(nx, ny, k, Lx, Ly):
    print(f"nl_residual nx={nx} ny={ny} k={k}", flush=True)
    P, S = make_pair(nx, ny, k, 9.81, 1.0, 0.01, Lx=Lx, Ly=Ly)
    q = bump_state(P, seed=nx * 7 + k, umax=0.3)
    ref = swe.nl_residual(P.mesh, q, P.phi_B)
    got = from_dev(S.nl_residual(to_dev(q, S)), S, P.mesh)
    torch.cuda.synchronize()
    assert rel_err(got, ref) < 1e-12


@pytest.mark.parametrize("nx,ny,k,Lx,Ly", MESHES)
def test_linear_residual_with_traces(nx, ny, k, Lx, Ly):
    """M^-1 L(Q, Qhat) with arbitrary traces against the oracle's HDG form,
    and with the conservative trace against the DG-LF form."""
    print(f"linear_residual nx={nx} ny={ny} k={k}", flush=True)
    P, S = make_pair(nx, ny, k, 2.0, 1.5, 0.01, Lx=Lx, Ly=Ly)
    rng = np.random.default_rng(nx + 10 * ny + 100 * k)
    Q = rng.standard_normal(P.mesh.shape)
    qx = rng.standard_normal((3, ny, nx, k + 1))
    qy = rng.standard_normal((3, ny, nx, k + 1))
    qhat = torch.from_numpy(np.concatenate([qx.transpose(0, 3, 1, 2).ravel(),
                                            qy.transpose(0, 3, 1, 2).ravel()])).to(S.device)
    got = from_dev(S.linear_residual(to_dev(Q, S), qhat), S, P.mesh)
    ref = hdg_dense.hdg_L(P.mesh, Q, qx, qy, P.phi_B)
    assert rel_err(got, ref) < 1e-12
    tx, ty = swe.hdg_trace(P.mesh, Q, P.phi_B)
    qhat = torch.from_numpy(np.concatenate([tx.transpose(0, 3, 1, 2).ravel(),
                                            ty.transpose(0, 3, 1, 2).ravel()])).to(S.device)
    got = from_dev(S.linear_residual(to_dev(Q, S), qhat), S, P.mesh)
    assert rel_err(got, swe.linear_dglf_residual(P.mesh, Q, P.phi_B)) < 1e-12


@pytest.mark.parametrize("nx,ny,k,Lx,Ly", MESHES)
def test_stage_solve(nx, ny, k, Lx, Ly):
    """Static condensation + trace solve + recovery vs the oracle's direct
    DG-LF stage solve and closed-form trace."""
    print(f"stage_solve nx={nx} ny={ny} k={k}", flush=True)
    P, S = make_pair(nx, ny, k, 9.81, 1.0, 0.02, Lx=Lx, Ly=Ly)
    rng = np.random.default_rng(3 * nx + ny + k)
    R = bump_state(P, seed=k) + 0.01 * rng.standard_normal(P.mesh.shape)
    Q, qh, iters, relres = S.stage_solve(to_dev(R, S))
    Qg = from_dev(Q, S, P.mesh)
    Qo = P.stage_solve(R)
    assert relres <= 1e-13
    assert rel_err(Qg, Qo) < 1e-12
    tx, ty = swe.hdg_trace(P.mesh, Qo, P.phi_B)
    gx, gy = traces_from_dev(qh, S, P.mesh)
    assert rel_err(gx, tx) < 1e-11 and rel_err(gy, ty) < 1e-11


def _run_both(P, S, q0, nsteps):
    S.set_state(*q0.reshape(3, -1), vars=m.VARS_GEOPOTENTIAL)
    S.step(nsteps)
    got = np.stack(S.get_state(vars=m.VARS_GEOPOTENTIAL)).reshape(P.mesh.shape)
    ref = P.run(q0, nsteps)
    return got, ref


def test_config1_standing_wave_100_steps():
    """8x8, k=2, linearized, g=H=1, dt=0.01, 100 steps: FP64 parity 1e-11."""
    wl = W.WORKLOADS["standing_wave_8x8_k2"]
    P, S = make_pair(wl.n, wl.n, wl.k, wl.g, wl.H, wl.dt, nonlinear=False)
    x, y = P.mesh.coords()
    q0 = swe.from_user(*wl.initial_state(x, y), wl.g, wl.H)
    got, ref = _run_both(P, S, q0, wl.steps)
    err = swe.rel_l2(P.mesh, got, ref)
    print("config1 rel L2", err, flush=True)
    assert np.all(err < 1e-11)
    qe = swe.from_user(*W.standing_wave(x, y, wl.steps * wl.dt, wl.g, wl.H), wl.g, wl.H)
    assert swe.rel_l2(P.mesh, got, qe)[0] < 0.02


@pytest.mark.parametrize("nx,ny,k,scheme", [(12, 10, 3, m.SCHEME_ARS232),
                                            (7, 9, 4, m.SCHEME_ARS443),
                                            (2, 3, 2, m.SCHEME_ARS232)])
def test_nonlinear_steps(nx, ny, k, scheme):
    print(f"steps nx={nx} ny={ny} k={k} scheme={scheme}", flush=True)
    P, S = make_pair(nx, ny, k, 9.81, 1.0, 0.006, scheme=scheme)
    q0 = bump_state(P, seed=k + nx, umax=0.2)
    got, ref = _run_both(P, S, q0, 20)
    err = swe.rel_l2(P.mesh, got, ref)
    print("rel L2", err, flush=True)
    assert np.all(err < 1e-11)


def test_config2_short_run_live_oracle():
    """64x64, k=4, g=9.81, dt = 2 dx_min (the workload's step): 10 steps against the oracle."""
    wl = W.WORKLOADS["bump_64x64_k4"]
    P, S = make_pair(wl.n, wl.n, wl.k, wl.g, wl.H, wl.dt, solver="circulant")
    x, y = P.mesh.coords()
    q0 = swe.from_user(*wl.initial_state(x, y), wl.g, wl.H)
    got, ref = _run_both(P, S, q0, 10)
    err = swe.rel_l2(P.mesh, got, ref)
    print("config2 10-step rel L2", err, S.diag(), flush=True)
    assert np.all(err < 1e-11)


def test_mass_conservation_and_determinism():
    P, S = make_pair(24, 20, 3, 9.81, 1.0, 0.01)
    q0 = bump_state(P, seed=9, umax=0.2)
    S.set_state(*q0.reshape(3, -1), vars=m.VARS_GEOPOTENTIAL)
    d0 = S.diag()
    S.step(15)
    d1 = S.diag()
    a = np.stack(S.get_state(vars=m.VARS_GEOPOTENTIAL))
    scale = np.abs(q0).reshape(3, -1).sum(axis=1) * P.mesh.mass().ravel()[0] * 10
    for c in range(3):
        assert abs(d1["mass"][c] - d0["mass"][c]) <= 1e-12 * max(scale[c], 1e-30) + 1e-15
    S.set_state(*q0.reshape(3, -1), vars=m.VARS_GEOPOTENTIAL)
    S.step(15)
    b = np.stack(S.get_state(vars=m.VARS_GEOPOTENTIAL))
    assert np.array_equal(a, b)


def test_error_paths():
    P, S = make_pair(4, 4, 2, 1.0, 1.0, 0.01)
    with pytest.raises(m.ImexError) as e:
        S.step(1)
    assert e.value.code == m.E_STATE
    n = S.n_nodes
    with pytest.raises(m.ImexError) as e:
        S.set_state(np.full(n, -0.5), np.zeros(n), np.zeros(n))     # h <= 0
    assert e.value.code == m.E_INVAL
    with pytest.raises(m.ImexError) as e:
        S.set_state(np.full(n, np.nan), np.zeros(n), np.zeros(n))
    assert e.value.code == m.E_INVAL
    # a one-iteration budget cannot reach the tolerance
    P2, S2 = make_pair(8, 8, 3, 9.81, 1.0, 0.02, krylov_max_iter=1, check_every=1, refine_max=1)
    q0 = bump_state(P2, seed=1)
    S2.set_state(*q0.reshape(3, -1), vars=m.VARS_GEOPOTENTIAL)
    with pytest.raises(m.ImexError) as e:
        S2.step(1)
    assert e.value.code == m.E_NOCONV


# ------------------------------------------------------ mixed precision
@pytest.mark.parametrize("nx,ny,k", [(16, 16, 4), (10, 7, 3), (16, 8, 6)])
def test_mixed_stage_solve(nx, ny, k):
    """FP32 inner BiCGStab with FP64 refinement reaches the FP64 tolerance."""
    print(f"mixed stage_solve nx={nx} ny={ny} k={k}", flush=True)
    P, S = make_pair(nx, ny, k, 9.81, 1.0, 0.02, precision=m.PREC_MIXED,
                     krylov_rtol=1e-6, refine_rtol=1e-12, refine_max=8)
    R = bump_state(P, seed=k)
    Q, qh, iters, relres = S.stage_solve(to_dev(R, S))
    assert relres <= 1e-12
    assert rel_err(from_dev(Q, S, P.mesh), P.stage_solve(R)) < 1e-10


def test_mixed_steps_bound():
    """Mixed path (refine_rtol 1e-10) stays within 1e-8 of the FP64 oracle
    after 20 nonlinear steps."""
    P, S = make_pair(16, 16, 4, 9.81, 1.0, 0.004, precision=m.PREC_MIXED,
                     krylov_rtol=1e-6, refine_rtol=1e-10, refine_max=8)
    q0 = bump_state(P, seed=3, umax=0.1)
    got, ref = _run_both(P, S, q0, 20)
    err = swe.rel_l2(P.mesh, got, ref)
    print("mixed rel L2 after 20 steps", err, S.diag(), flush=True)
    assert np.all(err < 1e-8)
