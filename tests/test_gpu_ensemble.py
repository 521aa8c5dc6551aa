"""Ensembles: members of different meshes and time steps stepped together,
every launch covering all members.  Each member must evolve exactly as it
would alone (the same kernels run its arithmetic on its own slice, with its
own reductions and convergence flags), so members are compared with single
contexts and, on small meshes, with the oracle."""
import numpy as np
import pytest

from oracle import imex, swe
from paper_1711_02751_amd import imexhdg as m
from paper_1711_02751_amd import workloads as W

pytestmark = pytest.mark.gpu

# (nx, ny): tiled (multiples of 16 x 4) and untiled meshes in one batch
MESHES = [(16, 8), (10, 7), (12, 12), (32, 16), (9, 11)]


def _cfg(nx, ny, k, prec, **kw):
    dt = W.bump_dt(max(nx, ny), k)
    cfg = m.default_config(nx=nx, ny=ny, Lx=1.0, Ly=1.0, degree=k, g=9.81, H=1.0, dt=dt,
                           precision=prec, launch=m.LAUNCH_GRAPH, **kw)
    if prec != m.PREC_FP64:      # MIXED and the FP32 / BF16 modes: FP32 inner solve
        cfg.krylov_rtol = 1e-6
        cfg.refine_rtol = 1e-11
        cfg.refine_max = 8
    return cfg


def _ic(nx, ny, k, seed):
    mesh = swe.Mesh(nx, ny, 1.0, 1.0, k)
    x, y = mesh.coords()
    h, hu, hv = W.bump_flow(x, y, seed, H=1.0, Lx=1.0, Ly=1.0, umax=0.2)
    return mesh, swe.from_user(h, hu, hv, 9.81, 1.0)


def _single(cfg, q0, nsteps):
    S = m.Solver(cfg)
    S.set_state(*q0.reshape(3, -1), vars=m.VARS_GEOPOTENTIAL)
    S.step(nsteps)
    return np.stack(S.get_state(vars=m.VARS_GEOPOTENTIAL)).reshape(q0.shape)


@pytest.mark.parametrize("prec", [m.PREC_FP64, m.PREC_MIXED, m.PREC_FP32, m.PREC_BF16])
def test_members_evolve_as_alone(prec):
    k, nsteps = 3, 12
    print(f"ensemble of {len(MESHES)} prec={prec}", flush=True)
    cfgs = [_cfg(nx, ny, k, prec) for nx, ny in MESHES]
    E = m.Ensemble(cfgs)
    ics = []
    for i, (nx, ny) in enumerate(MESHES):
        mesh, q0 = _ic(nx, ny, k, seed=100 + i)
        ics.append((mesh, q0))
        E.set_state(i, *q0.reshape(3, -1), vars=m.VARS_GEOPOTENTIAL)
    E.step(nsteps)
    d = E.diag(0)
    print("ensemble diag", d, "schedule", E.schedule(), flush=True)
    assert d["graph_steps"] >= nsteps - 3
    tol = 1e-12 if prec == m.PREC_FP64 else 1e-10
    for i, (mesh, q0) in enumerate(ics):
        got = np.stack(E.get_state(i, vars=m.VARS_GEOPOTENTIAL)).reshape(q0.shape)
        ref = _single(cfgs[i], q0, nsteps)
        err = swe.rel_l2(mesh, got, ref)
        print(f"member {i} {MESHES[i]} vs single: {err}", flush=True)
        assert np.all(err < tol)


def test_members_match_oracle():
    k, nsteps = 3, 6
    sel = [(10, 7), (16, 8)]
    cfgs = [_cfg(nx, ny, k, m.PREC_FP64) for nx, ny in sel]
    E = m.Ensemble(cfgs)
    ics = []
    for i, (nx, ny) in enumerate(sel):
        mesh, q0 = _ic(nx, ny, k, seed=200 + i)
        ics.append((mesh, q0))
        E.set_state(i, *q0.reshape(3, -1), vars=m.VARS_GEOPOTENTIAL)
    E.step(nsteps)
    for i, (nx, ny) in enumerate(sel):
        mesh, q0 = ics[i]
        P = imex.Problem(nx, ny, 1.0, 1.0, k, 9.81, 1.0, cfgs[i].dt, nonlinear=True)
        ref = q0
        for _ in range(nsteps):
            ref = P.step(ref)
        got = np.stack(E.get_state(i, vars=m.VARS_GEOPOTENTIAL)).reshape(q0.shape)
        err = swe.rel_l2(mesh, got, ref)
        print(f"member {i} vs oracle: {err}", flush=True)
        assert np.all(err < 1e-11)


def test_member_mass_conserved():
    k = 3
    cfgs = [_cfg(nx, ny, k, m.PREC_FP64) for nx, ny in MESHES[:3]]
    E = m.Ensemble(cfgs)
    q0s = []
    for i, (nx, ny) in enumerate(MESHES[:3]):
        _, q0 = _ic(nx, ny, k, seed=300 + i)
        q0s.append(q0)
        E.set_state(i, *q0.reshape(3, -1), vars=m.VARS_GEOPOTENTIAL)
    d0 = [E.diag(i) for i in range(3)]
    E.step(8)
    for i in range(3):
        d1 = E.diag(i)
        scale = np.abs(q0s[i]).reshape(3, -1).sum(axis=1).max()
        for c in range(3):
            assert abs(d1["mass"][c] - d0[i]["mass"][c]) <= 1e-13 * scale + 1e-15


def test_ensemble_errors():
    a = _cfg(8, 8, 3, m.PREC_FP64)
    b = _cfg(8, 8, 4, m.PREC_FP64)
    with pytest.raises(m.ImexError) as e:
        m.Ensemble([a, b])
    assert e.value.code == m.E_INVAL
    h = _cfg(8, 8, 3, m.PREC_FP64)
    h.launch = m.LAUNCH_HOST
    with pytest.raises(m.ImexError) as e:
        m.Ensemble([h, h])
    assert e.value.code == m.E_INVAL
    E = m.Ensemble([a, _cfg(12, 6, 3, m.PREC_FP64)])
    _, q0 = _ic(8, 8, 3, seed=1)
    E.set_state(0, *q0.reshape(3, -1), vars=m.VARS_GEOPOTENTIAL)
    with pytest.raises(m.ImexError) as e:
        E.step(1)
    assert e.value.code == m.E_STATE
    buf = np.empty(E.n_nodes[0])
    assert E.lib.imexhdg_ens_get_state(E._ens, 2, m.VARS_DEPTH, m._ptr(buf), m._ptr(buf),
                                       m._ptr(buf)) == m.E_INVAL


def test_ensemble_64_members_sampled():
    """64 members on meshes of 32^2 ... 128^2 elements, k = 3, dt_m = 2
    dx_min(m): three steps; three members checked against single contexts."""
    members = W.ensemble_members()
    print("64-member ensemble, elements:", sum(w.n * w.n for w in members), flush=True)
    cfgs = [m.default_config(nx=w.n, ny=w.n, Lx=w.L, Ly=w.L, degree=w.k, g=w.g, H=w.H,
                             dt=w.dt, launch=m.LAUNCH_GRAPH) for w in members]
    E = m.Ensemble(cfgs)
    q0s = []
    for i, w in enumerate(members):
        x, y = E.nodes(i)
        h, hu, hv = w.initial_state(x, y)
        q0s.append((h, hu, hv))
        E.set_state(i, h, hu, hv)
    E.step(3)
    print("schedule", E.schedule(), E.diag(0), flush=True)
    for i in (0, 17, 63):
        w = members[i]
        S = m.Solver(cfgs[i])
        S.set_state(*q0s[i])
        S.step(3)
        mesh = swe.Mesh(w.n, w.n, w.L, w.L, w.k)
        a = np.stack(E.get_state(i, vars=m.VARS_GEOPOTENTIAL)).reshape(mesh.shape)
        b = np.stack(S.get_state(vars=m.VARS_GEOPOTENTIAL)).reshape(mesh.shape)
        err = swe.rel_l2(mesh, a, b)
        print(f"member {i} n={w.n}: {err}", flush=True)
        assert np.all(err < 1e-12)


def test_ensemble_64_members_mixed_vs_oracle():
    """The 64-member configuration on the mixed path (FP32 inner solves,
    krylov_rtol 1e-6, FP64 refinement to 1e-9) as the benchmark runs it:
    20 steps, then the smallest, a middle and the largest member against
    the FP64 oracle (block-circulant direct stage solve) within 1e-6."""
    members = W.ensemble_members()
    cfgs = [m.default_config(nx=w.n, ny=w.n, Lx=w.L, Ly=w.L, degree=w.k, g=w.g, H=w.H,
                             dt=w.dt, launch=m.LAUNCH_GRAPH, precision=m.PREC_MIXED,
                             krylov_rtol=1e-6, refine_rtol=1e-9, refine_max=8)
            for w in members]
    E = m.Ensemble(cfgs)
    q0s = []
    for i, w in enumerate(members):
        x, y = E.nodes(i)
        h, hu, hv = w.initial_state(x, y)
        q0s.append(swe.from_user(h, hu, hv, w.g, w.H))
        E.set_state(i, h, hu, hv)
    steps = 20
    E.step(steps)
    print("mixed 64-member schedule", E.schedule(), flush=True)
    sizes = [w.n for w in members]
    picks = [int(np.argmin(sizes)), int(np.argsort(sizes)[len(sizes) // 2]), int(np.argmax(sizes))]
    for i in picks:
        w = members[i]
        P = imex.Problem(w.n, w.n, w.L, w.L, w.k, w.g, w.H, w.dt, solver="circulant")
        ref = P.run(q0s[i].reshape(P.mesh.shape), steps)
        got = np.stack(E.get_state(i, vars=m.VARS_GEOPOTENTIAL)).reshape(P.mesh.shape)
        err = swe.rel_l2(P.mesh, got, ref)
        print(f"member {i} n={w.n}: rel L2 vs oracle after {steps} steps {err}", flush=True)
        assert np.all(err < 1e-6)


def test_ensemble_autotune_restores_state(tmp_path):
    k = 3
    cfgs = [_cfg(nx, ny, k, m.PREC_MIXED) for nx, ny in MESHES]
    E = m.Ensemble(cfgs)
    for i, (nx, ny) in enumerate(MESHES):
        _, q0 = _ic(nx, ny, k, seed=400 + i)
        E.set_state(i, *q0.reshape(3, -1), vars=m.VARS_GEOPOTENTIAL)
    E.step(3)
    before = [np.stack(E.get_state(i, vars=m.VARS_GEOPOTENTIAL)) for i in range(len(MESHES))]
    cache = tmp_path / "ens_tune.txt"
    f, tpb = E.autotune(str(cache))
    print("ensemble face blocks", f, tpb, open(cache).read(), flush=True)
    assert (tpb == 0 and f in (16, 32, 48, 64, 96, 128, 1024)) or (f == 4096 and tpb in (2, 3, 4, 6, 8))
    for i in range(len(MESHES)):
        assert np.array_equal(before[i], np.stack(E.get_state(i, vars=m.VARS_GEOPOTENTIAL)))
    assert E.diag(0)["steps"] == 3
    assert E.autotune(str(cache)) == (f, tpb)
    assert len(open(cache).read().splitlines()) == 1
    E.step(2)
    assert E.diag(0)["steps"] == 5
