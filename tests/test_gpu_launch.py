"""Graph stepping (IMEXHDG_LAUNCH_GRAPH) against host-driven stepping.

On the fixed launch schedule every convergence decision of the trace solve
is taken on the device; a step is one graph launch.  With a schedule long
enough for the solves the graph path runs the same kernels on the same data
as the host-driven path, so the two agree to round-off of the reductions
that decide when to stop; with a schedule too short the step is redone
host-driven, and the state still agrees."""
import numpy as np
import pytest

from oracle import swe
from paper_1711_02751_amd import imexhdg as m
from gpu_helpers import make_pair, bump_state

pytestmark = pytest.mark.gpu

CASES = [(16, 8, 4, m.PREC_FP64), (10, 7, 3, m.PREC_FP64), (16, 8, 4, m.PREC_MIXED),
         (9, 11, 5, m.PREC_MIXED)]


def _solver(nx, ny, k, prec, launch, dt=0.006):
    kw = dict(precision=prec, launch=launch)
    if prec == m.PREC_MIXED:
        kw.update(krylov_rtol=1e-6, refine_rtol=1e-11, refine_max=8)
    return make_pair(nx, ny, k, 9.81, 1.0, dt, **kw)


def _run(S, q0, calls):
    S.set_state(*q0.reshape(3, -1), vars=m.VARS_GEOPOTENTIAL)
    for n in calls:
        S.step(n)
    return np.stack(S.get_state(vars=m.VARS_GEOPOTENTIAL)).reshape(q0.shape)


@pytest.mark.parametrize("nx,ny,k,prec", CASES)
def test_graph_matches_host_driven(nx, ny, k, prec):
    print(f"graph vs host nx={nx} ny={ny} k={k} prec={prec}", flush=True)
    P, G = _solver(nx, ny, k, prec, m.LAUNCH_GRAPH)
    _, H = _solver(nx, ny, k, prec, m.LAUNCH_HOST)
    q0 = bump_state(P, seed=nx + k, umax=0.2)
    a = _run(G, q0, [20])
    b = _run(H, q0, [20])
    d = G.diag()
    print("diag", d, "schedule", G.schedule(), flush=True)
    assert d["graph_steps"] + d["redo_steps"] >= 18
    assert d["graph_steps"] >= 10
    err = swe.rel_l2(P.mesh, a, b)
    print("graph vs host rel L2", err, flush=True)
    assert np.all(err < 1e-12)
    assert d["max_relres"] <= G.cfg.refine_rtol


def test_graph_replays_equal_one_call():
    """Ten one-step calls (each synchronises) replay the captured graphs with
    host work between them and give the bits of one ten-step call."""
    P, G = _solver(16, 8, 4, m.PREC_FP64, m.LAUNCH_GRAPH)
    q0 = bump_state(P, seed=2, umax=0.2)
    a = _run(G, q0, [1] * 10)
    b = _run(G, q0, [10])
    assert np.array_equal(a, b)


def test_short_schedule_is_redone_and_widened():
    print("short schedule redo", flush=True)
    P, G = _solver(16, 8, 4, m.PREC_FP64, m.LAUNCH_GRAPH)
    _, H = _solver(16, 8, 4, m.PREC_FP64, m.LAUNCH_HOST)
    q0 = bump_state(P, seed=7, umax=0.2)
    G.set_schedule([1])
    assert G.schedule() == (1, [1])
    a = _run(G, q0, [8])
    b = _run(H, q0, [8])
    d = G.diag()
    print("diag", d, "schedule", G.schedule(), flush=True)
    assert d["redo_steps"] >= 1
    sweeps, budget = G.schedule()
    assert sweeps >= 1 and budget[0] > 1
    err = swe.rel_l2(P.mesh, a, b)
    assert np.all(err < 1e-12)


def test_schedule_errors():
    _, G = _solver(8, 8, 3, m.PREC_FP64, m.LAUNCH_GRAPH)
    with pytest.raises(m.ImexError) as e:
        G.set_schedule([0])
    assert e.value.code == m.E_INVAL
    with pytest.raises(m.ImexError) as e:
        G.set_schedule([5] * 9)
    assert e.value.code == m.E_INVAL
    _, H = _solver(8, 8, 3, m.PREC_FP64, m.LAUNCH_HOST)
    with pytest.raises(m.ImexError) as e:
        H.set_schedule([5])
    assert e.value.code == m.E_STATE


# ------------------------------------------------------ launch geometry
@pytest.mark.parametrize("fg,eg", [(8, 8), (16, 4096), (4096, 24)])
def test_launch_geometry_does_not_change_results(fg, eg):
    """Grid caps only change how tiles are dealt to blocks and the order of
    the partial sums; the steps agree with the default geometry."""
    print(f"geometry fg={fg} eg={eg}", flush=True)
    P, A = _solver(32, 16, 4, m.PREC_FP64, m.LAUNCH_GRAPH)
    _, B = _solver(32, 16, 4, m.PREC_FP64, m.LAUNCH_GRAPH)
    B.set_launch_geometry(fg, eg)
    q0 = bump_state(P, seed=11, umax=0.2)
    a = _run(A, q0, [6])
    b = _run(B, q0, [6])
    err = swe.rel_l2(P.mesh, a, b)
    print("rel L2", err, flush=True)
    assert np.all(err < 1e-12)


def test_autotune_restores_state_and_caches(tmp_path):
    print("autotune", flush=True)
    P, S = _solver(64, 64, 4, m.PREC_MIXED, m.LAUNCH_GRAPH, dt=0.004)
    q0 = bump_state(P, seed=12, umax=0.2)
    S.set_state(*q0.reshape(3, -1), vars=m.VARS_GEOPOTENTIAL)
    S.step(3)
    before = np.stack(S.get_state(vars=m.VARS_GEOPOTENTIAL))
    cache = tmp_path / "tune.txt"
    f, e = S.autotune(str(cache))
    print("tuned", f, e, open(cache).read(), flush=True)
    assert 8 <= f <= 4096 and 8 <= e <= 4096
    after = np.stack(S.get_state(vars=m.VARS_GEOPOTENTIAL))
    assert np.array_equal(before, after)
    assert S.diag()["steps"] == 3
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].endswith(f"\t{f}\t{e}")
    # a second context reads the cached choice
    _, S2 = _solver(64, 64, 4, m.PREC_MIXED, m.LAUNCH_GRAPH, dt=0.004)
    S2.set_state(*q0.reshape(3, -1), vars=m.VARS_GEOPOTENTIAL)
    assert S2.autotune(str(cache)) == (f, e)
    assert len(open(cache).read().splitlines()) == 1
    # stepping after tuning matches stepping on the default geometry
    S.step(4)
    _, R = _solver(64, 64, 4, m.PREC_MIXED, m.LAUNCH_GRAPH, dt=0.004)
    R.set_state(*before.reshape(3, -1), vars=m.VARS_GEOPOTENTIAL)
    R.step(4)
    err = swe.rel_l2(P.mesh, np.stack(S.get_state(vars=m.VARS_GEOPOTENTIAL)).reshape(q0.shape),
                     np.stack(R.get_state(vars=m.VARS_GEOPOTENTIAL)).reshape(q0.shape))
    assert np.all(err < 1e-9)


def test_launch_geometry_errors():
    _, S = _solver(8, 8, 3, m.PREC_FP64, m.LAUNCH_GRAPH)
    for fg, eg in [(4, 1024), (1024, 5000), (0, 0)]:
        with pytest.raises(m.ImexError) as e:
            S.set_launch_geometry(fg, eg)
        assert e.value.code == m.E_INVAL
    with pytest.raises(m.ImexError) as e:
        S.autotune()
    assert e.value.code == m.E_STATE


@pytest.mark.parametrize("prec", [m.PREC_FP64, m.PREC_MIXED])
def test_trace_guess_same_state_fewer_iterations(prec):
    """The extrapolated trace guess is a heuristic of the solver: against the
    last stage solution as the guess, the states agree to the solve
    tolerance and the stage solves take fewer inner iterations.  64^2, k = 4,
    the bump recipe at its time step, 12 graph steps."""
    from paper_1711_02751_amd import workloads as W
    wl = W.WORKLOADS["bump_64x64_k4"]
    print(f"trace guess prec={prec}", flush=True)
    out = {}
    for guess in (m.GUESS_LAST, m.GUESS_EXTRAPOLATE):
        cfg = m.default_config(nx=wl.n, ny=wl.n, Lx=wl.L, Ly=wl.L, degree=wl.k, g=wl.g, H=wl.H,
                               dt=wl.dt, precision=prec, launch=m.LAUNCH_GRAPH,
                               trace_guess=guess)
        if prec == m.PREC_MIXED:
            cfg.krylov_rtol, cfg.refine_rtol, cfg.refine_max = 1e-6, 1e-9, 8
        S = m.Solver(cfg)
        x, y = S.nodes()
        S.set_state(*wl.initial_state(x, y))
        S.step(12)
        d = S.diag()
        out[guess] = (np.stack(S.get_state(vars=m.VARS_GEOPOTENTIAL)), d)
        print(f"  guess {guess}: {d['krylov_iters']} inner iterations over "
              f"{d['stage_solves']} solves, schedule {S.schedule()}", flush=True)
        S.close()
    mesh = swe.Mesh(wl.n, wl.n, wl.L, wl.L, wl.k)
    a = out[m.GUESS_LAST][0].reshape(mesh.shape)
    b = out[m.GUESS_EXTRAPOLATE][0].reshape(mesh.shape)
    err = swe.rel_l2(mesh, a, b)
    print("  state difference", err, flush=True)
    assert np.all(err < (1e-11 if prec == m.PREC_FP64 else 1e-7))
    assert (out[m.GUESS_EXTRAPOLATE][1]["krylov_iters"]
            < out[m.GUESS_LAST][1]["krylov_iters"])
