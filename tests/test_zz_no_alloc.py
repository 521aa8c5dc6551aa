"""The allocation-free stage solve (imexhdg_stage_solve_noalloc) against
imexhdg_stage_solve: two calls in a row on two contexts, the second with a
smaller mesh (the scratch array keeps the first call's contents), FP64 and
mixed precision; a mesh beyond the scratch limit is rejected up front."""
import numpy as np
import pytest

from paper_1711_02751_amd import imexhdg as m
from gpu_helpers import make_pair, bump_state, to_dev

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _solve_both(nx, ny, k, seed, **kw):
    P, S = make_pair(nx, ny, k, 9.81, 1.0, 0.006, **kw)
    res0 = to_dev(bump_state(P, seed=seed, umax=0.2), S)
    guess = torch.zeros(S.n_trace, dtype=torch.float64, device=S.device)
    Qa, qha, ita, rra = S.stage_solve(res0, guess)
    Qb = torch.full_like(Qa, float("nan"))
    qhb = guess.clone()
    alloc = torch.cuda.memory_allocated()
    itb, rrb = S.stage_solve_noalloc(res0, Qb, qhb)
    assert torch.cuda.memory_allocated() == alloc
    print(f"noalloc {nx}x{ny} k={k} {kw}: iters {ita} / {itb}, relres {rra:.3e} / {rrb:.3e}",
          flush=True)
    assert ita == itb and rra == rrb
    assert torch.equal(Qa, Qb) and torch.equal(qha, qhb)
    assert rrb <= S.cfg.refine_rtol
    S.close()


@pytest.mark.parametrize("prec", [m.PREC_FP64, m.PREC_MIXED])
def test_noalloc_matches_stage_solve_twice(prec):
    kw = dict(precision=prec)
    if prec == m.PREC_MIXED:
        kw.update(krylov_rtol=1e-6, refine_rtol=1e-11, refine_max=8)
    _solve_both(40, 24, 4, 3, **kw)      # several 16 x 4 tiles, ragged in y
    _solve_both(10, 7, 3, 4, **kw)       # smaller, on the array the first call left


def test_noalloc_rejects_mesh_beyond_scratch():
    cfg = m.default_config(nx=256, ny=256, degree=4, g=9.81, H=1.0, dt=0.002)
    S = m.Solver(cfg)
    res0 = S.volume_empty().zero_()
    Q = S.volume_empty()
    qh = S.trace_zeros()
    with pytest.raises(m.ImexError) as ei:
        S.stage_solve_noalloc(res0, Q, qh)
    assert ei.value.code == m.E_INVAL
    assert "scratch" in str(ei.value)
    S.close()
