"""Evidence for the time step of the bump workloads (oracle, CPU).

An advective Courant number of 0.5 in the Courant reading used for the
paper's printed values (Cr = dt max(|u| + sqrt(phi)) / dx_min, dx_min the
smallest LGL spacing; here the advective part dt |u| / dx_min) means
dt = 5 dx_min at |u| = 0.1.  The explicit nonlinear part of the IMEX step is
then past its stability limit at k = 4: the oracle blows up within a few
dozen steps.  The workloads take dt = 2 dx_min (advective Courant 0.2,
gravity Courant about 6.5, still far past the explicit gravity-wave limit
that the implicit HDG part removes), which stays bounded.
"""
import numpy as np
import pytest

from oracle import imex, swe
from paper_1711_02751_amd import workloads as W


def _growth(n, k, dt_factor, steps, seed=2):
    """Largest max|q_c(t)| / max|q_c(0)| over components and steps (inf once
    the state is not finite)."""
    xi1 = {4: 1.0 - np.sqrt(3.0 / 7.0), 6: 0.16977610372143304}[k]
    dt = dt_factor * xi1 / 2.0 / n
    P = imex.Problem(n, n, 1.0, 1.0, k, 9.81, 1.0, dt)
    x, y = P.mesh.coords()
    h, hu, hv = W.bump_flow(x, y, seed)
    q = swe.from_user(h, hu, hv, 9.81, 1.0)
    ref = np.abs(q).reshape(3, -1).max(axis=1)
    worst = 1.0
    for s in range(steps):
        q = P.step(q)
        if not np.all(np.isfinite(q)):
            return np.inf, s + 1
        worst = max(worst, float((np.abs(q).reshape(3, -1).max(axis=1) / ref).max()))
        if worst > 1e3:
            return worst, s + 1
    return worst, steps


def test_advective_courant_half_is_unstable_at_k4():
    g, s = _growth(32, 4, 5.0, 40)
    assert g > 100.0, (g, s)


def test_workload_time_step_stays_bounded_at_k4():
    g, s = _growth(32, 4, W.ADVECTIVE_DT_FACTOR, 100)
    assert W.ADVECTIVE_DT_FACTOR == 2.0
    assert g < 2.0, (g, s)
