"""Write the stored oracle references used by the full-size GPU parity tests.

    python tests/golden/make_oracle_refs.py [name ...]

Calls only the CPU oracle and the seeded input generators; nothing here
comes from the HIP library.  Outputs (next to this file):
  oracle_<workload>.npz   final state after the workload's step count, in
                          the C ABI host ordering (3, n_nodes), as
                          (phi_eta, U, V); for large meshes a seeded sample
                          of node indices and their values instead of the
                          whole state; plus mass, energy and M-norms.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import imex, swe  # noqa: E402
from paper_1711_02751_amd import workloads as W  # noqa: E402

FULL_STATE_MAX_NODES = 200_000
N_SAMPLES = 8192


def make(name):
    wl = W.WORKLOADS[name]
    P = imex.Problem(wl.n, wl.n, wl.L, wl.L, wl.k, wl.g, wl.H, wl.dt,
                     nonlinear=wl.nonlinear, solver="circulant")
    x, y = P.mesh.coords()
    q = swe.from_user(*wl.initial_state(x, y), wl.g, wl.H)
    t0 = time.time()
    for s in range(wl.steps):
        q = P.step(q)
        if s % 25 == 0:
            print(f"{name}: step {s} ({time.time() - t0:.0f} s)", flush=True)
        if not np.all(np.isfinite(q)):
            raise RuntimeError(f"{name}: non-finite state at step {s}")
    m = P.mesh.mass()
    norms = np.array([np.sqrt(np.sum(m * q[c] ** 2)) for c in range(3)])
    out = dict(name=name, steps=wl.steps, dt=wl.dt, n=wl.n, k=wl.k,
               mass=swe.mass(P.mesh, q), energy=swe.energy(P.mesh, q, P.phi_B),
               mnorm=norms)
    host = q.reshape(3, -1)
    if host.shape[1] <= FULL_STATE_MAX_NODES:
        out["state"] = host
    else:
        rng = np.random.Generator(np.random.PCG64(1234))
        idx = np.sort(rng.choice(host.shape[1], size=N_SAMPLES, replace=False))
        out["sample_idx"] = idx
        out["sample_val"] = host[:, idx]
    path = os.path.join(HERE, f"oracle_{name}.npz")
    np.savez_compressed(path, **out)
    print(f"wrote {path} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or ["bump_64x64_k4", "bump_256x256_k4"]
    for nm in names:
        make(nm)
