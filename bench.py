#!/usr/bin/env python3
"""Throughput of the IMEX HDG-DG step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one ARS(2,3,2) IMEX step of Algorithm 1 over the whole mesh: three
nonlinear DG residuals, two HDG stage solves (condensation, block-Jacobi
BiCGStab with FP64 refinement on the trace system, local recovery) and the
stage combinations.  The state is resident in HBM before the timed region.
Prints one JSON line; progress goes to stderr.

The timed region steps on the fixed launch schedule (one graph launch per
step).  The roofline object covers the kernel class with the largest device
time in a short all-classes profiling pass; its launches are then timed with
HIP events on the library's stream over the same steps run host-driven.  The CPU baseline is
the FP64 oracle on a bounded sample of the same workload recipe.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DOF-updates/s per IMEX step, mixed vs FP64 at fixed L2 err; HBM GB/s, MFMA %"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6          # FP64 vector and matrix-core peak
FP32_MFMA_PEAK_TFLOPS = 157.3    # dense FP32 matrix-core peak
MIXED_KRYLOV_RTOL = 1e-6
MIXED_REFINE_RTOL = 1e-9     # 500 steps at 256^2: 1.9e-8 from the FP64 path (bound 1e-6)
WORKING_LAUNCH_US = 10.0     # shorter launches of the timed class returned at entry


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_cost(name, wl, n_dof, isz=8):
    """(bytes, flops) one launch of a kernel class must move / compute:
    every input read once and every output written once.  FP64 state and
    trace right-hand sides; `isz` bytes per value of the inner-solve vectors
    (8 FP64, 4 FP32)."""
    K = wl.k + 1
    nel = wl.n * wl.n
    N = n_dof
    T = 6 * K * nel
    nfaces = 2 * nel
    b3 = 3 * K
    table = {
        # first K1 of a solve: read r, p, v, rh; write p, v
        "bicg_k1": (6 * T * isz, 2.0 * 7 * b3 * b3 * nfaces),
        # read r, v, rh; write t (s = r - alpha v is formed, not stored)
        "bicg_k2": (4 * T * isz, 2.0 * 7 * b3 * b3 * nfaces),
        # fused K1: read r, t, p, v, rh, d; write r, p, v, d
        "bicg_k1f": (10 * T * isz, 2.0 * 7 * b3 * b3 * nfaces),
        # read x, g (FP64); write rin (inner); G x over 7 slots, P^-1 g and P^-1 r
        "trace_residual": (2 * T * 8 + T * isz, 2.0 * 9 * b3 * b3 * nfaces),
        "local_apply": (2 * N * 8, 2.0 * (3 * K * K) ** 2 * nel),
        "recover": ((2 * N + T) * 8, 2.0 * (3 * K * K) * 12 * K * nel),
        # read Z at the face nodes, x, x_prev; write g, x, x_prev
        "trace_rhs": (6 * T * 8, 2.0 * b3 * b3 * nfaces),
        "axpy": (2 * T * 8 + T * isz, 2.0 * T),
        # read Q, write NL and the combination, read about 2.5 inputs on average
        "nl_residual": (5.5 * N * 8, 60.0 * N),
    }
    return table.get(name)


def kernel_symbol(kernel_class, K, mixed):
    """Demangled symbol (as a kernel trace names it) of a kernel class's
    host-driven launches."""
    T = "float" if mixed else "double"
    face = {"bicg_k1": "k_bicg_k1", "bicg_k2": "k_bicg_k2", "bicg_k1f": "k_bicg_k1f"}
    # template flags: the fixed schedule (false: host-driven), the bounded
    # mesh variant (false: periodic)
    if kernel_class in face:
        return f"{face[kernel_class]}<{K}, {T}, false, false>"
    if kernel_class == "trace_residual":
        return f"k_trace_residual<{K}, {T}, false>"
    if kernel_class in ("bicg_init", "axpy"):
        return f"k_{kernel_class}<{T}>"
    if kernel_class == "nl_residual":
        return f"k_nl<{K}, double>"
    if kernel_class == "local_apply":
        return f"k_local_apply_lds<{K}>" if K <= 4 else f"k_local_apply<{K}>"
    if kernel_class == "recover":
        return f"k_recover_lds<{K}>" if K <= 6 else f"k_recover<{K}>"
    base = {"trace_rhs": "k_trace_rhs", "diag": "k_diag", "linear_residual": "k_linres"}
    if kernel_class in base:
        return f"{base[kernel_class]}<{K}>"
    return "k_" + kernel_class


def measured_traffic(kernel_class, wl, precision="fp64"):
    """HBM bytes per working dispatch (the launches that did work, as for
    `achieved`) from the committed FETCH_SIZE / WRITE_SIZE profile of this
    workload, or None when the kernel source has changed since the counters
    were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{wl.name}_{precision}.json")
    src = os.path.join(ROOT, "paper_1711_02751_amd", "csrc", "kernels.hip")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    if d.get("kernels_hip_sha256") != sha:
        return None
    rec = d["per_dispatch"].get(kernel_symbol(kernel_class, wl.k + 1, precision == "mixed"))
    if rec is None:
        return None
    return rec.get("working_hbm_bytes", rec["hbm_bytes"])


def lgl_weights(k):
    """Legendre-Gauss-Lobatto quadrature weights of degree k on [-1, 1]:
    w_i = 2 / (k (k + 1) P_k(x_i)^2) at x = -1, 1 and the roots of P_k'."""
    from numpy.polynomial import legendre as leg
    pk = leg.Legendre.basis(k)
    x = np.concatenate([[-1.0], np.sort(pk.deriv().roots().real), [1.0]])
    return 2.0 / (k * (k + 1) * pk(x) ** 2)


def rel_l2_mass(a, b, k):
    """Per-variable ||a - b||_M / ||b||_M with the LGL mass of uniform
    elements (the element area cancels), for states of shape (3, n_nodes)
    in the host ordering (element-major, node j K + i within an element)."""
    w = lgl_weights(k)
    K = k + 1
    wn = np.tile(np.outer(w, w).ravel(), a.shape[1] // (K * K))
    out = []
    for c in range(3):
        num = np.sqrt(np.sum(wn * (a[c] - b[c]) ** 2))
        den = np.sqrt(np.sum(wn * b[c] ** 2))
        out.append(float(num / den) if den > 0 else float(num))
    return out


def cpu_model():
    """CPU model string of the host (Linux /proc/cpuinfo), or the platform's."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def _oracle_rate(wl, n, threads, seconds):
    """Steps of the FP64 oracle on an n x n sample of the workload's recipe
    (same physics, degree, seed and Courant number: dt scaled with the mesh)
    with at most `threads` BLAS / FFT threads, timed after its one-off
    factorisation and one warm step.  Returns (DOF-updates/s, steps,
    wall s, effective cores = process CPU time / wall time)."""
    from threadpoolctl import threadpool_limits
    from oracle import imex, swe
    from paper_1711_02751_amd import workloads as W
    dt = wl.dt * wl.n / n
    with threadpool_limits(limits=threads):
        P = imex.Problem(n, n, wl.L, wl.L, wl.k, wl.g, wl.H, dt, nonlinear=wl.nonlinear,
                         solver="circulant")
        x, y = P.mesh.coords()
        h, hu, hv = W.bump_flow(x, y, wl.seed, H=wl.H, n_bumps=wl.n_bumps, Lx=wl.L, Ly=wl.L)
        q = swe.from_user(h, hu, hv, wl.g, wl.H)
        q = P.step(q)  # first step outside the clock
        steps, t0, c0 = 0, time.perf_counter(), time.process_time()
        while time.perf_counter() - t0 < seconds:
            q = P.step(q)
            steps += 1
        el, cpu = time.perf_counter() - t0, time.process_time() - c0
    ndof = 3 * n * n * (wl.k + 1) ** 2
    return ndof * steps / el, steps, el, cpu / el


def cpu_baseline(wl_name, seconds=15.0):
    """FP64 oracle on a bounded sample: the same recipe (physics, degree,
    dt = 2 dx_min, seed) on a 64 x 64 mesh, with all host cores' worth of
    BLAS / FFT threads and with one thread, each timed for `seconds` / 2
    after its one-off factorisation.  The oracle is plain NumPy / SciPy:
    most of its work runs on one thread whatever the limit, which the
    effective core count (CPU time / wall time) shows."""
    from paper_1711_02751_amd import workloads as W
    wl = W.WORKLOADS[wl_name]
    n = min(wl.n, 64)
    nproc = os.cpu_count() or 1
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    many = _oracle_rate(wl, n, nproc, seconds / 2)
    one = _oracle_rate(wl, n, 1, seconds / 2)
    best, threads = (many, nproc) if many[0] >= one[0] else (one, 1)
    return {"value": best[0], "unit": "DOF-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{n}x{n} mesh, k={wl.k}, same recipe and Courant number, "
                      f"{best[1]} ARS2 steps after one warm step (block-circulant direct "
                      f"stage solve), best of {nproc} threads and 1 thread",
            "seconds": best[2], "effective_cores": best[3],
            "threads_nproc": {"threads": nproc, "value": many[0], "steps": many[1],
                              "effective_cores": many[3]},
            "threads_1": {"threads": 1, "value": one[0], "steps": one[1],
                          "effective_cores": one[3]},
            "cpu_model": cpu_model()}


TUNE_CACHE = os.path.join(ROOT, "paper_1711_02751_amd", "tuning_cache.txt")


PRECISIONS = ("fp64", "mixed", "fp32", "bf16")
MFMA_PEAK_TFLOPS = {"fp64": FP64_PEAK_TFLOPS, "fp32": FP32_MFMA_PEAK_TFLOPS,
                    "bf16": 2500.0}                # dense BF16 matrix-core peak


def local_solve_mfma(per, wl, n_dof, precision, ndc):
    """Matrix-core rate of the element-local solve Z = A^-1 Res0 (kernel
    class local_apply) against the peak of the precision its contraction
    runs in, with the cap its arithmetic intensity puts on that fraction
    (one solve: 2 (3K^2)^2 flop per element over the FP64 state read and
    written, 16 (3K^2) bytes, at 8 TB/s).  Reduced-precision modes run
    1 + ndc contractions (the first solve and ndc defect-correction
    sweeps)."""
    rec = per.get("local_apply")
    if not rec:
        return None
    K = wl.k + 1
    nel = wl.n * wl.n
    nl = 3 * K * K
    gemm = 2.0 * nl * nl * nel
    cp = {"fp64": "fp64", "mixed": "fp64", "fp32": "fp32", "bf16": "bf16"}[precision]
    runs = 1 if cp == "fp64" else 1 + ndc
    t = rec["avg_us"] * 1e-6
    peak = MFMA_PEAK_TFLOPS[cp]
    achieved = runs * gemm / t / 1e12
    ai = gemm / (2 * n_dof * 8)
    return {"contraction": cp, "contractions_per_launch": runs,
            "achieved_tflops": achieved, "peak_tflops": peak, "frac": achieved / peak,
            "roofline_cap_frac": min(1.0, ai * HBM_PEAK_GBS * 1e9 / (peak * 1e12)),
            "avg_launch_us": rec["avg_us"]}


def measure_copy_bandwidth(gib=2, reps=5):
    """Achieved HBM bandwidth of a plain device-to-device copy (torch's copy
    kernel) of `gib` GiB, bytes read plus written per second, best of
    `reps`: the practical ceiling of a streaming kernel beside the nominal
    8 TB/s."""
    import torch
    n = gib * (1 << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        b.synchronize()
        best = min(best, a.elapsed_time(b) / 1000.0)
    del src, dst
    torch.cuda.empty_cache()
    return 2 * n * 8 / best / 1e9


def measure_gemm_peak(n=8192, reps=5):
    """Matrix-core rate a large library GEMM reaches (torch.matmul of two
    contiguous n x n matrices, best of `reps`) in FP64, FP32 and BF16
    (FP32 accumulation): the practical ceiling beside the nominal peaks.
    TFLOP/s per precision."""
    import torch
    out = {}
    prev = torch.backends.cuda.matmul.allow_tf32
    torch.backends.cuda.matmul.allow_tf32 = False
    try:
        for name, dt in (("fp64", torch.float64), ("fp32", torch.float32),
                         ("bf16", torch.bfloat16)):
            a = torch.randn(n, n, device="cuda").to(dt).contiguous()
            b = torch.randn(n, n, device="cuda").to(dt).contiguous()
            c = torch.matmul(a, b)
            best = float("inf")
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                c = torch.matmul(a, b)
                e1.record()
                e1.synchronize()
                best = min(best, e0.elapsed_time(e1) / 1000.0)
            out[name] = 2.0 * n ** 3 / best / 1e12
            del a, b, c
    finally:
        torch.backends.cuda.matmul.allow_tf32 = prev
    torch.cuda.empty_cache()
    return out


def run_path(m, wl, precision, steps, warmup, tune_cache=TUNE_CACHE):
    """Run one precision path; returns (result dict, final state).

    Timed region: `steps` steps on the fixed launch schedule, one graph
    launch per step, after the warm-up (which learns the schedule and
    captures the graphs) and one untimed step from the initial state (a
    cold start runs host-driven).  Roofline: the same steps again, host
    driven, with the dominant kernel class timed by HIP events around each
    of its launches on the library's stream.  The kernels are the same in
    both modes; the graph launches carry their own symbols (a SCHED
    template tag), so a profile tells the two apart."""
    import torch
    mixed = precision != "fp64"     # FP32 inner Krylov solve
    code = {"fp64": m.PREC_FP64, "mixed": m.PREC_MIXED, "fp32": m.PREC_FP32,
            "bf16": m.PREC_BF16}[precision]
    cfg = m.default_config(nx=wl.n, ny=wl.n, Lx=wl.L, Ly=wl.L, degree=wl.k, g=wl.g, H=wl.H,
                           dt=wl.dt, scheme=m.SCHEME_ARS232,
                           physics=m.PHYSICS_NONLINEAR if wl.nonlinear else m.PHYSICS_LINEARIZED,
                           precision=code, launch=m.LAUNCH_GRAPH)
    if mixed:
        cfg.krylov_rtol = MIXED_KRYLOV_RTOL
        cfg.refine_rtol = MIXED_REFINE_RTOL
        cfg.refine_max = 8
    S = m.Solver(cfg)
    x, y = S.nodes()
    h, hu, hv = wl.initial_state(x, y)
    S.set_state(h, hu, hv)
    n_dof = 3 * S.n_nodes
    log(f"[bench] {precision}: {n_dof} DOFs, {S.n_trace} trace unknowns; warmup {warmup}")
    S.step(max(warmup, 3))
    fg, eg = S.autotune(tune_cache)
    log(f"[bench] {precision}: autotuned grid caps: face {fg}, elementwise {eg}")
    S.step(2)
    torch.cuda.synchronize()
    # short all-classes pass (host-driven) to find the dominant kernel
    S.profile(-1)
    S.step(2)
    per = {}
    for name in m.KERNELS:
        n, ms = S.profile_read(name)
        if n:
            per[name] = {"launches": n, "total_ms": ms, "avg_us": 1000.0 * ms / n}
    S.profile(-2)
    dominant = max(per, key=lambda k: per[k]["total_ms"])
    log(f"[bench] {precision}: dominant kernel class {dominant} "
        f"({per[dominant]['avg_us']:.2f} us avg over {per[dominant]['launches']} launches)")
    # timed run: restart from the initial state, one cold step outside the clock
    S.set_state(h, hu, hv)
    S.step(1)
    d0 = S.diag()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    el = t1 - t0
    d1 = S.diag()
    sched = S.schedule()
    state = np.stack(S.get_state(vars=m.VARS_GEOPOTENTIAL))
    value = n_dof * steps / el
    log(f"[bench] {precision}: {steps} graph steps in {el:.3f} s -> {value:.4g} DOF-updates/s "
        f"(schedule {sched}, redone steps {d1['redo_steps'] - d0['redo_steps']})")
    # roofline run: same steps host-driven, each launch of the dominant class
    # timed by start / stop events on its own dispatch
    S.set_state(h, hu, hv)
    S.step(1)
    S.profile(dominant)
    S.step(steps)
    nl_all, ms_all = S.profile_read(dominant)
    # launches that did work: a launch of a converged solve returns at entry
    # (a few us); the working launches of this workload take well over
    # WORKING_LAUNCH_US
    nl, ms = S.profile_read(dominant, min_us=WORKING_LAUNCH_US)
    S.profile(-2)
    isz = 4 if mixed else 8
    avg_s = ms / 1000.0 / nl
    nbytes, nflops = algorithmic_cost(dominant, wl, n_dof, isz)
    matrix = dominant in ("bicg_k1", "bicg_k2", "bicg_k1f", "trace_residual")
    fpeak = (FP32_MFMA_PEAK_TFLOPS if mixed and dominant != "trace_residual"
             else FP64_PEAK_TFLOPS)
    t_hbm = nbytes / (HBM_PEAK_GBS * 1e9)
    t_alu = nflops / (fpeak * 1e12)
    if t_hbm >= t_alu:
        roof = {"bound": "hbm", "achieved": nbytes / avg_s / 1e9, "peak": HBM_PEAK_GBS,
                "unit": "GB/s"}
    else:
        roof = {"bound": "mfma" if matrix else "alu", "achieved": nflops / avg_s / 1e12,
                "peak": fpeak, "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(dominant, wl, precision)
    roof["symbol"] = kernel_symbol(dominant, wl.k + 1, mixed)
    roof["kernel"] = dominant
    roof["avg_launch_us"] = avg_s * 1e6
    roof["launches"] = nl
    roof["avg_launch_us_all"] = 1000.0 * ms_all / nl_all
    roof["launches_all"] = nl_all
    roof["timed_in"] = ("host-driven run of the same steps; HIP start/stop events on each "
                        f"launch's dispatch; launches of at least {WORKING_LAUNCH_US:g} us "
                        "(the rest returned at entry)")
    roof["algorithmic_bytes_per_launch"] = nbytes
    roof["algorithmic_flops_per_launch"] = nflops
    iters = ((d1["krylov_iters"] - d0["krylov_iters"])
             / max(1, d1["stage_solves"] - d0["stage_solves"]))
    ndc = {"fp32": 1, "bf16": 3}.get(precision, 0)
    res = {"value": value, "ms_per_step": 1000.0 * el / steps, "roofline": roof,
           "local_solve_mfma": local_solve_mfma(per, wl, n_dof, precision, ndc),
           "schedule": {"sweeps": sched[0], "inner_budget": sched[1]},
           "grid_caps": {"face": fg, "elementwise": eg},
           "graph_steps": d1["graph_steps"] - d0["graph_steps"],
           "redone_steps": d1["redo_steps"] - d0["redo_steps"],
           "krylov_iters_per_stage": iters, "max_trace_relres": d1["max_relres"],
           "kernels": per, "n_dof": n_dof, "n_trace": S.n_trace}
    S.close()
    return res, state


def run_large(m, wl, steps, warmup, tune_cache=TUNE_CACHE):
    """The large single-mesh workload (1024^2, k = 6): both paths, each
    with its own roofline object, and the mixed-vs-FP64 error of the final
    states."""
    log(f"[bench] large workload {wl.name}: {wl.n}x{wl.n}, k={wl.k}, dt={wl.dt:.6g}")
    f64, s64 = run_path(m, wl, "fp64", steps, warmup, tune_cache)
    mix, smx = run_path(m, wl, "mixed", steps, warmup, tune_cache)
    err = rel_l2_mass(smx, s64, wl.k)
    del s64, smx
    keep = ("value", "ms_per_step", "roofline", "local_solve_mfma", "krylov_iters_per_stage",
            "max_trace_relres",
            "schedule", "grid_caps", "graph_steps", "redone_steps", "kernels")
    return {"workload": wl.name, "mesh": f"{wl.n}x{wl.n}", "degree": wl.k,
            "n_dof": mix["n_dof"], "n_trace": mix["n_trace"], "dt": wl.dt, "steps": steps,
            "unit": "DOF-updates/s",
            "mixed": {k: mix[k] for k in keep}, "fp64": {k: f64[k] for k in keep},
            "speedup_mixed_vs_fp64": mix["value"] / f64["value"],
            "mixed_rel_l2_vs_fp64": [float(e) for e in err],
            "note": f"mixed vs FP64 after the same {steps} + 1 steps from the initial state"}


# Moving vortex of Sec. 6.1 (eq. tc_vortex_ic) on [0, 4]^2 (the paper's
# [-2, 2]^2 translated, centre (2, 2)): H_inf = 1, (u_inf, v_inf) = (1, 0),
# beta = 5, g = 2, exact solution as boundary data, ARS3, dt per degree,
# errors at T = 2.  Printed errors (Tables 1 and 2): L1 and L2 of eta, L2 of
# u and v, sqrt(E).
VORTEX_DT = {2: 0.005, 3: 0.0025, 4: 0.00125, 5: 0.000625}
VORTEX_PAPER = {
    (2, 4): (2.036e-01, 8.189e-02, 1.654e-01, 2.277e-01, 2.072e-01),
    (2, 8): (4.455e-02, 1.693e-02, 4.993e-02, 4.260e-02, 4.793e-02),
    (2, 16): (6.561e-03, 2.793e-03, 1.196e-02, 5.513e-03, 9.517e-03),
    (2, 32): (1.057e-03, 5.412e-04, 2.534e-03, 9.236e-04, 1.945e-03),
    (3, 4): (8.991e-02, 3.645e-02, 1.665e-01, 8.503e-02, 1.347e-01),
    (3, 8): (1.001e-02, 4.226e-03, 9.142e-03, 5.988e-03, 8.285e-03),
    (3, 16): (1.139e-03, 5.864e-04, 9.278e-04, 7.128e-04, 9.254e-04),
    (3, 32): (6.117e-05, 3.228e-05, 5.166e-05, 4.479e-05, 5.347e-05),
    (4, 4): (1.999e-02, 8.123e-03, 1.734e-02, 1.707e-02, 1.814e-02),
    (4, 8): (1.287e-03, 5.723e-04, 1.199e-03, 1.092e-03, 1.216e-03),
    (4, 16): (5.053e-05, 2.705e-05, 5.942e-05, 3.699e-05, 5.306e-05),
    (4, 32): (2.244e-06, 1.467e-06, 3.593e-06, 1.660e-06, 2.985e-06),
    (5, 4): (7.790e-03, 3.015e-03, 1.403e-02, 6.759e-03, 1.121e-02),
    (5, 8): (2.856e-04, 1.408e-04, 2.666e-04, 1.623e-04, 2.421e-04),
    (5, 16): (6.040e-06, 3.378e-06, 5.734e-06, 3.357e-06, 5.270e-06),
    (5, 32): (6.822e-08, 4.193e-08, 6.808e-08, 4.744e-08, 6.574e-08),
}
VORTEX_ERR = ("eta_L1", "eta_L2", "u_L2", "v_L2", "sqrtE")


def vortex_state(x, y, t):
    from paper_1711_02751_amd import workloads as W
    h, hu, hv = W.moving_vortex(x, y, t, xc=2.0, yc=2.0, g=2.0)
    return np.stack([2.0 * (h - 1.0), 2.0 * hu, 2.0 * hv])


def vortex_errors(q, qe, n, k):
    """The error norms of Sec. 6.1 with LGL quadrature: L1, L2 of eta =
    phi_eta / g, L2 of u = U / phi and v, sqrt((||eta||^2 + ||u||^2) / 2)."""
    w = lgl_weights(k)
    K = k + 1
    area = (4.0 / n) ** 2 / 4.0
    wn = np.tile(np.outer(w, w).ravel(), q.shape[1] // (K * K)) * area
    g, phiB = 2.0, 2.0
    de = (q[0] - qe[0]) / g
    du = q[1] / (q[0] + phiB) - qe[1] / (qe[0] + phiB)
    dv = q[2] / (q[0] + phiB) - qe[2] / (qe[0] + phiB)
    l2 = math.sqrt(np.sum(wn * de * de))
    eu, ev = math.sqrt(np.sum(wn * du * du)), math.sqrt(np.sum(wn * dv * dv))
    return (float(np.sum(wn * np.abs(de))), l2, eu, ev,
            math.sqrt(0.5 * (l2 * l2 + eu * eu + ev * ev)))


def run_vortex(m, warm=20):
    """Every mesh and degree of Tables 1 and 2 to T = 2 on one GPU (FP64,
    captured schedule): the errors beside the printed ones, and the step
    rate after `warm` steps (schedule learning and capture)."""
    import torch
    rows = []
    for (p, n) in sorted(VORTEX_PAPER):
        dt = VORTEX_DT[p]
        steps = int(round(2.0 / dt))
        cfg = m.default_config(nx=n, ny=n, Lx=4.0, Ly=4.0, degree=p, g=2.0, H=1.0, dt=dt,
                               scheme=m.SCHEME_ARS443, physics=m.PHYSICS_NONLINEAR,
                               boundary=m.BOUNDARY_VORTEX, vortex=(1.0, 0.0, 5.0, 2.0, 2.0))
        S = m.Solver(cfg)
        x, y = S.nodes()
        S.set_state(*vortex_state(x, y, 0.0), vars=m.VARS_GEOPOTENTIAL)
        S.step(warm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.step(steps - warm)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        q = np.stack(S.get_state(vars=m.VARS_GEOPOTENTIAL))
        e = vortex_errors(q, vortex_state(x, y, steps * dt), n, p)
        d = S.diag()
        ndof = 3 * n * n * (p + 1) ** 2
        rows.append({"p": p, "mesh": f"{n}x{n}", "steps": steps, "dt": dt,
                     "ms_per_step": 1e3 * el / (steps - warm),
                     "dof_updates_per_s": ndof * (steps - warm) / el,
                     "errors": dict(zip(VORTEX_ERR, e)),
                     "paper": dict(zip(VORTEX_ERR, VORTEX_PAPER[(p, n)])),
                     "max_rel_dev_from_paper": max(abs(a - b) / b for a, b in
                                                   zip(e, VORTEX_PAPER[(p, n)])),
                     "krylov_iters_per_stage": d["krylov_iters"] / max(d["stage_solves"], 1),
                     "graph_steps": d["graph_steps"], "redone_steps": d["redo_steps"]})
        log(f"[bench] vortex p={p} {n}x{n}: {rows[-1]['ms_per_step']:.3f} ms/step, "
            f"L2(eta) {e[1]:.4e} (paper {VORTEX_PAPER[(p, n)][1]:.4e})")
        S.close()
        del S
    return {"workload": "moving vortex, Sec. 6.1 (Tables 1-2), ARS3, FP64, exact-solution "
                        "boundary data", "T": 2.0, "cases": rows}


# Water-height perturbation of Sec. 6.2 (Table 3) on [0, 2]^2 (the paper's
# [-1, 1]^2 translated): 20 x 20 elements of degree 8, H_inf = 100, g = 1,
# drop of width sigma = 0.1 (the paper prints none) at rest, reflecting
# walls, ARS2, T = 0.16; the paper's wall-clock time per step (its own
# machine, serial, sparse LU) for context.
WATER_DROP_PAPER_S_PER_STEP = {0.002: (20 * 60 + 41) / 80.0, 0.02: (2 * 60 + 28) / 8.0}


def run_water_drop(m, precision="fp64"):
    """Both ARS2 time steps of Table 3 to T = 0.16 on one GPU, timed over
    the whole run (the first steps learn the schedule and capture it) and
    over the steps after the capture; mass drift of phi_eta."""
    import torch
    from paper_1711_02751_amd import workloads as W
    rows = []
    for dt in (0.002, 0.02):
        steps = int(round(0.16 / dt))
        kw = {}
        if precision == "mixed":
            kw = dict(precision=m.PREC_MIXED, krylov_rtol=MIXED_KRYLOV_RTOL,
                      refine_rtol=MIXED_REFINE_RTOL, refine_max=8)
        cfg = m.default_config(nx=20, ny=20, Lx=2.0, Ly=2.0, degree=8, g=1.0, H=100.0, dt=dt,
                               scheme=m.SCHEME_ARS232, physics=m.PHYSICS_NONLINEAR,
                               boundary=m.BOUNDARY_WALL, **kw)
        S = m.Solver(cfg)
        x, y = S.nodes()
        h, hu, hv = W.water_drop(x, y, H_inf=100.0, sigma=0.1)
        S.set_state(h, hu, hv, vars=m.VARS_DEPTH)
        m0 = S.diag()["mass"][0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.step(2)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        S.step(steps - 2)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        d = S.diag()
        from numpy.polynomial import legendre as leg
        xi = np.concatenate([[-1.0], np.sort(leg.Legendre.basis(8).deriv().roots().real), [1.0]])
        dx_min = 0.1 / 2.0 * np.min(np.diff(xi))
        rows.append({"dt": dt, "steps": steps,
                     "courant": dt * math.sqrt(100.0) / dx_min,   # gravity, sqrt(g H) = 10
                     "s_whole_run": t2 - t0, "ms_per_step_after_capture": 1e3 * (t2 - t1) / (steps - 2),
                     "paper_s_per_step": WATER_DROP_PAPER_S_PER_STEP[dt],
                     "mass_drift": d["mass"][0] - m0,
                     "krylov_iters_per_stage": d["krylov_iters"] / max(d["stage_solves"], 1),
                     "graph_steps": d["graph_steps"], "redone_steps": d["redo_steps"]})
        log(f"[bench] water drop dt={dt} ({precision}): {rows[-1]['ms_per_step_after_capture']:.3f} "
            f"ms/step, whole run {t2 - t0:.3f} s")
        S.close()
        del S
    return {"workload": "water-height perturbation, Sec. 6.2 (Table 3): 20x20, degree 8, "
                        "H_inf = 100, g = 1, sigma = 0.1, walls, ARS2, T = 0.16",
            "precision": precision, "n_dof": 3 * 20 * 20 * 81, "cases": rows,
            "note": "paper_s_per_step: the paper's own machine (serial code, sparse LU), context only"}


def run_bathymetry(m, n=128, k=4, amp=0.2, steps=10, warmup=2):
    """Variable depth B = H (1 + amp sin(2 pi x) cos(2 pi y) + amp / 2 cos(4 pi
    y)) on the periodic n x n mesh of degree k (g = 9.81, H = 1, the bump
    recipe's state and time step), host-driven steps with defect-corrected
    stage solves, beside the flat-bottom path on the same mesh, also
    host-driven; and the same depth and state in a closed basin (reflecting
    walls on the four sides)."""
    import torch
    from paper_1711_02751_amd import workloads as W
    dt = W.bump_dt(n, k)
    out = {"workload": f"variable depth, {n}x{n}, k={k}, bottom +-{amp:.0%} (+-{amp / 2:.0%}), "
                       f"ARS2, dt={dt:.4g}; periodic, and a closed basin (walls)",
           "n_dof": 3 * n * n * (k + 1) ** 2, "steps": steps}
    mixed = dict(precision=m.PREC_MIXED, krylov_rtol=MIXED_KRYLOV_RTOL,
                 refine_rtol=MIXED_REFINE_RTOL, refine_max=8)
    wall = dict(boundary=m.BOUNDARY_WALL)
    for label, vd, kw in (("variable", 1, {}), ("variable_mixed", 1, mixed), ("flat", 0, {}),
                          ("flat_mixed", 0, mixed), ("basin", 1, wall),
                          ("basin_mixed", 1, dict(mixed, **wall))):
        cfg = m.default_config(nx=n, ny=n, degree=k, g=9.81, H=1.0, dt=dt,
                               launch=m.LAUNCH_HOST, variable_depth=vd, **kw)
        S = m.Solver(cfg)
        x, y = S.nodes()
        B = np.ones_like(x)
        if vd:
            B = (1.0 + amp * np.sin(2 * math.pi * x) * np.cos(2 * math.pi * y)
                 + 0.5 * amp * np.cos(4 * math.pi * y))
            S.set_depth(B)
        h, hu, hv = W.bump_flow(x, y, 3, H=1.0, n_bumps=16)
        S.set_state(B + (h - 1.0), hu, hv, vars=m.VARS_DEPTH)   # the same surface elevation
        S.step(warmup)
        d0 = S.diag()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S.step(steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        d = S.diag()
        solves = d["stage_solves"] - d0["stage_solves"]
        corr = d["depth_corrections"] - d0["depth_corrections"]
        stages = solves - corr
        out[label] = {"ms_per_step": 1e3 * el / steps,
                      "dof_updates_per_s": out["n_dof"] * steps / el,
                      "depth_corrections_per_stage": corr / max(stages, 1),
                      "krylov_iters_per_solve": (d["krylov_iters"] - d0["krylov_iters"]) /
                      max(solves, 1)}
        log(f"[bench] bathymetry {label}: {out[label]['ms_per_step']:.3f} ms/step, "
            f"{out[label]['depth_corrections_per_stage']:.1f} corrections per stage")
        S.close()
        del S
    out["cost_vs_flat"] = out["variable"]["ms_per_step"] / out["flat"]["ms_per_step"]
    out["cost_vs_flat_mixed"] = (out["variable_mixed"]["ms_per_step"] /
                                 out["flat_mixed"]["ms_per_step"])
    return out


def run_ensemble(m, steps, warmup, mixed=True, tune_cache=TUNE_CACHE):
    """The 64-member ensemble (meshes 32^2 ... 128^2, k = 3, dt_m = 2 dx_min):
    every launch covers all members, one graph launch per step."""
    import torch
    from paper_1711_02751_amd import workloads as W
    members = W.ensemble_members()
    cfgs = []
    for w in members:
        cfg = m.default_config(nx=w.n, ny=w.n, Lx=w.L, Ly=w.L, degree=w.k, g=w.g, H=w.H,
                               dt=w.dt, physics=m.PHYSICS_NONLINEAR,
                               precision=m.PREC_MIXED if mixed else m.PREC_FP64,
                               launch=m.LAUNCH_GRAPH)
        if mixed:
            cfg.krylov_rtol = MIXED_KRYLOV_RTOL
            cfg.refine_rtol = MIXED_REFINE_RTOL
            cfg.refine_max = 8
        cfgs.append(cfg)
    E = m.Ensemble(cfgs)
    for i, w in enumerate(members):
        x, y = E.nodes(i)
        E.set_state(i, *w.initial_state(x, y))
    n_dof = 3 * sum(E.n_nodes)
    log(f"[bench] ensemble: {len(members)} members, {n_dof} DOFs; warmup {max(warmup, 3)}")
    E.step(max(warmup, 3))
    fg, tpb = E.autotune(tune_cache)
    log(f"[bench] ensemble: autotuned face blocks per member: "
        + (f"{tpb} tiles per block" if tpb else f"cap {fg}"))
    E.step(1)
    d0 = E.diag(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E.step(steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    d1 = E.diag(0)
    value = n_dof * steps / el
    log(f"[bench] ensemble: {steps} graph steps in {el:.3f} s -> {value:.4g} DOF-updates/s "
        f"(schedule {E.schedule()})")
    res = {"workload": "ensemble_64_members_k3", "members": len(members),
           "mesh_sizes": f"{min(w.n for w in members)}^2..{max(w.n for w in members)}^2",
           "n_dof": n_dof, "value": value, "unit": "DOF-updates/s",
           "ms_per_step": 1000.0 * el / steps, "steps": steps,
           "precision": "mixed" if mixed else "fp64",
           "schedule": {"sweeps": E.schedule()[0], "inner_budget": E.schedule()[1]},
           "face_grid_cap_per_member": fg,
           "face_tiles_per_block": tpb,
           "graph_steps": d1["graph_steps"] - d0["graph_steps"],
           "redone_steps": d1["redo_steps"] - d0["redo_steps"]}
    E.close()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="bump_256x256_k4")
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed",
                    help="headline path; the FP64 path is always measured too")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true",
                    help="skip the 64-member ensemble measurement")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="launch-geometry cache: a line for this device and workload is "
                         "used as is, else the autotuner times the candidates and appends one")
    ap.add_argument("--large-workload", default="bump_1024x1024_k6",
                    help="second workload measured beside the headline one (both paths)")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the large-workload measurement")
    ap.add_argument("--vortex-only", action="store_true",
                    help="run only the moving-vortex tables and print their JSON")
    ap.add_argument("--bathymetry-only", action="store_true",
                    help="run only the variable-depth measurement (Sec. 3.1 source term)")
    ap.add_argument("--water-drop-only", action="store_true",
                    help="run only the water-height perturbation (walls, Sec. 6.2)")
    ap.add_argument("--no-vortex", action="store_true",
                    help="skip the bounded-mesh workloads (moving vortex of Sec. 6.1, "
                         "water-height perturbation of Sec. 6.2) and the variable depth")
    ap.add_argument("--no-modes", action="store_true",
                    help="skip the FP32 / BF16 precision modes")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: --gpus {args.gpus} is not supported; the solver runs and is "
              f"measured on a single GPU (the multi-GPU decomposition is design only).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1711_02751_amd import imexhdg as m
    from paper_1711_02751_amd import workloads as W

    wl = W.WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    if args.vortex_only:
        print(json.dumps({"vortex": run_vortex(m)}))
        return
    if args.bathymetry_only:
        print(json.dumps({"bathymetry": run_bathymetry(m)}))
        return
    if args.water_drop_only:
        print(json.dumps({"water_drop": {"fp64": run_water_drop(m),
                                         "mixed": run_water_drop(m, "mixed")}}))
        return
    if args.calib_copy_mib > 0:
        # one plain elementwise pass over a known size: its FETCH_SIZE and
        # WRITE_SIZE counters scale the others to bytes
        n = args.calib_copy_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)     # reads and writes calib_copy_mib MiB once
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.calib_copy_mib} MiB done")
        del src, dst
    hbm_copy = measure_copy_bandwidth()
    log(f"[bench] device copy bandwidth (torch copy of 2 GiB): {hbm_copy:.0f} GB/s")
    gemm_peak = measure_gemm_peak()
    log(f"[bench] library GEMM rates (TFLOP/s): {gemm_peak}")
    log(f"[bench] workload {wl.name}: {wl.n}x{wl.n}, k={wl.k}, dt={wl.dt:.6g}")
    fp64, s64 = run_path(m, wl, "fp64", args.steps, args.warmup, args.tune_cache)
    if args.precision == "fp64":
        head, smx = fp64, None
    else:
        head, smx = run_path(m, wl, "mixed", args.steps, args.warmup, args.tune_cache)
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "DOF-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if smx is None else "f64+f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "mesh": f"{wl.n}x{wl.n}", "degree": wl.k,
                   "n_dof": head["n_dof"], "n_trace": head["n_trace"], "dt": wl.dt,
                   "scheme": "ARS232",
                   "precision": "fp64" if smx is None else
                   f"mixed (FP32 inner Krylov rtol {MIXED_KRYLOV_RTOL:g}, FP64 refinement to "
                   f"{MIXED_REFINE_RTOL:g})",
                   "parallelism": "single GPU"},
        "roofline": head["roofline"],
        "hbm_copy_gbs": hbm_copy,
        "gemm_tflops_measured": gemm_peak,
        "mfma_peak_tflops_nominal": {"fp64": FP64_PEAK_TFLOPS, "fp32": FP32_MFMA_PEAK_TFLOPS,
                                     "bf16": 2500.0},
        "krylov_iters_per_stage": head["krylov_iters_per_stage"],
        "max_trace_relres": head["max_trace_relres"],
        "launch": {k: head[k] for k in ("schedule", "grid_caps", "graph_steps",
                                        "redone_steps")},
        "kernels": head["kernels"],
    }
    if smx is not None:
        err = rel_l2_mass(smx, s64, wl.k)
        out["fp64"] = {"value": fp64["value"], "ms_per_step": fp64["ms_per_step"],
                       "roofline": fp64["roofline"],
                       "launch": {k: fp64[k] for k in ("schedule", "grid_caps",
                                                       "graph_steps", "redone_steps")},
                       "krylov_iters_per_stage": fp64["krylov_iters_per_stage"]}
        out["speedup_mixed_vs_fp64"] = head["value"] / fp64["value"]
        out["mixed_rel_l2_vs_fp64"] = [float(e) for e in err]
    if smx is not None and not args.no_modes:
        # the precision modes with reduced-precision local solves and DG
        # residual, beside MIXED, each with its error against the FP64 path
        out["precision_modes"] = {}
        for prec in ("fp32", "bf16"):
            r, st = run_path(m, wl, prec, args.steps, args.warmup, args.tune_cache)
            e = rel_l2_mass(st, s64, wl.k)
            out["precision_modes"][prec] = {
                "value": r["value"], "ms_per_step": r["ms_per_step"],
                "rel_l2_vs_fp64": [float(x) for x in e],
                "local_solve_mfma": r["local_solve_mfma"],
                "speedup_vs_fp64": r["value"] / fp64["value"]}
        out["precision_modes"]["mixed"] = {
            "value": head["value"], "ms_per_step": head["ms_per_step"],
            "rel_l2_vs_fp64": out["mixed_rel_l2_vs_fp64"],
            "local_solve_mfma": head["local_solve_mfma"],
            "speedup_vs_fp64": head["value"] / fp64["value"]}
        out["precision_modes"]["fp64"] = {"value": fp64["value"],
                                         "ms_per_step": fp64["ms_per_step"],
                                         "local_solve_mfma": fp64["local_solve_mfma"]}
    if not args.no_large and args.large_workload != wl.name:
        out["large"] = run_large(m, W.WORKLOADS[args.large_workload], args.steps, args.warmup,
                                 args.tune_cache)
    if not args.no_vortex:
        out["vortex"] = run_vortex(m)
        out["water_drop"] = {"fp64": run_water_drop(m), "mixed": run_water_drop(m, "mixed")}
        out["bathymetry"] = run_bathymetry(m)
    if not args.no_ensemble:
        out["ensemble"] = run_ensemble(m, args.steps, args.warmup,
                                       mixed=args.precision == "mixed",
                                       tune_cache=args.tune_cache)
    if not args.no_cpu_baseline:
        log(f"[bench] CPU oracle baseline (~{args.cpu_seconds:.0f} s)")
        out["cpu_baseline"] = cpu_baseline(wl.name, args.cpu_seconds)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out))


if __name__ == "__main__":
    main()
