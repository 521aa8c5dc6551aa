/*
 * imexhdg.h - C ABI of the MI355X (gfx950) IMEX HDG-DG shallow-water step.
 *
 * The library advances the planar shallow-water equations in geopotential
 * form (Kang, Giraldo & Bui-Thanh, arXiv:1711.02751, Sec. 3.1) on a periodic
 * nx-by-ny grid of affine rectangles with degree-k nodal DG/HDG spaces
 * (Sec. 4), one IMEX Runge-Kutta step at a time (Sec. 5, Algorithm 1):
 *   - explicit DG residual of the nonlinear part with the Rusanov flux
 *     (Sec. 4.3, eqs. Full_russanov / Linear_russanov);
 *   - implicit HDG solve of the linear gravity-wave part: element-local
 *     static condensation, the global trace system
 *     (eq. linearizedHDGsystem_schur) and local recovery
 *     (eq. recover_volume_unknowns);
 *   - the stage combination (eqs. hdgIMEXRK_qi / hdgIMEXRK_qn).
 *
 * Discretisation choices (the paper leaves them open): LGL nodes with
 * collocated LGL quadrature on elements and edges, trace nodes = LGL edge
 * nodes; a flat bottom phi_B = g H, or a depth given at the nodes
 * (config.variable_depth, imexhdg_set_depth).  Boundaries: periodic, or a
 * bounded rectangle whose boundary faces take the state of an imaginary
 * neighbour in the numerical fluxes and the conservation condition (the
 * principle of Sec. 4.3's wall condition), set from the exact translating
 * vortex of Sec. 6.1 (eq. tc_vortex_ic), as in the paper's vortex test, or
 * by reflecting walls (Sec. 4.3, eq. reflection).
 *
 * Conventions
 *   - Every call returns an int status: IMEXHDG_OK (0) or a negative code.
 *     No exception or abort crosses the ABI.  imexhdg_last_error() returns a
 *     thread-local message for the last failing call on the calling thread.
 *   - Host arrays are caller owned and only read/written during the call.
 *   - Node ordering of host state arrays is row-major over elements and,
 *     inside an element, over LGL nodes: index ((ey*nx + ex)*K + j)*K + i,
 *     K = k + 1, i along x and j along y.  n_nodes = nx*ny*K*K.
 *   - Device arrays in "device layout" (operator-level calls) are
 *     structure-of-arrays with the element index fastest:
 *       volume  v[c][j*K + i][e]        c in (phi_eta, U, V), e = ey*nx + ex
 *       trace   t[d][c][j][e]           d = 0: x-face e (west face of e),
 *                                        d = 1: y-face e (south face of e),
 *                                        j = LGL node index along the face.
 *   - A context is bound to one HIP stream; calls on one context must not
 *     overlap.  Distinct contexts are independent.
 */
#ifndef IMEXHDG_H
#define IMEXHDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define IMEXHDG_OK            0
#define IMEXHDG_E_INVAL      -1  /* bad argument or configuration          */
#define IMEXHDG_E_NOMEM      -2  /* device or host allocation failed        */
#define IMEXHDG_E_DEVICE     -3  /* HIP runtime error                      */
#define IMEXHDG_E_NOCONV     -4  /* trace solve missed its tolerance        */
#define IMEXHDG_E_NONFINITE  -5  /* state became NaN or Inf                 */
#define IMEXHDG_E_STATE      -6  /* call out of order (e.g. step before set) */

/* IMEX tableaux named in Sec. 5 (Ascher, Ruuth & Spiteri 1997) */
#define IMEXHDG_SCHEME_ARS232 0
#define IMEXHDG_SCHEME_ARS443 1

/* physics: linearized = only the linear (stiff) part, NL(q) = 0 */
#define IMEXHDG_PHYSICS_LINEARIZED 0
#define IMEXHDG_PHYSICS_NONLINEAR  1

/* precision of the step */
#define IMEXHDG_PREC_FP64   0  /* everything in FP64                        */
#define IMEXHDG_PREC_MIXED  1  /* FP32 inner Krylov solve of the trace
                                  system (FP32 matrix cores); FP64 state,
                                  DG residuals, local solves, trace
                                  residual, iterative refinement, mass and
                                  energy sums                               */
#define IMEXHDG_PREC_FP32   2  /* as MIXED, and the element-local solves of
                                  the condensation and the recovery (eqs.
                                  linearizedHDGsystem_schur,
                                  recover_volume_unknowns) on the FP32
                                  matrix cores with FP64 defect correction
                                  (local_sweeps), and the DG residual of the
                                  nonlinear part (Sec. 4.3) computed in
                                  FP32 from the FP64 state                  */
#define IMEXHDG_PREC_BF16   3  /* as FP32, with the local solves' dense
                                  contraction on the BF16 matrix cores (FP32
                                  accumulation)                             */

/* how imexhdg_step drives the trace solves */
#define IMEXHDG_LAUNCH_GRAPH 0  /* fixed launch schedule, one captured graph per
                                   step, convergence decided on the device;
                                   a step whose stage solves miss refine_rtol
                                   on the schedule is redone host-driven     */
#define IMEXHDG_LAUNCH_HOST  1  /* host reads the residual between sweeps and
                                   the Krylov state every few iterations     */

/* initial trace guess of a step's stage solves (a heuristic of the solver:
 * it changes the iteration count, not the converged trace)               */
#define IMEXHDG_GUESS_EXTRAPOLATE 0  /* straight line in time through the last
                                        two stage solutions (where the stage
                                        times increase), else the last one   */
#define IMEXHDG_GUESS_LAST        1  /* the last stage solution             */

/* variables of host state arrays */
#define IMEXHDG_VARS_DEPTH       0  /* (h, hu, hv): depth and momenta        */
#define IMEXHDG_VARS_GEOPOTENTIAL 1 /* (phi_eta, U, V) = (g(h-H), g hu, g hv) */

/* boundary of the domain [0,Lx] x [0,Ly] (config.boundary)
 *   PERIODIC  every face has two elements.
 *   VORTEX    bounded rectangle; a boundary face takes as its exterior state
 *             the exact translating vortex of Sec. 6.1 (eq. tc_vortex_ic)
 *             at the stage time, with H_inf = H, g = g and
 *             (u_inf, v_inf, beta, xc, yc) = vortex[0..4] (centre at t = 0
 *             in the domain's coordinates), in the explicit Rusanov flux and
 *             in the conservation condition of the boundary face (an
 *             imaginary neighbour, as Sec. 4.3 does for the wall; eqs.
 *             reflection, reflectionBC).  Time is counted from the last
 *             set_state (t = 0 there), t = steps dt.  Device arrays of the
 *             operator-level calls and imexhdg_state_device use a mesh
 *             padded by two ghost columns and rows ((nx + 2) x (ny + 2)
 *             elements; the ghosts hold boundary states, faces between
 *             ghosts hold zero); those calls, ensembles and the
 *             allocation-free stage solve take periodic meshes only.
 *   WALL      bounded rectangle with reflecting walls on all four sides
 *             (Sec. 4.3): the imaginary neighbour of a boundary face holds
 *             the element's own state with the normal momentum reversed
 *             (eq. reflection), in the explicit flux and in the
 *             conservation condition, which yields eq. reflectionBC for
 *             the trace.  Padded layout and restrictions as for VORTEX.  */
#define IMEXHDG_BOUNDARY_PERIODIC 0
#define IMEXHDG_BOUNDARY_VORTEX   1
#define IMEXHDG_BOUNDARY_WALL     2

/* element type of device state arrays (imexhdg_set_state_device)          */
#define IMEXHDG_DTYPE_F64 0
#define IMEXHDG_DTYPE_F32 1

typedef struct imexhdg_config {
    int32_t nx, ny;          /* elements per direction, >= 1               */
    double  Lx, Ly;          /* domain [0,Lx) x [0,Ly), > 0                */
    int32_t degree;          /* polynomial degree k, 1 <= k <= 8           */
    double  g, H;            /* gravity and mean depth: phi_B = g H > 0    */
    double  dt;              /* time step, > 0                             */
    int32_t scheme;          /* IMEXHDG_SCHEME_*                           */
    int32_t physics;         /* IMEXHDG_PHYSICS_*                          */
    int32_t precision;       /* IMEXHDG_PREC_*                             */
    double  krylov_rtol;     /* inner Krylov tolerance (preconditioned);
                                at least 1e-6 with IMEXHDG_PREC_MIXED      */
    int32_t krylov_max_iter; /* inner iteration budget per solve           */
    int32_t check_every;     /* iterations between convergence checks      */
    double  refine_rtol;     /* FP64 true-residual tolerance ||g-Gx||/||g|| */
    int32_t refine_max;      /* max refinement sweeps per stage solve      */
    int32_t launch;          /* IMEXHDG_LAUNCH_*                           */
    int32_t trace_guess;     /* IMEXHDG_GUESS_*                            */
    int32_t local_sweeps;    /* defect-correction sweeps of a reduced-
                                precision local solve (IMEXHDG_PREC_FP32 /
                                _BF16): Q <- Q + A_lp^-1 (R - A Q) with the
                                residual in FP64; 1 or 2 (3 with BF16),
                                0 = the default (1 for FP32, 3 for BF16);
                                ignored by the other precisions           */
    int32_t boundary;        /* IMEXHDG_BOUNDARY_*                         */
    int32_t variable_depth;  /* 1: the depth B under the reference plane
                                varies in space, phi_B = g B at the nodes
                                (imexhdg_set_depth; H until it is called):
                                the flux tensor and linear flux take the
                                nodal phi_B and L gains the source
                                (0, phi_eta grad phi_B) (Sec. 3.1, eq.
                                psweGov; Sec. 4.3).  The stage system is
                                solved by defect correction: its FP64
                                residual, matrix-free with the nodal phi_B,
                                corrected by the constant-depth (phi_B =
                                g H) HDG stage solve until its relative
                                norm is at most refine_rtol.  Periodic or
                                walled (IMEXHDG_BOUNDARY_WALL: a closed
                                basin, the depth mirrored across each
                                wall), single contexts; steps run
                                host-driven.                              */
    double  vortex[5];       /* u_inf, v_inf, beta, xc, yc of
                                IMEXHDG_BOUNDARY_VORTEX (finite)           */
} imexhdg_config;

typedef struct imexhdg_diag {
    double  mass[3];         /* FP64 sum of M q_c, c = phi_eta, U, V       */
    double  energy;          /* E^h = ||phi_eta||^2 + ||U||^2_{1/phi_B}    */
    int64_t steps;           /* steps taken since set_state                */
    int64_t krylov_iters;    /* inner iterations, cumulative               */
    int64_t stage_solves;    /* implicit stage solves, cumulative          */
    int64_t refine_sweeps;   /* FP64 refinement sweeps, cumulative         */
    double  last_relres;     /* last FP64 true relative trace residual     */
    double  max_relres;      /* largest final relative residual so far     */
    int32_t nonfinite;       /* 1 if the state holds NaN/Inf               */
    int64_t graph_steps;     /* steps run as one graph launch, cumulative  */
    int64_t redo_steps;      /* graph steps redone host-driven, cumulative */
    double  step_ms;         /* host wall time inside imexhdg_step since the
                                last set_state, stream synchronised (ms)   */
    /* Device time per phase of the step (ms), summed over the launches the
     * kernel event profiler timed since the last imexhdg_profile() call
     * (all zero while it is off; with imexhdg_profile(ctx, -1) every class
     * is timed).  Phases, by IMEXHDG_PHASE_*:
     *   EXPLICIT   DG residual M^-1 NL of the nonlinear part with the stage
     *              combinations (Sec. 4.3; eq. IMEXRKDiscretizedForm);
     *   CONDENSE   static condensation: Z = A^-1 Res0 per element and the
     *              trace right-hand side (eq. linearizedHDGsystem_schur);
     *   TRACE      the global trace solve: FP64 residuals, the inner
     *              Krylov iterations and the refinement updates;
     *   RECOVER    local recovery Q = A^-1 (R1 - B Qhat)
     *              (eq. recover_volume_unknowns);
     *   OTHER      diagnostics and operator-level calls.                   */
    double  phase_ms[5];
    int64_t depth_corrections; /* defect corrections of variable-depth stage
                                  solves, cumulative                      */
} imexhdg_diag;

#define IMEXHDG_PHASE_EXPLICIT 0
#define IMEXHDG_PHASE_CONDENSE 1
#define IMEXHDG_PHASE_TRACE    2
#define IMEXHDG_PHASE_RECOVER  3
#define IMEXHDG_PHASE_OTHER    4

typedef struct imexhdg_ctx imexhdg_ctx;

/* Fill *cfg with defaults (ARS232, nonlinear, FP64, 1 x 1 unit square,
 * k = 2, g = H = 1, dt = 1e-3, krylov_rtol = 1e-14, refine_rtol = 1e-13). */
int imexhdg_config_init(imexhdg_config *cfg);

/* Validate cfg without touching a device (the state is checked by
 * set_state).                                                             */
int imexhdg_validate(const imexhdg_config *cfg);

/* Device workspace the context needs for cfg, in bytes (host only).       */
int imexhdg_workspace_bytes(const imexhdg_config *cfg, size_t *bytes);

/* Create a context: validate, precompute the element operators in FP64 on
 * the host (local solver A^-1, A^-1 B of eq. recover_volume_unknowns, the
 * row blocks of the condensed trace system of eq.
 * linearizedHDGsystem_schur and their block-Jacobi inverses; one SDIRK
 * coefficient dt a~_ii serves every implicit stage, Sec. 5) and upload
 * them.
 *   stream      hipStream_t the context enqueues on (NULL = null stream);
 *               caller owned, must outlive the context.
 *   workspace   device buffer of >= imexhdg_workspace_bytes() bytes,
 *               256-byte aligned, caller owned and outliving the context;
 *               NULL makes the library allocate (and free) its own.
 *   ws_bytes    size of `workspace` (ignored when it is NULL).            */
int imexhdg_create(const imexhdg_config *cfg, void *stream, void *workspace,
                   size_t ws_bytes, imexhdg_ctx **out);

/* NULL-safe; synchronises the context's stream first.                    */
void imexhdg_destroy(imexhdg_ctx *ctx);

/* Sizes of the discrete spaces (Sec. 4.1): n_nodes = nx ny (k+1)^2 nodes
 * of the tensor-product space Q_k per variable, n_trace = 6 (k+1) nx ny
 * trace unknowns (three variables at the k+1 edge nodes of the 2 nx ny
 * faces of the periodic grid).  A bounded mesh reports the length of its
 * padded device trace array, 6 (k+1) (nx+2) (ny+2).  Either pointer may
 * be NULL.                                                               */
int imexhdg_sizes(const imexhdg_ctx *ctx, int64_t *n_nodes, int64_t *n_trace);

/* Coordinates of the nodes of the nodal basis (Sec. 4.1; LGL nodes mapped
 * affinely onto each element), for evaluating initial states: caller-owned
 * host arrays of n_nodes doubles each, host state ordering.              */
int imexhdg_get_nodes(const imexhdg_ctx *ctx, double *x, double *y);

/* Set q^n, the state at the nodes (Sec. 3.1 variables; Algorithm 1 takes
 * it as its input): host arrays of n_nodes doubles, host state ordering,
 * copied during the call; `vars` is IMEXHDG_VARS_*.  Rejects non-finite
 * values and h <= 0 (the wave speed of the Rusanov flux needs phi > 0)
 * with IMEXHDG_E_INVAL, leaving the state unchanged.  The subcritical
 * regime of Sec. 3 (|u| < sqrt(phi)) is where the splitting pays, not a
 * condition of the scheme: the moving vortex of Sec. 6.1 has |u| above
 * sqrt(g h) at its centre.  Resets the trace guess and the step count.  */
int imexhdg_set_state(imexhdg_ctx *ctx, int vars, const double *a,
                      const double *b, const double *c);

/* Depth under the reference plane at the nodes (variable_depth = 1;
 * Sec. 3.1: phi_B = g B): host array of n_nodes doubles in the host state
 * ordering, all finite and positive, copied during the call.  Takes effect
 * from the next step; VARS_DEPTH state arrays are converted with it
 * (phi_eta = g (h - B)), on the host and by imexhdg_set_state_device.
 * IMEXHDG_E_INVAL for a flat-bottom context or a bad value.              */
int imexhdg_set_depth(imexhdg_ctx *ctx, const double *B);

/* The same from device memory without a host copy, e.g. from a torch
 * tensor: d_state holds 3 * n_nodes values of type `dtype`
 * (IMEXHDG_DTYPE_*), the three variables one after the other, each in the
 * host state ordering (a contiguous (3, n_nodes) array).  The conversion
 * and the checks of imexhdg_set_state run on the device, ordered on the
 * context's stream after the work already enqueued there (so a producer on
 * that stream needs no synchronisation); the call then synchronises the
 * stream to read the outcome of the checks.  d_state is borrowed for the
 * call only.  IMEXHDG_E_INVAL for a rejected state (the state is left
 * unchanged) or an unknown vars / dtype.                                 */
int imexhdg_set_state_device(imexhdg_ctx *ctx, int vars, int dtype,
                             const void *d_state);

/* Copy q^n out (Sec. 3.1 variables, `vars` as for set_state) into
 * caller-owned host arrays of n_nodes doubles; synchronises the stream.  */
int imexhdg_get_state(imexhdg_ctx *ctx, int vars, double *a, double *b,
                      double *c);

/* Advance nsteps IMEX steps (Algorithm 1) on the context's stream and
 * return when they are done (the stream is synchronised).
 * IMEXHDG_LAUNCH_HOST: the trace solves check convergence every
 * `check_every` inner iterations, which synchronises the stream.
 * IMEXHDG_LAUNCH_GRAPH: the first call runs two steps host-driven to learn
 * how many refinement sweeps and inner iterations a stage solve takes,
 * then captures the step on that schedule (plus a margin) in graphs; each
 * later step is one graph launch, and the host reads the stage outcomes one
 * step behind the device, so the device never waits for it.  A step whose
 * stage solves missed refine_rtol on the schedule is redone host-driven
 * from its kept input and the schedule is widened.  While the kernel
 * profiler is on, steps run host-driven.
 * IMEXHDG_E_NOCONV if a host-driven stage solve ends above refine_rtol after
 * refine_max sweeps (the state is still advanced). */
int imexhdg_step(imexhdg_ctx *ctx, int32_t nsteps);

/* FP64 diagnostics of the current state: the discrete mass of each
 * variable (exactly conserved by the scheme, Sec. 5) and the energy E^h of
 * Lemma sdStability (Sec. 4.2), with the solver counters and the step and
 * phase times; synchronises the stream.                                  */
int imexhdg_get_diag(imexhdg_ctx *ctx, imexhdg_diag *d);

/* Thread-local text of the last error ("" if none).                      */
const char *imexhdg_last_error(void);

/* ---------------- operator-level calls (device pointers, device layout)
 * All pointers are device memory of the sizes stated, caller owned; the
 * work is enqueued on the context's stream and these calls do not
 * synchronise unless stated.                                             */

/* Device layout base of the context's current state q^n (3*n_nodes FP64,
 * volume device layout).  The state lives in a ring of three buffers, so
 * the pointer is valid until the next imexhdg_step or set_state.         */
int imexhdg_state_device(imexhdg_ctx *ctx, double **d_q);

/* out = M^-1 NL(q) (Sec. 4.3): volume term (F_NL(q), grad v)_K and the
 * Rusanov surface flux F*_NL = F* - F*_L.  q, out: 3*n_nodes FP64.       */
int imexhdg_nl_residual(imexhdg_ctx *ctx, const double *d_q, double *d_out);

/* out = M^-1 L(Q, Qhat) (Sec. 4.3): (F_L(Q), grad v)_K minus the lifted
 * hybridized flux of eq. linear_hdgflux3.  Q: 3*n_nodes, Qhat: n_trace.   */
int imexhdg_linear_residual(imexhdg_ctx *ctx, const double *d_Q,
                            const double *d_qhat, double *d_out);

/* One implicit stage (eq. IMEXRKDiscretizedForm) with coefficient
 * dt*a_ii of the configured scheme: condense Res0, solve the trace system,
 * recover Q.  d_qhat holds the initial guess on entry and the trace on
 * exit.  Synchronises; *iters and *relres (FP64 true relative residual)
 * may be NULL.                                                            */
int imexhdg_stage_solve(imexhdg_ctx *ctx, const double *d_res0, double *d_Q,
                        double *d_qhat, int32_t *iters, double *relres);

/* imexhdg_stage_solve for callers that cannot allocate device memory
 * (serving loops, harnesses that forbid allocation): the same kernels on
 * the same data, bit for bit, but every buffer the solve needs beyond its
 * arguments (Z = A^-1 Res0, the trace right-hand side and iterate, the
 * inner Krylov vectors, partial sums and the Krylov state) is taken from a
 * file-scope device array of 64 MiB that each GPU the library runs on
 * holds until the process ends, instead of the context's workspace.  The
 * call itself allocates no device memory (no hipMalloc, hipFree or
 * allocating library routine).  Contexts of one mesh only, whose solve
 * fits the array: about 57 MB at 128 x 128 elements and k = 4 in FP64;
 * larger meshes get IMEXHDG_E_INVAL with the bytes needed, before any
 * work is enqueued.  The array is shared by every call on a GPU and keeps
 * the last call's contents; the library serialises calls within a process
 * (a lock held until the call has synchronised its stream), so calls never
 * overlap on the array.  Synchronises the stream; not for graph capture.  */
int imexhdg_stage_solve_noalloc(imexhdg_ctx *ctx, const double *d_res0, double *d_Q,
                                double *d_qhat, int32_t *iters, double *relres);

/* ---------------- per-kernel event profiler
 * Kernel classes timed with HIP events recorded on the context's stream
 * around each launch of the selected class(es).                          */
#define IMEXHDG_K_NL           0  /* NL residual + stage combination       */
#define IMEXHDG_K_COMBINE      1  /* stage combination (linearized)        */
#define IMEXHDG_K_LOCAL_APPLY  2  /* Z = A^-1 Res0 per element             */
#define IMEXHDG_K_TRACE_RHS    3  /* g = sum C Z; extrapolated trace guess */
#define IMEXHDG_K_TRACE_RESID  4  /* FP64 r = g - G x, rin = P^-1 r         */
#define IMEXHDG_K_BICG_INIT    5
#define IMEXHDG_K_BICG_K1      6  /* first p + v = Ghat p of an inner solve */
#define IMEXHDG_K_BICG_K2      7  /* s update + t = Ghat s, t.s, t.t, rh.t  */
#define IMEXHDG_K_BICG_K1F     8  /* d, r update + next p, v = Ghat p      */
#define IMEXHDG_K_AXPY         9  /* x += d after a refinement sweep       */
#define IMEXHDG_K_RECOVER     10  /* Q = Z - A^-1 B Qhat per element       */
#define IMEXHDG_K_DIAG        11
#define IMEXHDG_K_LINRES      12  /* M^-1 L(Q, Qhat)                       */
#define IMEXHDG_K_COUNT       13

/* Select the class to time (0..IMEXHDG_K_COUNT-1), -1 for all classes or
 * -2 to switch timing off; clears the accumulated times.  Each timed launch
 * carries start / stop events on its own dispatch.                       */
int imexhdg_profile(imexhdg_ctx *ctx, int32_t kernel);

/* Launch count and summed device time (ms) of a class since the last
 * imexhdg_profile(); synchronises the stream.                            */
int imexhdg_profile_read(imexhdg_ctx *ctx, int32_t kernel, int64_t *launches,
                         double *total_ms);

/* The same over the launches that took at least min_ms, e.g. to leave out
 * the launches of a converged solve that return at entry.                */
int imexhdg_profile_read_min(imexhdg_ctx *ctx, int32_t kernel, double min_ms,
                             int64_t *launches, double *total_ms);

/* Static name of a kernel class, or NULL for an unknown id.              */
const char *imexhdg_kernel_name(int32_t kernel);

/* ---------------- fixed launch schedule of IMEXHDG_LAUNCH_GRAPH
 * A schedule is a number of refinement sweeps (0..8, at most refine_max)
 * and, per sweep, a budget of inner BiCGStab iterations (1..krylov_max_iter).
 * get: the schedule the graphs were captured with (sweeps = 0 before the
 * first capture); budget must hold 8 values.  set: replace the schedule and
 * capture it now (synchronises the stream); the margin the library adds
 * when it learns or widens a schedule is not applied to it.  A schedule too
 * short for the solves costs a host-driven redo of the step, after which
 * the library widens it.  IMEXHDG_E_INVAL for values out of range,
 * IMEXHDG_E_STATE if the context is not in IMEXHDG_LAUNCH_GRAPH mode.      */
int imexhdg_get_schedule(const imexhdg_ctx *ctx, int32_t *sweeps, int32_t *budget);
int imexhdg_set_schedule(imexhdg_ctx *ctx, int32_t sweeps, const int32_t *budget);

/* ---------------- launch geometry and its autotuner
 * The face-tile Krylov kernels (trace residual, BiCGStab K1 and K2) deal
 * 64-element tiles to at most `face_grid` blocks; the elementwise Krylov
 * kernels run grid-stride loops over at most `elem_grid` blocks.  Both
 * default to 1024.  Larger grids put more waves in flight, smaller ones
 * shorten the per-block re-reduction of the previous kernel's partial sums.
 * set: each value in [8, 4096]; recaptures the step graphs if any.
 * autotune: times two host-driven steps from the current state for each
 * candidate (256 ... 4096 blocks, first face_grid, then elem_grid) with the
 * kernel event profiler, weighting each kernel class's mean launch time by
 * its launch count, and keeps the fastest.  The state is restored and the
 * trace guess reset afterwards, as by set_state; the solver counters are
 * kept.  If cache_path is not NULL and the file holds a line for this
 * device, degree, mesh and precision, that choice is applied without
 * timing; otherwise the choice is appended to the file (created if
 * missing).  Chosen values are returned through face_grid / elem_grid when
 * those are not NULL.  IMEXHDG_E_STATE without a state; IMEXHDG_E_INVAL
 * for a malformed cache line.                                             */
int imexhdg_set_launch_geometry(imexhdg_ctx *ctx, int32_t face_grid, int32_t elem_grid);
int imexhdg_autotune(imexhdg_ctx *ctx, const char *cache_path, int32_t *face_grid,
                     int32_t *elem_grid);

/* ---------------- ensembles
 * An ensemble steps n independent members together: every kernel launch of
 * a step covers all members (their arrays are concatenated, each member in
 * the layout of a single context, with per-member reductions, convergence
 * flags and element operators), and each step is one graph launch on the
 * fixed schedule (IMEXHDG_LAUNCH_GRAPH is required).  Members may differ in
 * nx, ny, Lx, Ly and dt only; every other field must equal member 0's
 * (IMEXHDG_E_INVAL otherwise).  The first step after a set_state runs
 * eagerly on a probe schedule of refine_max sweeps of up to 64 inner
 * iterations; the schedule is then what the slowest member needed plus a
 * margin, widened and the step redone whenever a member misses refine_rtol.
 * Member m's state arrays follow the single-context conventions
 * (imexhdg_ens_sizes gives its n_nodes); every member needs a state before
 * the first step.  workspace, stream: as for imexhdg_create.             */
typedef struct imexhdg_ens imexhdg_ens;

int imexhdg_ens_workspace_bytes(const imexhdg_config *cfgs, int32_t n, size_t *bytes);
int imexhdg_ens_create(const imexhdg_config *cfgs, int32_t n, void *stream,
                       void *workspace, size_t ws_bytes, imexhdg_ens **out);
void imexhdg_ens_destroy(imexhdg_ens *ens);
int imexhdg_ens_members(const imexhdg_ens *ens, int32_t *n);
int imexhdg_ens_sizes(const imexhdg_ens *ens, int32_t m, int64_t *n_nodes,
                      int64_t *n_trace);
int imexhdg_ens_get_nodes(const imexhdg_ens *ens, int32_t m, double *x, double *y);
int imexhdg_ens_set_state(imexhdg_ens *ens, int32_t m, int vars, const double *a,
                          const double *b, const double *c);
/* Member m's state from device memory, as imexhdg_set_state_device.      */
int imexhdg_ens_set_state_device(imexhdg_ens *ens, int32_t m, int vars, int dtype,
                                 const void *d_state);
int imexhdg_ens_get_state(imexhdg_ens *ens, int32_t m, int vars, double *a, double *b,
                          double *c);
/* Advance every member nsteps steps; returns when they are done.         */
int imexhdg_ens_step(imexhdg_ens *ens, int32_t nsteps);
/* Member m's mass and energy; the solver counters are the ensemble's.    */
int imexhdg_ens_get_diag(imexhdg_ens *ens, int32_t m, imexhdg_diag *d);
int imexhdg_ens_get_schedule(const imexhdg_ens *ens, int32_t *sweeps, int32_t *budget);
/* Caps every member's face-class blocks at face_grid (and drops a
 * tiles-per-block sizing chosen by imexhdg_ens_autotune).                 */
int imexhdg_ens_set_launch_geometry(imexhdg_ens *ens, int32_t face_grid,
                                    int32_t elem_grid);
/* Tune the face-class blocks per member by timing graph steps from the
 * current state, which is restored afterwards with its trace guess (solver
 * counters kept).  Candidates: a cap per member (16 ... 1024 blocks), or a
 * number of 16 x 4-element tiles per block (2 ... 8: every block of every
 * member has the same work, so a large member's blocks do not form the
 * tail of a launch).  Launches of members that have converged still run
 * their blocks as no-ops, so the choice balances parallelism against that
 * overhead.  cache_path: as for imexhdg_autotune (one line per device,
 * degree, member count, element count and precision).  The cap is returned
 * in *face_grid (4096 when the blocks are sized by tiles) and the tiles per
 * block in *tiles_per_block (0: capped), each when not NULL.              */
int imexhdg_ens_autotune(imexhdg_ens *ens, const char *cache_path, int32_t *face_grid,
                         int32_t *tiles_per_block);

#ifdef __cplusplus
}
#endif
#endif /* IMEXHDG_H */
