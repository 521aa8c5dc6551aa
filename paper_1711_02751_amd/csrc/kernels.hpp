// Device kernels of one IMEX HDG-DG step and their launchers.
//
// Every kernel runs over a batch of members: independent periodic meshes of
// the same degree and physical constants, stored one after the other in
// concatenated arrays (each member in its own layout, below).  A launch
// covers all members; block b belongs to the member whose block range holds
// it, and every reduction and convergence flag is per member.  A single
// mesh is the batch of one member.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace imexhdg {

constexpr int kMaxK = 9;        // K = degree + 1 <= 9
constexpr int kLanes = 64;      // elements (or faces) per workgroup, one per lane
constexpr int kMaxComb = 12;    // inputs of a stage combination

// Reference-element tables and constants shared by every member.
struct Geom {
    int K;
    double phiB, tau;           // phi_B, sqrt(phi_B)
    double winv0, winvk;        // 1/w_0, 1/w_k
    double w[kMaxK];            // LGL weights
    double xi[kMaxK];           // LGL nodes on [-1, 1]
    double Dw[kMaxK * kMaxK];   // Dw[m*K + a] = w_m D[m][a] / w_a (weak derivative)
    double D[kMaxK * kMaxK];    // D[a*K + m] = l_m'(x_a) (strong derivative)
};

// One member: its mesh, its slices of the concatenated arrays, its element
// operators and its block ranges in the four launch classes.
struct Member {
    int nx, ny, nel;
    double sx, sy;              // 2/hx, 2/hy
    double area;                // hx hy / 4: the mass of node (i, j) is area w_i w_j
    double dt;                  // time step (scales the NL residual of a step)
    size_t vo, to;              // first volume value, first trace value
    int bv, nbv;                // volume class: 64-element blocks
    int bf, nbf;                // face class: blocks walking 64-element tiles
    int be, nbe;                // elementwise trace class: grid-stride blocks
    int bd, nbd;                // diagnostics class
    // element operators: A^-1 and W as local matrix-core fragments, G and
    // Ghat as face row-block fragments, the block-Jacobi inverses dense
    const double *Ainv, *W, *G, *Gh, *Px, *Py;
    const float *Ghf;                            // FP32 Ghat fragments
    const void *Alp;    // A^-1 as FP32 or BF16 fragments of the reduced-precision local solve
    // Bounded rectangle (bx > 0): bx x by elements padded by two ghost
    // columns and rows (nx = bx + 2, ny = by + 2).  Ghost column bx lies east
    // of the domain, bx + 1 west of it (the periodic wrap of the padded grid
    // makes it column 0's west neighbour); ghost rows by (north) and by + 1
    // (south) likewise.  x-face (i, j) is the west face of element (i, j):
    // a boundary face at i = 0 (W) and i = bx (E) for j < by; y-faces (i, 0)
    // (S) and (i, by) (N) for i < bx; the faces between ghosts are not
    // unknowns and hold zero.  A boundary row of the trace system has one
    // element and the imaginary neighbour: its self block lacks the ghost
    // side's C A^-1 B term and, with walls (bwall), gains the reflected
    // real element's coupling over that element's four faces.  dG / dGh /
    // dGhf hold, per side [W, E, S, N], four entries packed like one slot of
    // G / Ghat: the real element's faces, the boundary face (the self slot)
    // first (see side_slot).
    int bx, by, bwall;
    const double *dG, *dGh;
    const float *dGhf;
};

struct Batch {
    const Member *m;            // device array of nm members
    int nm;
    int nbv, nbf, nbe, nbd;     // blocks per class over all members
    int box;                    // 1: a bounded member (the face kernels' bounded variant)
};

// Largest face or elementwise grid of one member, and the default caps.
constexpr int kMaxLaunchGrid = 4096;

// out = self * X + sum_p coef[p] * in[p]   (X the kernel's own result)
// and, if store != nullptr, store = X.  Base pointers of the concatenated
// volume arrays; the coefficients are the same for every member.
struct Comb {
    const double *in[kMaxComb];
    double coef[kMaxComb];
    int n;
    double self;
    double *out;
    double *store;
};

// BiCGStab recurrence scalars of one member in device memory.  Each field is
// written by the first block of the member in exactly one kernel and read
// only by later kernels.
struct KrylovState {
    double rho, alpha, omega;   // rho = rh.r of the last K2, alpha, omega
    double rv;                  // rh.v of the last K2
    double rr;                  // last ||r||^2 seen by K1 or K2
    double tol2;                // stop when ||r||^2 <= tol2
    int32_t conv, breakdown, iters;
    int32_t force_brk;          // debug: the next K1f takes its breakdown branch (set by the
                                // host between launches, never written by a kernel)
    // device-driven refinement of one stage solve (fixed launch schedule)
    double relres;              // FP64 true relative residual at the last check
    int32_t stage_done;         // refine_rtol reached: later launches are no-ops
    int32_t sweep;              // sweeps started
    int32_t sweep_iters[8];     // inner iterations per sweep
};

// Outcome of one stage solve of one member on the fixed launch schedule.
constexpr int kMaxSweeps = 8;
struct StageStatus {
    double relres;
    int32_t converged, sweeps, iters_total, pad;
    int32_t sweep_iters[kMaxSweeps];
};

// Per-block partial sums of the BiCGStab reductions, [quantity][block]:
// P1 (rh.v, rh.r, r.r) of K1 / K1f, P2 (t.s, t.t, rh.t) of K2, P3 (rh.r,
// r.r) of init / refinement check.
struct KrylovBufs {
    double *P1, *P2, *P3;
    int stride;                 // >= blocks of any partial-producing class
    int sched;                  // 1: launches of the fixed schedule (own kernel symbols,
                                // so profiles keep them apart from host-driven launches)
};

// Block counts of one member (host side), for grid caps fgrid / egrid.
int member_tiles(int nx, int ny);                     // 16 x 4 element tiles
// min(tiles, fgrid), multiple of 8; with tpb > 0, min(ceil(tiles / tpb), fgrid)
int member_face_blocks(int nx, int ny, int fgrid, int tpb = 0);
int member_elem_blocks(int nel, int K, int egrid);
int member_vol_blocks(int nel);
int member_diag_blocks(int nel);

// Start / stop events for the next kernel launch of the calling thread
// (kernel profiler); cleared by that launch.
void set_launch_events(hipEvent_t start, hipEvent_t stop);

// ---------------------------------------------------------------- launchers
// All return hipError_t of the launch; each launches one kernel.  Pointers are the base pointers of
// the concatenated arrays.
// NL residual (with the stage combination); fp32: the residual's
// arithmetic in FP32 from the FP64 state, the combination in FP64.
hipError_t launch_nl(const Geom &g, const Batch &b, const double *q, const Comb &comb,
                     bool scale_dt, hipStream_t s, bool fp32 = false);
hipError_t launch_combine(const Comb &comb, size_t n, hipStream_t s);
hipError_t launch_linear_residual(const Geom &g, const Batch &b, const double *Q,
                                  const double *qhat, double *out, hipStream_t s);
hipError_t launch_local_apply(const Geom &g, const Batch &b, const double *R, double *Z,
                              hipStream_t s);
// Reduced-precision local solve with FP64 defect correction (ndc sweeps, 1
// or 2 with FP32, 1 to 3 with BF16): out = A^-1 (R - B qhat) per element, the contraction on FP32
// (bf16 = false) or BF16 matrix cores with the member's Alp fragments;
// qhat == nullptr gives Z = A^-1 R.  aii: the tableau's a~_ii (c = dt a~_ii
// per member).  status (fixed schedule): as for launch_recover.
hipError_t launch_local_lp(const Geom &g, const Batch &b, const double *R, const double *qhat,
                           double aii, double *out, bool bf16, int ndc, hipStream_t s,
                           const KrylovState *ks = nullptr, const double *partials = nullptr,
                           int stride = 0, StageStatus *status = nullptr);
// Fragment layout of the reduced-precision local solve's A^-1 (element
// type 4 bytes FP32 or 2 bytes BF16): frag[mb][kk][lane][v] =
// A^-1[16 mb + lane % 16][kw kk + (kw / 4)(lane / 16) + v], kw = 4 (FP32)
// or 32 (BF16), zero past the matrix.
int local_lp_kw(bool bf16);

// g = sum C Z per face (the trace system's right-hand side); begin (fixed
// schedule): also reset each member's stage-solve state; x (steps): the
// trace guess by linear extrapolation, x <- x + xcoef (x - xprev) and
// xprev <- x (x: last stage's solution, xprev: the one before).
hipError_t launch_trace_rhs(const Geom &g, const Batch &b, const double *Z, double *gvec,
                            hipStream_t s, KrylovState *begin = nullptr, double *x = nullptr,
                            double *xprev = nullptr, double xcoef = 0.0);
// status (fixed schedule): also record each member's stage-solve outcome
// from ks and the final trace_residual's partials [4][stride].
hipError_t launch_recover(const Geom &g, const Batch &b, const double *Z, const double *qhat,
                          double *Q, hipStream_t s, const KrylovState *ks = nullptr,
                          const double *partials = nullptr, int stride = 0,
                          StageStatus *status = nullptr);
// FP64 r = g - G x (its norm only) and rin = P^-1 r = ghat - Ghat x (stored
// in the inner solve's precision); partials [4][face blocks] of ||r||^2,
// ||g||^2, ||ghat||^2, ||rin||^2.  With `skip`, members whose stage solve is
// done return.
// BiCGStab on Ghat d = rin with d0 = 0: init and K1, then per iteration
// K2 and K1f (the next K1 fused with this iteration's d and r updates;
// s = r - alpha v is formed by both, never stored, so r is double buffered
// like p and v: K1f reads r and writes r' to the other buffer); x += d
// after the sweep.  Each exists for an FP64 and an FP32 inner solve
// (matrix-core fragments in the same precision).
#define IMEXHDG_KRYLOV_DECLS(T)                                                                \
    hipError_t launch_trace_residual(const Geom &g, const Batch &b, const double *x,          \
                                     const double *gvec, T *rin, double *partials,            \
                                     int stride, const KrylovState *skip, hipStream_t s);     \
    hipError_t launch_bicg_init(const Geom &g, const Batch &b, const T *rin, T *r, T *rh,     \
                                T *p, T *v, T *d, KrylovState *ks, double tol2,               \
                                const KrylovBufs &kb, hipStream_t s);                         \
    hipError_t launch_bicg_k1(const Geom &g, const Batch &b, const T *r, const T *rh,         \
                              const T *pin, const T *vin, T *pout, T *vout, KrylovState *ks,  \
                              const KrylovBufs &kb, hipStream_t s);                           \
    hipError_t launch_bicg_k2(const Geom &g, const Batch &b, const T *r, const T *v,          \
                              const T *rh, T *t, KrylovState *ks, const KrylovBufs &kb,       \
                              hipStream_t s);                                                 \
    hipError_t launch_bicg_k1f(const Geom &g, const Batch &b, const T *rin, const T *t,       \
                               const T *rh, const T *pin, const T *vin, T *pout, T *vout,     \
                               T *rout, T *d, KrylovState *ks, const KrylovBufs &kb,          \
                               hipStream_t s);                                                \
    hipError_t launch_axpy(double *y, const T *x, double a, size_t n, hipStream_t s);
IMEXHDG_KRYLOV_DECLS(double)
IMEXHDG_KRYLOV_DECLS(float)
#undef IMEXHDG_KRYLOV_DECLS
// Device-driven refinement (no host reads inside a stage solve), per
// stage: trace_rhs(begin = ks); per sweep trace_residual(skip = ks),
// refine_k1 (reduces the residual norms, ends the member's stage solve
// when relres <= refine_rtol, else starts its inner solve with its
// tolerance and runs the first K1), the inner iterations and
// axpy_guarded; finally trace_residual and recover(status), which records
// a StageStatus per member.
#define IMEXHDG_REFINE_DECLS(T)                                                                \
    hipError_t launch_refine_k1(const Geom &g, const Batch &b, const T *rin, T *r, T *rh,     \
                                T *p, T *v, T *d, KrylovState *ks, const double *partials,    \
                                int stride, double refine_rtol, double inner_rtol,            \
                                const KrylovBufs &kb, hipStream_t s);                         \
    hipError_t launch_axpy_guarded(const Geom &g, const Batch &b, double *y, const T *x,      \
                                   KrylovState *ks, hipStream_t s);
IMEXHDG_REFINE_DECLS(double)
IMEXHDG_REFINE_DECLS(float)
#undef IMEXHDG_REFINE_DECLS

// Boundary states of a bounded member (bx > 0) into its ghost elements of
// the volume array q.  Exact-solution data: the translating vortex of eq.
// tc_vortex_ic (Sec. 6.1) at time tstep[0] dt + toff, evaluated at the
// boundary point each ghost node faces (ghost column bx: x = Lx at the
// node's y; column bx + 1: x = 0; row by: y = Ly; row by + 1: y = 0).
// Walls (bwall): the reflection (eq. reflection) of the adjacent real
// element's value at the boundary node the ghost node faces, read from q
// itself.  Corner ghosts are zero.
// tstep[0] is the step count of the state (an integer held as a double);
// with tnext != nullptr the kernel also writes tnext[0] = tstep[0] + 1.
struct Vortex {
    double H, g, uinf, vinf, beta, xc, yc;
};
hipError_t launch_bc_fill(const Geom &g, const Batch &b, double *q, const double *tstep,
                          double toff, double *tnext, const Vortex &vx, hipStream_t s);
// Variable bathymetry (nodal phi_B in pB, the volume layout of one
// variable, N / 3 values): the explicit residual M^-1 NL with the stage
// combination, as launch_nl; and the stage residual of the linear part,
// out = R - (Q - a~_ii dt M^-1 L(Q)) with the source term, partials
// [2][volume blocks] of ||out||^2 and ||R||^2 (see k_dg_var).
hipError_t launch_nl_var(const Geom &g, const Batch &b, const double *q, const double *pB,
                         const Comb &comb, bool scale_dt, hipStream_t s);
hipError_t launch_stage_res_var(const Geom &g, const Batch &b, const double *Q,
                                const double *pB, const double *R, double aii, double *out,
                                double *partials, int stride, hipStream_t s);

// p[0] = v (one thread; stream ordered, so a host value can be placed
// between kernels without a copy from host memory).
hipError_t launch_put(double *p, double v, hipStream_t s);

// partials [5][diag blocks]: mass of phi_eta, U, V; energy; non-finite count
// (bounded members: over the real elements only)
hipError_t launch_diag(const Geom &g, const Batch &b, const double *q, double *partials,
                       int stride, hipStream_t s);

// Scratch of the allocation-free stage solve: a file-scope device array of
// kScratchBytes per GPU.  scratch_init(dev) takes its address on device
// `dev` (which must be current) once per device; scratch_base(dev) returns
// it afterwards (nullptr before).
constexpr size_t kScratchBytes = (size_t)64 << 20;
hipError_t scratch_init(int dev);
void *scratch_base(int dev);
// n32 zero words at p (a fill kernel, so that no memset node is ever
// recorded into a caller's graph).
hipError_t launch_zero(void *p, size_t n32, hipStream_t s);

// One member's state from a caller's device array `src` (3 nel K^2 values,
// FP64 or, with f32, FP32; variable-major, each variable in the host state
// ordering [e][j K + i]) into the volume device layout at dst, converting
// depth variables (h, hu, hv) to (phi_eta, U, V) when `depth` is set.
// partials [1][blocks]: per block, the count of nodes that are not finite
// or not of positive depth.
// bx > 0 (bounded member): src holds the bx x (nel / bx) real elements and
// dst is the padded layout with nxp = bx + 2 elements per row.  pBn: the
// nodal phi_B in dst's layout (variable depth: phi_eta = g h - phi_B at the
// node), or nullptr for phi_B = g H.
hipError_t launch_state_in(const void *src, bool f32, bool depth, double g, double H,
                           int nel, int K, double *dst, double *partials, int blocks,
                           hipStream_t s, int bx = 0, int nxp = 0,
                           const double *pBn = nullptr);
// Blocks launch_state_in uses for nel elements of degree K - 1 (at most cap).
int state_in_blocks(int nel, int K, int cap);

}  // namespace imexhdg
