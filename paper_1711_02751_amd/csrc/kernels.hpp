// Device kernels of one IMEX HDG-DG step and their launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace imexhdg {

constexpr int kMaxK = 9;        // K = degree + 1 <= 9
constexpr int kLanes = 64;      // elements (or faces) per workgroup, one per lane
constexpr int kMaxComb = 12;    // inputs of a stage combination

// Mesh geometry and the small reference-element tables, passed by value.
struct Geom {
    int nx, ny, nel, K;
    double sx, sy;              // 2/hx, 2/hy
    double phiB, tau;           // phi_B, sqrt(phi_B)
    double winv0, winvk;        // 1/w_0, 1/w_k
    double Dw[kMaxK * kMaxK];   // Dw[m*K + a] = w_m D[m][a] / w_a (weak derivative)
    double mass[kMaxK * kMaxK]; // (hx/2)(hy/2) w_i w_j at node j*K + i
    int fgrid, egrid;           // grid caps of the face-tile and elementwise Krylov
                                // launches (launch geometry, tuned per mesh)
};

// Largest grid of any launch that leaves per-block partial sums.
constexpr int kMaxLaunchGrid = 4096;

// out = self * X + sum_p coef[p] * in[p]   (X the kernel's own result)
// and, if store != nullptr, store = X.  Volume device layout.
struct Comb {
    const double *in[kMaxComb];
    double coef[kMaxComb];
    int n;
    double self;
    double *out;
    double *store;
};

// BiCGStab recurrence scalars in device memory.  Each field is written by
// block 0 of exactly one kernel and read only by later kernels.
struct KrylovState {
    double rho, alpha, omega;   // rho = rh.r of the last K2, alpha, omega
    double rr;                  // last ||r||^2 seen by K1
    double tol2;                // stop when ||r||^2 <= tol2
    int32_t conv, breakdown, iters, pad;
    // device-driven refinement of one stage solve (fixed launch schedule)
    double relres;              // FP64 true relative residual at the last check
    int32_t stage_done;         // refine_rtol reached: later launches are no-ops
    int32_t sweep;              // sweeps started
    int32_t sweep_iters[8];     // inner iterations per sweep
};

// Outcome of one stage solve on the fixed launch schedule.
constexpr int kMaxSweeps = 8;
struct StageStatus {
    double relres;
    int32_t converged, sweeps, iters_total, pad;
    int32_t sweep_iters[kMaxSweeps];
};

// Per-block partial sums of the three BiCGStab reductions, [quantity][block].
struct KrylovBufs {
    double *P1, *P2, *P3;
    int stride;                 // >= max grid of any Krylov launch
    int sched;                  // 1: launches of the fixed schedule (own kernel symbols,
                                // so profiles keep them apart from host-driven launches)
};

// Capped grid sizes of the face-tile kernels, the elementwise Krylov
// kernels and the diagnostics kernel; partial arrays hold this many blocks.
struct Geom;
bool is_tiled(const Geom &g);   // mesh is a whole number of 16 x 4 tiles
unsigned face_grid(const Geom &g);
unsigned elem_grid(const Geom &g);
unsigned diag_grid(const Geom &g);

// ---------------------------------------------------------------- launchers
// All return hipError_t of the launch.
hipError_t launch_nl(const Geom &g, const double *q, const Comb &comb, hipStream_t s);
hipError_t launch_combine(const Geom &g, const Comb &comb, size_t n, hipStream_t s);
hipError_t launch_linear_residual(const Geom &g, const double *Q, const double *qhat,
                                  double *out, hipStream_t s);
hipError_t launch_local_apply(const Geom &g, const double *Ainv, const double *R,
                              double *Z, hipStream_t s);
hipError_t launch_trace_rhs(const Geom &g, const double *Z, const double *Pxinv,
                            const double *Pyinv, double *gvec, double *ghat, hipStream_t s);
hipError_t launch_recover(const Geom &g, const double *W, const double *Z,
                          const double *qhat, double *Q, hipStream_t s);
// FP64 r = g - G x and rin = ghat - Ghat x (stored in the inner solve's
// precision); partials [4][face_grid] of ||r||^2, ||g||^2, ||ghat||^2,
// ||rin||^2.  BiCGStab on Ghat d = rin with d0 = 0: init, then per
// iteration K1, K2, K3; x += d after the sweep.  Each exists for an FP64
// and an FP32 inner solve (matrix-core fragments in the same precision).
#define IMEXHDG_KRYLOV_DECLS(T)                                                                \
    hipError_t launch_trace_residual(const Geom &g, const double *G, const double *Gh,        \
                                     const double *x, const double *gvec,                     \
                                     const double *ghat, double *r, T *rin, double *partials, \
                                     int stride, const int32_t *skip, hipStream_t s);         \
    hipError_t launch_bicg_init(const Geom &g, const T *rin, T *r, T *rh, T *p, T *v, T *d,  \
                                KrylovState *ks, double tol2, const KrylovBufs &kb,           \
                                hipStream_t s);                                               \
    hipError_t launch_bicg_k1(const Geom &g, const T *Gh, const T *r, const T *rh,            \
                              const T *pin, const T *vin, T *pout, T *vout, KrylovState *ks,  \
                              const KrylovBufs &kb, hipStream_t s);                           \
    hipError_t launch_bicg_k2(const Geom &g, const T *Gh, const T *r, const T *v, T *sv,      \
                              T *t, KrylovState *ks, const KrylovBufs &kb, hipStream_t s);    \
    hipError_t launch_bicg_k3(const Geom &g, T *d, T *r, const T *rh, const T *p,             \
                              const T *sv, const T *t, KrylovState *ks, const KrylovBufs &kb, \
                              hipStream_t s);                                                 \
    hipError_t launch_axpy(double *y, const T *x, double a, size_t n, hipStream_t s);
IMEXHDG_KRYLOV_DECLS(double)
IMEXHDG_KRYLOV_DECLS(float)
#undef IMEXHDG_KRYLOV_DECLS
// Device-driven refinement (no host reads inside a stage solve):
//   stage_begin; then per sweep: trace_residual(skip = &ks->stage_done),
//   refine_check (reduces the residual norms, stops the stage solve when
//   relres <= refine_rtol, else initialises the inner solve with its
//   tolerance), inner iterations, axpy_guarded; finally trace_residual and
//   stage_finish, which records a StageStatus.
hipError_t launch_stage_begin(KrylovState *ks, hipStream_t s);
#define IMEXHDG_REFINE_DECLS(T)                                                                \
    hipError_t launch_refine_check(const Geom &g, const T *rin, T *r, T *rh, T *p, T *v,      \
                                   T *d, KrylovState *ks, const double *partials, int stride, \
                                   double refine_rtol, double inner_rtol,                     \
                                   const KrylovBufs &kb, hipStream_t s);                      \
    hipError_t launch_axpy_guarded(double *y, const T *x, size_t n, KrylovState *ks,          \
                                   hipStream_t s);
IMEXHDG_REFINE_DECLS(double)
IMEXHDG_REFINE_DECLS(float)
#undef IMEXHDG_REFINE_DECLS
hipError_t launch_stage_finish(const Geom &g, KrylovState *ks, const double *partials,
                               int stride, StageStatus *out, hipStream_t s);

// partials [5][diag_grid]: mass of phi_eta, U, V; energy; non-finite count
hipError_t launch_diag(const Geom &g, const double *q, double *partials, int stride,
                       hipStream_t s);

}  // namespace imexhdg
