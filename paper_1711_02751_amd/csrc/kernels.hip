// HIP kernels for gfx950 (CDNA4, wave64) of one IMEX HDG-DG step.
//
// Layouts (element index e = ey*nx + ex fastest, so a wave of 64 lanes that
// handles 64 consecutive elements reads 64 consecutive doubles per access):
//   volume v[c][j*K + i][e]     c = phi_eta, U, V;  N = 3 K^2 nel values
//   trace  t[d][c][j][e]        d = 0 x-face e (west face of element e),
//                               d = 1 y-face e (south face of element e)
// Workgroups are 64 lanes (elements or faces) x K "rows"; the row index is
// wave-uniform, so every reference-element matrix entry a wave needs is the
// same for all its lanes and is read through the scalar unit.  Each member
// of a batch has this layout within its slice of the concatenated arrays.
#include "kernels.hpp"

#include <hip/hip_ext.h>

#include <algorithm>
#include <mutex>

namespace imexhdg {

// Events for the next launch on this thread (kernel profiler): attached to
// the dispatch itself, so they time the same interval a kernel trace does.
thread_local hipEvent_t t_launch_ev[2] = {nullptr, nullptr};

void set_launch_events(hipEvent_t start, hipEvent_t stop) {
    t_launch_ev[0] = start;
    t_launch_ev[1] = stop;
}

#define KLAUNCH(kernel, grid, block, shm, stream, ...)                                 \
    do {                                                                               \
        if (t_launch_ev[0]) {                                                          \
            hipExtLaunchKernelGGL(kernel, grid, block, shm, stream, t_launch_ev[0],    \
                                  t_launch_ev[1], 0, __VA_ARGS__);                     \
            t_launch_ev[0] = t_launch_ev[1] = nullptr;                                 \
        } else {                                                                       \
            hipLaunchKernelGGL(kernel, grid, block, shm, stream, __VA_ARGS__);         \
        }                                                                              \
    } while (0)

namespace {

__device__ __forceinline__ int wave_id() {
    return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// v from lane l ^ m within groups of lanes (data-parallel primitives: a
// quad permutation or a row mirror), in two 32-bit halves.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double lane_d(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the wave, the same value in every lane: within each row of 16
// lanes by exchanges between lanes (quad xor 1, quad xor 2, half-row
// mirror, row mirror; both partners of an exchange add the same two values,
// so every lane of a row holds the same sum), then the four row sums in a
// fixed order.  Every lane of the wave must be active (callers: whole
// blocks of multiples of 64 threads in uniform control flow).
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_d<0xB1>(v);    // quad_perm [1, 0, 3, 2]
    v += dpp_d<0x4E>(v);    // quad_perm [2, 3, 0, 1]
    v += dpp_d<0x141>(v);   // row_half_mirror
    v += dpp_d<0x140>(v);   // row_mirror
    return (lane_d(v, 0) + lane_d(v, 16)) + (lane_d(v, 32) + lane_d(v, 48));
}

// Matrices shared by all lanes of a wave are read through the constant
// address space, so wave-uniform indices compile to scalar loads.
typedef const __attribute__((address_space(4))) double cdouble;

__device__ __forceinline__ const cdouble *as_const(const double *p) {
    return (const cdouble *)(p);
}

struct Nbr {
    int e, east, west, north, south;
};

__device__ __forceinline__ Nbr neighbours(int e, int nx, int ny) {
    Nbr n;
    const int ex = e % nx, ey = e / nx;
    n.e = e;
    n.east = ey * nx + (ex + 1 == nx ? 0 : ex + 1);
    n.west = ey * nx + (ex == 0 ? nx - 1 : ex - 1);
    n.north = (ey + 1 == ny ? 0 : ey + 1) * nx + ex;
    n.south = (ey == 0 ? ny - 1 : ey - 1) * nx + ex;
    return n;
}

// Members are read through the constant address space: a block-uniform
// member index compiles to scalar loads.
typedef const __attribute__((address_space(4))) Member cmember;

enum { CV = 0, CF = 1, CE = 2, CD = 3 };   // volume, face, elementwise, diagnostics

template <int C> __device__ __forceinline__ int first_block(const cmember &m) {
    return C == CV ? m.bv : C == CF ? m.bf : C == CE ? m.be : m.bd;
}

// Member holding block b of launch class C (binary search over the first
// blocks), and b's index within the member.
template <int C>
__device__ __forceinline__ int member_of(const Batch &bt, int b, int &local) {
    const cmember *m = (const cmember *)bt.m;
    int lo = 0, hi = bt.nm - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (first_block<C>(m[mid]) <= b) lo = mid;
        else hi = mid - 1;
    }
    local = b - first_block<C>(m[lo]);
    return lo;
}

__device__ __forceinline__ Member load_member(const Batch &bt, int i) {
    const cmember &c = ((const cmember *)bt.m)[i];
    Member r;
    r.nx = c.nx; r.ny = c.ny; r.nel = c.nel;
    r.sx = c.sx; r.sy = c.sy; r.area = c.area; r.dt = c.dt;
    r.vo = c.vo; r.to = c.to;
    r.bv = c.bv; r.nbv = c.nbv; r.bf = c.bf; r.nbf = c.nbf;
    r.be = c.be; r.nbe = c.nbe; r.bd = c.bd; r.nbd = c.nbd;
    r.Ainv = c.Ainv; r.W = c.W; r.G = c.G; r.Gh = c.Gh; r.Px = c.Px; r.Py = c.Py;
    r.Ghf = c.Ghf;
    r.Alp = c.Alp;
    r.bx = c.bx; r.by = c.by; r.bwall = c.bwall;
    r.dG = c.dG; r.dGh = c.dGh; r.dGhf = c.dGhf;
    return r;
}

// Bounded member (bx > 0): faces between ghost elements are not unknowns.
__device__ __forceinline__ bool dummy_face(int d, int ex, int ey, const Member &g) {
    return g.bx > 0 && (d == 0 ? (ey >= g.by || ex == g.bx + 1) : (ex >= g.bx || ey == g.by + 1));
}

// Side of a boundary face of a bounded member: 0 W, 1 E, 2 S, 3 N, -1 none.
__device__ __forceinline__ int boundary_side(int d, int ex, int ey, const Member &g) {
    if (g.bx == 0) return -1;
    if (d == 0) return ey < g.by ? (ex == 0 ? 0 : ex == g.bx ? 1 : -1) : -1;
    return ex < g.bx ? (ey == 0 ? 2 : ey == g.by ? 3 : -1) : -1;
}

// Deterministic reductions without fences or atomics.  A producer kernel
// stores one partial sum per block with a plain store; the partials become
// visible to the next kernel on the stream at the launch boundary, where
// every block of the consumer reduces them again in the same fixed order
// (per-member grids are capped, so this costs a few KB of L2 reads per
// block).  Partials are indexed by the global block; a member reduces its
// own block range.

// Workgroup barrier that orders LDS only.  __syncthreads() also orders
// global memory, which on this target waits for every vector memory
// operation in flight, loads included; a barrier that only hands LDS data
// between waves need not wait for the global loads issued ahead of it.
// Materialise a kernel argument in scalar registers here: the compiler
// otherwise loads arguments where they are first used, one dependent
// round trip each, on the path to the first global loads.
template <typename P> __device__ __forceinline__ void arg_now(P p) { asm volatile("" ::"s"(p)); }

__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Block sum of NV values per thread; the result is returned to every thread.
// BD > 0: the block size, known at compile time (no argument load).
template <int NV, int BD = 0>
__device__ void block_sum(double (&v)[NV]) {
    __shared__ double sred[16][NV];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nw = BD > 0 ? BD / 64 : (blockDim.x + 63) >> 6;
    lds_barrier();
    for (int q = 0; q < NV; ++q) {
        double s = wave_sum(v[q]);
        if (lane == 0) sred[w][q] = s;
    }
    lds_barrier();
    for (int q = 0; q < NV; ++q) {
        double s = 0.0;
        for (int i = 0; i < nw; ++i) s += sred[i][q];
        v[q] = s;
    }
    lds_barrier();
}

// partials[q * stride + blockIdx.x] = block sum of v[q], the same sum in
// the same order as block_sum, formed by thread 0 only.  Called once, at
// the end of a kernel (its LDS is not reused, so no barrier precedes it).
template <int NV, int BD = 0>
__device__ void store_partials(double (&v)[NV], double *partials, int stride) {
    __shared__ double sred[16][NV];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nw = BD > 0 ? BD / 64 : (blockDim.x + 63) >> 6;
    for (int q = 0; q < NV; ++q) {
        const double s = wave_sum(v[q]);
        if (lane == 0) sred[w][q] = s;
    }
    lds_barrier();
    if (threadIdx.x == 0)
        for (int q = 0; q < NV; ++q) {
            double s = 0.0;
            for (int i = 0; i < nw; ++i) s += sred[i][q];
            partials[q * stride + blockIdx.x] = s;
        }
}

// out[q] = sum_{b < n} partials[q * stride + b], identical in every block
// (four loads per quantity in flight per thread, in a fixed order)
template <int NV>
__device__ void reduce_partials(const double *__restrict__ partials, int stride, int n,
                                double (&out)[NV]) {
    const int bd = blockDim.x;
    for (int q = 0; q < NV; ++q) out[q] = 0.0;
    int i = threadIdx.x;
    for (; i + 3 * bd < n; i += 4 * bd) {
        double a[NV][4];
#pragma unroll
        for (int q = 0; q < NV; ++q)
#pragma unroll
            for (int u = 0; u < 4; ++u) a[q][u] = partials[q * stride + i + u * bd];
#pragma unroll
        for (int q = 0; q < NV; ++q) out[q] += (a[q][0] + a[q][1]) + (a[q][2] + a[q][3]);
    }
    for (; i < n; i += bd) {
        double a[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) a[q] = partials[q * stride + i];
#pragma unroll
        for (int q = 0; q < NV; ++q) out[q] += a[q];
    }
    block_sum<NV>(out);
}

// reduce_partials split in two, so that its loads can be issued ahead of
// other loads of the kernel: load() sums this thread's values (one per
// quantity unless the member has more blocks than threads) in a fixed
// order, finish() sums over the block.  Identical in every block.  Any
// loop over further values stays in load(), ahead of the loads issued
// between the two calls, so finish() waits for the partial sums only.
// Loads whose result is not needed read a valid address and are discarded
// rather than skipped: a load under a branch leaves the compiler unsure
// how many loads follow an earlier one, and it then waits for all of them.
template <int NV, int BD = 0> struct EarlyPartials {
    double a[NV], b[NV];   // this thread's first value, the sum of the others
    bool has;
    __device__ __forceinline__ void load(const double *__restrict__ partials, int stride, int n) {
        const int i = threadIdx.x;
        has = i < n;
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            a[q] = partials[q * stride + (has ? i : 0)];
            b[q] = 0.0;
        }
        const int bd = BD > 0 ? BD : (int)blockDim.x;
        for (int j = i + bd; j < n; j += bd)
#pragma unroll
            for (int q = 0; q < NV; ++q) b[q] += partials[q * stride + j];
    }
    __device__ __forceinline__ void finish(double (&out)[NV]) {
#pragma unroll
        for (int q = 0; q < NV; ++q) out[q] = has ? a[q] + b[q] : 0.0;
        block_sum<NV, BD>(out);
    }
};

// ------------------------------------------------------------- physics
// Nonlinear remainder of the flux, F_NL = F - F_L (Sec. 4.3), in closed form:
//   x: (0, U^2/phi + phi_eta^2/2, U V/phi),  y: (0, U V/phi, V^2/phi + phi_eta^2/2)
// Rusanov flux of the remainder (eqs. Full_russanov, Linear_russanov):
//   F*_NL . n = {F_NL} . n + (tau* - tau_L*) / 2 (q- - q+)
//   tau* = max over both sides of |u . n| + sqrt(phi),  tau_L* = sqrt(phi_B)
// TC: the arithmetic type (FP64, or FP32 for the reduced-precision DG
// residual).
template <typename TC>
__device__ __forceinline__ void nl_flux_n(TC p, TC U, TC V, TC phiB, TC nx, TC ny, TC &f1,
                                          TC &f2, TC &speed) {
    const TC phi = p + phiB;
    const TC inv = TC(1) / phi;
    const TC uu = U * U * inv, uv = U * V * inv, vv = V * V * inv;
    const TC hp = TC(0.5) * p * p;
    f1 = (uu + hp) * nx + uv * ny;
    f2 = uv * nx + (vv + hp) * ny;
    speed = fabs((U * nx + V * ny) * inv) + sqrt(phi);
}

template <typename TC>
__device__ __forceinline__ void rusanov_nl(const TC qm[3], const TC qp[3], TC nx, TC ny,
                                           TC phiB, TC tauL, TC out[3]) {
    TC fm1, fm2, sm, fp1, fp2, sp;
    nl_flux_n<TC>(qm[0], qm[1], qm[2], phiB, nx, ny, fm1, fm2, sm);
    nl_flux_n<TC>(qp[0], qp[1], qp[2], phiB, nx, ny, fp1, fp2, sp);
    const TC diss = TC(0.5) * (fmax(sm, sp) - tauL);
    out[0] = diss * (qm[0] - qp[0]);
    out[1] = TC(0.5) * (fm1 + fp1) + diss * (qm[1] - qp[1]);
    out[2] = TC(0.5) * (fm2 + fp2) + diss * (qm[2] - qp[2]);
}

// -------------------------------------------------- NL residual kernel
// One thread per (element, node row j).  Volume term in weak form,
//   M^-1 (F, grad v)_K at (a, b) = (2/hx) sum_m Dw[m][a] F_x(m, b)
//                                + (2/hy) sum_m Dw[m][b] F_y(a, m),
// with F_y exchanged through LDS; surface term -(2/h) Phi / w_end at the
// face nodes.  The epilogue applies the stage combination `comb`.
// Every load that does not depend on arithmetic is issued at the start (the
// row, its east and west neighbours and, for K <= 6, the neighbour row
// across the south or north face), so a block (one per CU at this register
// count) waits for memory once instead of once per face; the waves of the
// middle rows, which have no north or south face, load their own row
// instead of a neighbour's so that the loads stay unconditional (see
// EarlyPartials), and for K <= 6 the combination inputs are loaded one
// input ahead.  (Larger K would spill registers.)
template <int K, typename TC = double>
__global__ __launch_bounds__(64 * K) void k_nl(const double *__restrict__ q, const Geom g,
                                               const Batch bt, const Comb comb,
                                               int scale_dt) {
    __shared__ TC sFy[2][K][K][64];
    const int lane = threadIdx.x & 63;
    const int j = wave_id();
    int lb;
    const Member mb = load_member(bt, member_of<CV>(bt, blockIdx.x, lb));
    q += mb.vo;
    const int e = lb * 64 + lane;
    const bool active = e < mb.nel;
    const Nbr nb = neighbours(active ? e : 0, mb.nx, mb.ny);
    const size_t nel = mb.nel, NN = (size_t)K * K * nel;
    const TC phiB = (TC)g.phiB, tauL = (TC)g.tau;

    TC p[K], U[K], V[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const size_t o = (size_t)(j * K + i) * nel + nb.e;
        p[i] = (TC)q[o];
        U[i] = (TC)q[NN + o];
        V[i] = (TC)q[2 * NN + o];
    }
    // east neighbour's first node and west neighbour's last node of row j
    TC qe[3], qw[3];
    {
        const size_t oe = (size_t)(j * K + 0) * nel + nb.east;
        const size_t ow = (size_t)(j * K + K - 1) * nel + nb.west;
        qe[0] = (TC)q[oe]; qe[1] = (TC)q[NN + oe]; qe[2] = (TC)q[2 * NN + oe];
        qw[0] = (TC)q[ow]; qw[1] = (TC)q[NN + ow]; qw[2] = (TC)q[2 * NN + ow];
    }
    // across the north face (j = K - 1) or the south face (j = 0): the
    // neighbour's first or last row; the middle rows read their own row
    constexpr bool kHoist = K <= 6;
    const bool north = (j == K - 1), edge = (j == K - 1 || j == 0);
    TC qs[kHoist ? K : 1][3];
    if constexpr (kHoist) {
        const int other = north ? nb.north : j == 0 ? nb.south : nb.e;
        const int orow = north ? 0 : j == 0 ? K - 1 : j;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const size_t o = (size_t)(orow * K + i) * nel + other;
            qs[i][0] = (TC)q[o]; qs[i][1] = (TC)q[NN + o]; qs[i][2] = (TC)q[2 * NN + o];
        }
    }
    TC fx1[K], fx2[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const TC inv = TC(1) / (p[i] + phiB);
        const TC hp = TC(0.5) * p[i] * p[i];
        const TC uv = U[i] * V[i] * inv;
        fx1[i] = U[i] * U[i] * inv + hp;
        fx2[i] = uv;
        sFy[0][j][i][lane] = uv;
        sFy[1][j][i][lane] = V[i] * V[i] * inv + hp;
    }
    const TC sx = (TC)mb.sx, sy = (TC)mb.sy;
    TC o0[K], o1[K], o2[K];
#pragma unroll
    for (int a = 0; a < K; ++a) {
        TC s1 = 0, s2 = 0;
#pragma unroll
        for (int m = 0; m < K; ++m) {
            s1 += (TC)g.Dw[m * K + a] * fx1[m];
            s2 += (TC)g.Dw[m * K + a] * fx2[m];
        }
        o0[a] = 0;
        o1[a] = sx * s1;
        o2[a] = sx * s2;
    }
    // east and west faces of row j
    {
        TC qm[3], f[3];
        qm[0] = p[K - 1]; qm[1] = U[K - 1]; qm[2] = V[K - 1];
        rusanov_nl<TC>(qm, qe, TC(1), TC(0), phiB, tauL, f);
        const TC se = (TC)(mb.sx * g.winvk);
        o0[K - 1] -= se * f[0]; o1[K - 1] -= se * f[1]; o2[K - 1] -= se * f[2];
        qm[0] = p[0]; qm[1] = U[0]; qm[2] = V[0];
        rusanov_nl<TC>(qm, qw, TC(-1), TC(0), phiB, tauL, f);
        const TC sw = (TC)(mb.sx * g.winv0);
        o0[0] -= sw * f[0]; o1[0] -= sw * f[1]; o2[0] -= sw * f[2];
    }
    lds_barrier();
#pragma unroll
    for (int i = 0; i < K; ++i) {
        TC s1 = 0, s2 = 0;
#pragma unroll
        for (int m = 0; m < K; ++m) {
            s1 += (TC)g.Dw[m * K + j] * sFy[0][m][i][lane];
            s2 += (TC)g.Dw[m * K + j] * sFy[1][m][i][lane];
        }
        o1[i] += sy * s1;
        o2[i] += sy * s2;
    }
    if (edge) {
        const TC ny = north ? TC(1) : TC(-1);
        const TC sc = (TC)(mb.sy * (north ? g.winvk : g.winv0));
        const int other = north ? nb.north : nb.south;
        const int orow = north ? 0 : K - 1;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            TC qm[3] = {p[i], U[i], V[i]}, qp[3], f[3];
            if constexpr (kHoist) {
                qp[0] = qs[i][0]; qp[1] = qs[i][1]; qp[2] = qs[i][2];
            } else {
                const size_t o = (size_t)(orow * K + i) * nel + other;
                qp[0] = (TC)q[o]; qp[1] = (TC)q[NN + o]; qp[2] = (TC)q[2 * NN + o];
            }
            rusanov_nl<TC>(qm, qp, TC(0), ny, phiB, tauL, f);
            o0[i] -= sc * f[0]; o1[i] -= sc * f[1]; o2[i] -= sc * f[2];
        }
    }
    if (!active) return;
    // the step's combinations take dt NL (dt of the member); input by
    // input, the 3 K values of this row are loaded together
    const double sc = scale_dt ? mb.dt : 1.0;
    const size_t o = mb.vo + (size_t)(j * K) * nel + e;
    double d0[K], d1[K], d2[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        d0[i] = (double)o0[i] * sc;
        d1[i] = (double)o1[i] * sc;
        d2[i] = (double)o2[i] * sc;
    }
    if (comb.store) {
#pragma unroll
        for (int i = 0; i < K; ++i) {
            comb.store[o + (size_t)i * nel] = d0[i];
            comb.store[NN + o + (size_t)i * nel] = d1[i];
            comb.store[2 * NN + o + (size_t)i * nel] = d2[i];
        }
    }
#pragma unroll
    for (int i = 0; i < K; ++i) {
        d0[i] *= comb.self;
        d1[i] *= comb.self;
        d2[i] *= comb.self;
    }
    // input t + 1 is loaded while input t is added (the last round reloads
    // input n - 1 and discards it: unconditional, see EarlyPartials)
    double v0[K], v1[K], v2[K];
    if (kHoist && comb.n > 0) {
        const double *in = comb.in[0] + o;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            v0[i] = in[(size_t)i * nel];
            v1[i] = in[NN + (size_t)i * nel];
            v2[i] = in[2 * NN + (size_t)i * nel];
        }
    }
    for (int t = 0; t < comb.n; ++t) {
        if constexpr (!kHoist) {   // one input at a time
            const double *in = comb.in[t] + o;
#pragma unroll
            for (int i = 0; i < K; ++i) {
                v0[i] = in[(size_t)i * nel];
                v1[i] = in[NN + (size_t)i * nel];
                v2[i] = in[2 * NN + (size_t)i * nel];
            }
        }
        const double *in = comb.in[kHoist && t + 1 < comb.n ? t + 1 : t] + o;
        const double cf = comb.coef[t];
        double w0[K], w1[K], w2[K];
        if constexpr (kHoist) {
#pragma unroll
            for (int i = 0; i < K; ++i) {
                w0[i] = in[(size_t)i * nel];
                w1[i] = in[NN + (size_t)i * nel];
                w2[i] = in[2 * NN + (size_t)i * nel];
            }
        }
#pragma unroll
        for (int i = 0; i < K; ++i) {
            d0[i] += cf * v0[i];
            d1[i] += cf * v1[i];
            d2[i] += cf * v2[i];
            if constexpr (kHoist) {
                v0[i] = w0[i];
                v1[i] = w1[i];
                v2[i] = w2[i];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < K; ++i) {
        comb.out[o + (size_t)i * nel] = d0[i];
        comb.out[NN + o + (size_t)i * nel] = d1[i];
        comb.out[2 * NN + o + (size_t)i * nel] = d2[i];
    }
}

__global__ void k_combine(const Comb comb, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double acc = 0.0;
    for (int t = 0; t < comb.n; ++t) acc += comb.coef[t] * comb.in[t][i];
    comb.out[i] = acc;
}

// ------------------------------------------- linear HDG residual kernel
// M^-1 L(Q, Qhat) = M^-1 [ (F_L(Q), grad v)_K - <Fhat_L . n, v>_dK ] with
// n . Fhat_L = F_L(Q) . n + tau (Q - Qhat) (eq. linear_hdgflux3).
template <int K>
__global__ __launch_bounds__(64 * K) void k_linres(const double *__restrict__ Q,
                                                   const double *__restrict__ qh,
                                                   const Geom g, const Batch bt,
                                                   double *__restrict__ out) {
    __shared__ double sV[2][K][K][64];     // V and phi_B p, for d/dy
    const int lane = threadIdx.x & 63;
    const int j = wave_id();
    int lb;
    const Member mb = load_member(bt, member_of<CV>(bt, blockIdx.x, lb));
    Q += mb.vo;
    qh += mb.to;
    out += mb.vo;
    const int e = lb * 64 + lane;
    const bool active = e < mb.nel;
    const Nbr nb = neighbours(active ? e : 0, mb.nx, mb.ny);
    const size_t nel = mb.nel, NN = (size_t)K * K * nel, TT = (size_t)3 * K * nel;
    const double phiB = g.phiB, tau = g.tau;
    double p[K], U[K], V[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const size_t o = (size_t)(j * K + i) * nel + nb.e;
        p[i] = Q[o]; U[i] = Q[NN + o]; V[i] = Q[2 * NN + o];
        sV[0][j][i][lane] = V[i];
        sV[1][j][i][lane] = phiB * p[i];
    }
    double o0[K], o1[K], o2[K];
#pragma unroll
    for (int a = 0; a < K; ++a) {
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int m = 0; m < K; ++m) {
            s0 += g.Dw[m * K + a] * U[m];
            s1 += g.Dw[m * K + a] * p[m];
        }
        o0[a] = mb.sx * s0;
        o1[a] = mb.sx * phiB * s1;
        o2[a] = 0.0;
    }
    // west face = x-face e, east face = x-face east(e); node j
    {
        const size_t ow = (size_t)j * nel + nb.e, oe = (size_t)j * nel + nb.east;
        // east: n = (1, 0)
        double f0 = U[K - 1] + tau * (p[K - 1] - qh[oe]);
        double f1 = phiB * p[K - 1] + tau * (U[K - 1] - qh[nel * K + oe]);
        double f2 = tau * (V[K - 1] - qh[2 * nel * K + oe]);
        const double se = mb.sx * g.winvk;
        o0[K - 1] -= se * f0; o1[K - 1] -= se * f1; o2[K - 1] -= se * f2;
        // west: n = (-1, 0)
        f0 = -U[0] + tau * (p[0] - qh[ow]);
        f1 = -phiB * p[0] + tau * (U[0] - qh[nel * K + ow]);
        f2 = tau * (V[0] - qh[2 * nel * K + ow]);
        const double sw = mb.sx * g.winv0;
        o0[0] -= sw * f0; o1[0] -= sw * f1; o2[0] -= sw * f2;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < K; ++i) {
        double s0 = 0.0, s2 = 0.0;
#pragma unroll
        for (int m = 0; m < K; ++m) {
            s0 += g.Dw[m * K + j] * sV[0][m][i][lane];
            s2 += g.Dw[m * K + j] * sV[1][m][i][lane];
        }
        o0[i] += mb.sy * s0;
        o2[i] += mb.sy * s2;
    }
    if (j == K - 1 || j == 0) {
        const bool north = (j == K - 1);
        const int face = north ? nb.north : nb.e;      // y-face index
        const double ny = north ? 1.0 : -1.0;
        const double sc = mb.sy * (north ? g.winvk : g.winv0);
        const double *qy = qh + TT;
#pragma unroll
        for (int i = 0; i < K; ++i) {
            const size_t o = (size_t)i * nel + face;
            const double f0 = ny * V[i] + tau * (p[i] - qy[o]);
            const double f1 = tau * (U[i] - qy[nel * K + o]);
            const double f2 = ny * phiB * p[i] + tau * (V[i] - qy[2 * nel * K + o]);
            o0[i] -= sc * f0; o1[i] -= sc * f1; o2[i] -= sc * f2;
        }
    }
    if (!active) return;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const size_t o = (size_t)(j * K + i) * nel + e;
        out[o] = o0[i];
        out[NN + o] = o1[i];
        out[2 * NN + o] = o2[i];
    }
}

// ---------------------------------------------------- trace kernels
// Face tiles: tiles [0, nb) hold x-faces, [nb, 2 nb) y-faces, 64 faces
// each; thread (face lane, node j).  Krylov kernels loop over tiles with a
// capped grid.
struct FaceIdx {
    int d, f;            // direction, face index (= its element)
    bool active;
};

__device__ __forceinline__ FaceIdx face_of_tile(int tile, int nel) {
    const int nb = (nel + 63) / 64;
    FaceIdx fi;
    fi.d = tile >= nb ? 1 : 0;
    const int b = tile - fi.d * nb;
    fi.f = b * 64 + (threadIdx.x & 63);
    fi.active = fi.f < nel;
    if (!fi.active) fi.f = 0;
    return fi;
}

// Stage-solve state of one member on the fixed launch schedule.  At the
// start of a stage solve (run by trace_rhs): no sweep yet, no inner solve
// active until the first refinement check opens one.
__device__ __forceinline__ void stage_begin_state(KrylovState *ks) {
    ks->stage_done = 0;
    ks->sweep = 0;
    ks->relres = 0.0;
    ks->conv = 1;
    ks->iters = 0;
    for (int i = 0; i < kMaxSweeps; ++i) ks->sweep_iters[i] = 0;
}

// After the last sweep (run by one block of the member in recover): if the
// solve never met refine_rtol, take the residual of the final
// trace_residual [partials [4][face blocks]]; record the outcome.  Called
// by every thread of the block.
__device__ void stage_finish_block(const Member &mb, const KrylovState *ks,
                                   const double *res_partials, int stride, StageStatus *out) {
    double relres = ks->relres;
    const int done = ks->stage_done;
    if (!done) {
        double nrm[2];
        reduce_partials<2>(res_partials + mb.bf, stride, mb.nbf, nrm);
        relres = nrm[1] > 0.0 ? sqrt(nrm[0] / nrm[1]) : sqrt(nrm[0]);
    }
    if (threadIdx.x == 0) {
        out->relres = relres;
        out->converged = done;
        out->sweeps = ks->sweep;
        int tot = 0;
        for (int i = 0; i < kMaxSweeps; ++i) {
            out->sweep_iters[i] = ks->sweep_iters[i];
            tot += out->sweep_iters[i];
        }
        out->iters_total = tot;
    }
}

// g = sum over the two elements of C_K Z_K = F_L(Z) . n_K + tau Z at the
// face node.  `begin` (fixed schedule only): the member's first block also
// resets its stage-solve state (stage_begin_state).  `x` (steps only): the
// trace guess of this stage solve by linear extrapolation in time from the
// last two solutions, x <- x + xc (x - xp), xp <- x (x holds the last
// stage's solution, xp the one before; elementwise, each value has one
// thread).  The guess is the solver's heuristic, not the method: it
// changes the iterations, not the converged result.
template <int K>
__global__ __launch_bounds__(64 * K) void k_trace_rhs(const double *__restrict__ Z,
                                                      const Geom g, const Batch bt,
                                                      double *__restrict__ gv,
                                                      KrylovState *begin,
                                                      double *__restrict__ x,
                                                      double *__restrict__ xp, double xc) {
    const int j = wave_id();
    // the member's blocks are [2 bv, 2 (bv + nbv)): x-face tiles, then y
    int lb;
    const int mi = member_of<CV>(bt, blockIdx.x >> 1, lb);
    const Member mb = load_member(bt, mi);
    if (begin != nullptr && lb == 0 && (blockIdx.x & 1) == 0 && threadIdx.x == 0)
        stage_begin_state(begin + mi);
    Z += mb.vo;
    gv += mb.to;
    FaceIdx fi = face_of_tile(blockIdx.x - 2 * mb.bv, mb.nel);
    // faces between the ghost elements of a bounded member stay zero
    if (dummy_face(fi.d, fi.f % mb.nx, fi.f / mb.nx, mb)) fi.active = false;
    const Nbr n = neighbours(fi.f, mb.nx, mb.ny);
    const size_t nel = mb.nel, NN = (size_t)K * K * nel, TT = (size_t)3 * K * nel;
    const double phiB = g.phiB, tau = g.tau;
    // plus side: element f (face is its west / south), minus side: west /
    // south neighbour (face is its east / north)
    int np, nm;
    double nx, ny;
    if (fi.d == 0) { np = j * K + 0; nm = j * K + K - 1; nx = 1.0; ny = 0.0; }
    else { np = 0 * K + j; nm = (K - 1) * K + j; nx = 0.0; ny = 1.0; }
    const int em = fi.d == 0 ? n.west : n.south;
    const size_t op = (size_t)np * nel + n.e, om = (size_t)nm * nel + em;
    const double pp = Z[op], Up = Z[NN + op], Vp = Z[2 * NN + op];
    const double pm = Z[om], Um = Z[NN + om], Vm = Z[2 * NN + om];
    // minus side outward normal (nx, ny), plus side (-nx, -ny)
    const double g0 = (Um * nx + Vm * ny + tau * pm) + (-(Up * nx + Vp * ny) + tau * pp);
    const double g1 = (nx * phiB * pm + tau * Um) + (-nx * phiB * pp + tau * Up);
    const double g2 = (ny * phiB * pm + tau * Vm) + (-ny * phiB * pp + tau * Vp);
    const size_t base = fi.d * TT + (size_t)j * nel + fi.f;
    if (fi.active) {
        gv[base] = g0;
        gv[base + nel * K] = g1;
        gv[base + 2 * nel * K] = g2;
    }
    if (x != nullptr && fi.active) {
        double xv[3], pv[3];
        const size_t ob = mb.to + base;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xv[c] = x[ob + c * nel * K];
            pv[c] = xp[ob + c * nel * K];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            x[ob + c * nel * K] = xv[c] + xc * (xv[c] - pv[c]);
            xp[ob + c * nel * K] = xv[c];
        }
    }
}

// ---------------------------------------------- MFMA trace row blocks
// y_f = sum over the 7 neighbour slots of M[slot] x_{slot face}, one output
// row block (3K rows) per face, as a dense contraction on the FP64 matrix
// cores (v_mfma_f64_16x16x4f64): rows = A (16-row blocks of the shared
// matrix, host-packed per lane), k = (slot, c', j') of the gathered traces,
// columns = 16 faces per wave.  Operand layout of the instruction: lane l
// holds A[l % 16][l / 16] and B[l / 16][l % 16]; accumulator element r of
// lane l is D[4 r + l / 16][l % 16] for FP64 (see MfmaT for FP32).
typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Matrix-core 16x16x4 step per element type.  A and B operand layouts are
// the same for FP64 and FP32; the accumulator rows differ: lane l, element
// r holds row 4 r + l/16 (FP64) or 4 (l/16) + r (FP32), column l % 16.
template <typename T> struct MfmaT;
template <> struct MfmaT<double> {
    typedef v4d v4;
    static __device__ __forceinline__ v4 mma(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <> struct MfmaT<float> {
    typedef v4f v4;
    static __device__ __forceinline__ v4 mma(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

template <int K> struct MF {
    static constexpr int B3 = 3 * K;
    static constexpr int B3P = (B3 + 3) / 4 * 4;   // slot k-range padded to 4
    static constexpr int KS = B3P / 4;             // k steps per slot
    static constexpr int NKK = 7 * KS;             // k steps
    static constexpr int NMB = (B3 + 15) / 16;     // 16-row blocks
};

// ------------------------------------------------- local solver kernels
// Z = A^-1 R and Q = Z - W Qhat_dK (eq. recover_volume_unknowns) for every
// element as matrix-core contractions: the shared matrix (A^-1, 3K^2 x 3K^2;
// W = A^-1 B, 3K^2 x 12K) is the A operand, host-packed per lane as
// frag[mb][kk][lane] = M[16 mb + lane % 16][4 kk + lane / 16] (zero past the
// matrix); the B operand holds one element per column, 16 elements per wave,
// 64 per block; k steps of 4 run over the matrix columns.
template <int NR, int NC> struct LocalMF {
    static constexpr int NMB = (NR + 15) / 16, KS = (NC + 3) / 4;
};

template <int K>
__global__ __launch_bounds__(256) void k_local_apply(const double *__restrict__ R,
                                                     const Batch bt, double *__restrict__ Z) {
    constexpr int NL = 3 * K * K;
    using LM = LocalMF<NL, NL>;
    int lb;
    const Member mb = load_member(bt, member_of<CV>(bt, blockIdx.x, lb));
    R += mb.vo;
    Z += mb.vo;
    const double *__restrict__ A = mb.Ainv;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, q = lane >> 4;
    const int e = lb * 64 + w * 16 + (lane & 15);
    const bool active = e < mb.nel;
    const size_t nel = mb.nel, ec = active ? e : 0;
    v4d acc[LM::NMB];
#pragma unroll
    for (int m = 0; m < LM::NMB; ++m) acc[m] = v4d{0, 0, 0, 0};
    // B of k step kk: row 4 kk + q of R at this lane's element; the next
    // step's B and A operands are loaded before this step's products
    double b = q < NL ? R[(size_t)q * nel + ec] : 0.0;
    double a[LM::NMB];
#pragma unroll
    for (int m = 0; m < LM::NMB; ++m) a[m] = A[(size_t)m * LM::KS * 64 + lane];
#pragma unroll 2
    for (int kk = 0; kk < LM::KS; ++kk) {
        const int rn = 4 * (kk + 1) + q;
        const bool more = kk + 1 < LM::KS;
        const double bn = (more && rn < NL) ? R[(size_t)rn * nel + ec] : 0.0;
        double an[LM::NMB];
#pragma unroll
        for (int m = 0; m < LM::NMB; ++m)
            an[m] = more ? A[((size_t)m * LM::KS + kk + 1) * 64 + lane] : 0.0;
#pragma unroll
        for (int m = 0; m < LM::NMB; ++m)
            acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], b, acc[m], 0, 0, 0);
        b = bn;
#pragma unroll
        for (int m = 0; m < LM::NMB; ++m) a[m] = an[m];
    }
    if (!active) return;
#pragma unroll
    for (int m = 0; m < LM::NMB; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * m + 4 * r + q;
            if (row < NL) Z[(size_t)row * nel + e] = acc[m][r];
        }
}

// Local trace t = (f 3 + c) K + j of the element's faces f = W (x-face e),
// E (x-face east(e)), S (y-face e), N (y-face north(e)).
template <int K>
__device__ __forceinline__ double local_trace(const double *__restrict__ qh, const Nbr &nb,
                                              int t, size_t nel) {
    constexpr int NT = 12 * K;
    if (t >= NT) return 0.0;
    const int f = t / (3 * K), cj = t - f * 3 * K;
    const int face = f == 1 ? nb.east : f == 3 ? nb.north : nb.e;
    return qh[(f >= 2 ? (size_t)3 * K * nel : 0) + (size_t)cj * nel + face];
}

// `fout` (fixed schedule only): the member's first block also records the
// outcome of its stage solve (stage_finish_block).
template <int K>
__global__ __launch_bounds__(256) void k_recover(const double *__restrict__ Z,
                                                 const double *__restrict__ qh,
                                                 const Batch bt, double *__restrict__ Q,
                                                 const KrylovState *fks, const double *fpart,
                                                 int fstride, StageStatus *fout) {
    constexpr int NL = 3 * K * K, NT = 12 * K;
    using LM = LocalMF<NL, NT>;
    int lb;
    const int mi = member_of<CV>(bt, blockIdx.x, lb);
    const Member mb = load_member(bt, mi);
    if (fout != nullptr && lb == 0) stage_finish_block(mb, fks + mi, fpart, fstride, fout + mi);
    Z += mb.vo;
    qh += mb.to;
    Q += mb.vo;
    const double *__restrict__ Wf = mb.W;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, q = lane >> 4;
    const int e = lb * 64 + w * 16 + (lane & 15);
    const bool active = e < mb.nel;
    const size_t nel = mb.nel;
    const Nbr nb = neighbours(active ? e : 0, mb.nx, mb.ny);
    v4d acc[LM::NMB];
#pragma unroll
    for (int m = 0; m < LM::NMB; ++m) acc[m] = v4d{0, 0, 0, 0};
    double b = local_trace<K>(qh, nb, q, nel);
    double a[LM::NMB];
#pragma unroll
    for (int m = 0; m < LM::NMB; ++m) a[m] = Wf[(size_t)m * LM::KS * 64 + lane];
#pragma unroll 2
    for (int kk = 0; kk < LM::KS; ++kk) {
        const bool more = kk + 1 < LM::KS;
        const double bn = more ? local_trace<K>(qh, nb, 4 * (kk + 1) + q, nel) : 0.0;
        double an[LM::NMB];
#pragma unroll
        for (int m = 0; m < LM::NMB; ++m)
            an[m] = more ? Wf[((size_t)m * LM::KS + kk + 1) * 64 + lane] : 0.0;
#pragma unroll
        for (int m = 0; m < LM::NMB; ++m)
            acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m], b, acc[m], 0, 0, 0);
        b = bn;
#pragma unroll
        for (int m = 0; m < LM::NMB; ++m) a[m] = an[m];
    }
    if (!active) return;
#pragma unroll
    for (int m = 0; m < LM::NMB; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * m + 4 * r + q;
            if (row < NL) {
                const size_t o = (size_t)row * nel + e;
                Q[o] = Z[o] - acc[m][r];
            }
        }
}

// The same two contractions with the shared matrix staged in LDS once per
// block (its fragments are otherwise read from L2 by every wave) and every
// global load issued up front: the matrix fragments, this lane's B column
// for all k steps, and (recover) the Z values of its epilogue.  For the
// degrees whose matrix fits in 64 KB.
template <int NR, int NC> struct LocalLds {
    using LM = LocalMF<NR, NC>;
    static constexpr int NA = LM::NMB * LM::KS * 64;   // doubles of packed fragments
    static constexpr bool value = NA * 8 <= 64 * 1024;
    static constexpr int PER = (NA + 255) / 256;       // per thread of a 256-thread block
};

// Fragment loads of the packed matrix (A operand), to LDS after the caller
// has issued its other loads.
template <int NA, int PER> struct MatStage {
    double v[PER];
    __device__ __forceinline__ void load(const double *__restrict__ A) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = threadIdx.x + 256 * u;
            v[u] = A[i < NA ? i : 0];   // unconditional (see EarlyPartials)
        }
    }
    __device__ __forceinline__ void store(double *sA) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = threadIdx.x + 256 * u;
            if (i < NA) sA[i] = v[u];
        }
    }
};

template <int K>
__global__ __launch_bounds__(256, 3) void k_local_apply_lds(const double *__restrict__ R,
                                                         const Batch bt, double *__restrict__ Z) {
    constexpr int NL = 3 * K * K;
    using LL = LocalLds<NL, NL>;
    using LM = typename LL::LM;
    __shared__ double sA[LL::NA];
    int lb;
    const Member mb = load_member(bt, member_of<CV>(bt, blockIdx.x, lb));
    R += mb.vo;
    Z += mb.vo;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, q = lane >> 4;
    const int e = lb * 64 + w * 16 + (lane & 15);
    const bool active = e < mb.nel;
    const size_t nel = mb.nel, ec = active ? e : 0;
    MatStage<LL::NA, LL::PER> ms;
    ms.load(mb.Ainv);
    // B of k step kk: row 4 kk + q of R at this lane's element
    double b[LM::KS];
#pragma unroll
    for (int kk = 0; kk < LM::KS; ++kk) {
        const int row = 4 * kk + q;
        b[kk] = R[(size_t)(row < NL ? row : 0) * nel + ec];
    }
    ms.store(sA);
    lds_barrier();
    v4d acc[LM::NMB];
#pragma unroll
    for (int m = 0; m < LM::NMB; ++m) acc[m] = v4d{0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < LM::KS; ++kk) {
        const double bk = 4 * kk + q < NL ? b[kk] : 0.0;
#pragma unroll
        for (int m = 0; m < LM::NMB; ++m)
            acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(sA[(m * LM::KS + kk) * 64 + lane], bk,
                                                          acc[m], 0, 0, 0);
    }
    if (!active) return;
#pragma unroll
    for (int m = 0; m < LM::NMB; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * m + 4 * r + q;
            if (row < NL) Z[(size_t)row * nel + e] = acc[m][r];
        }
}

template <int K>
__global__ __launch_bounds__(256) void k_recover_lds(const double *__restrict__ Z,
                                                     const double *__restrict__ qh,
                                                     const Batch bt, double *__restrict__ Q,
                                                     const KrylovState *fks, const double *fpart,
                                                     int fstride, StageStatus *fout) {
    constexpr int NL = 3 * K * K, NT = 12 * K;
    using LL = LocalLds<NL, NT>;
    using LM = typename LL::LM;
    __shared__ double sA[LL::NA];
    int lb;
    const int mi = member_of<CV>(bt, blockIdx.x, lb);
    const Member mb = load_member(bt, mi);
    if (fout != nullptr && lb == 0) stage_finish_block(mb, fks + mi, fpart, fstride, fout + mi);
    Z += mb.vo;
    qh += mb.to;
    Q += mb.vo;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, q = lane >> 4;
    const int e = lb * 64 + w * 16 + (lane & 15);
    const bool active = e < mb.nel;
    const size_t nel = mb.nel, ec = active ? e : 0;
    const Nbr nb = neighbours((int)ec, mb.nx, mb.ny);
    MatStage<LL::NA, LL::PER> ms;
    ms.load(mb.W);
    // B of k step kk: local trace 4 kk + q of this lane's element
    double b[LM::KS];
#pragma unroll
    for (int kk = 0; kk < LM::KS; ++kk) {
        const int t = 4 * kk + q < NT ? 4 * kk + q : 0;
        const int f = t / (3 * K), cj = t - f * 3 * K;
        const int face = f == 1 ? nb.east : f == 3 ? nb.north : nb.e;
        b[kk] = qh[(f >= 2 ? (size_t)3 * K * nel : 0) + (size_t)cj * nel + face];
    }
    ms.store(sA);
    // the epilogue's Z values, in flight during the contraction
    double z[LM::NMB][4];
#pragma unroll
    for (int m = 0; m < LM::NMB; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * m + 4 * r + q;
            z[m][r] = Z[(size_t)(row < NL ? row : 0) * nel + ec];
        }
    lds_barrier();
    v4d acc[LM::NMB];
#pragma unroll
    for (int m = 0; m < LM::NMB; ++m) acc[m] = v4d{0, 0, 0, 0};
#pragma unroll
    for (int kk = 0; kk < LM::KS; ++kk) {
        const double bk = 4 * kk + q < NT ? b[kk] : 0.0;
#pragma unroll
        for (int m = 0; m < LM::NMB; ++m)
            acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(sA[(m * LM::KS + kk) * 64 + lane], bk,
                                                          acc[m], 0, 0, 0);
    }
    if (!active) return;
#pragma unroll
    for (int m = 0; m < LM::NMB; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * m + 4 * r + q;
            if (row < NL) Q[(size_t)row * nel + e] = z[m][r] - acc[m][r];
        }
}

// ----------------------- reduced-precision local solve, defect corrected
// Q = A^-1 R' per element, R' = R - B Qhat (recovery, eq.
// recover_volume_unknowns; Qhat = nullptr: Z = A^-1 R, the condensation of
// eq. linearizedHDGsystem_schur), with the dense contraction on the FP32
// (16x16x4) or BF16 (16x16x32, FP32 accumulation) matrix cores and NDC
// defect-correction sweeps
//   Q <- Q + A_lp^-1 (R' - A Q)
// whose residual R' - A Q = R' - Q + c Lq Q is formed in FP64, matrix free,
// from the local operator of the stage system (Sec. 5, eq.
// linearizedHDGsystem: A = I - c M^-1 dL/dQ, B = -c M^-1 dL/dQhat with the
// hybridized flux of eq. linear_hdgflux3, c = dt a~_ii).  Each sweep
// multiplies the error by I - A_lp^-1 A, whose norm is about the rounding
// unit of A_lp^-1 times the condition of A (about 50 for these operators:
// 2e-7 in FP32, 2e-2 in BF16), so the iterate reaches FP64 accuracy in one
// sweep from FP32 and to about 2e-8 relative in two from BF16.  The HBM
// traffic is that of one FP64 solve (R and Qhat read once, Q written once);
// the iterate stays in LDS in FP64.
//
// Roles in a block of EB elements (EB / 16 waves of 64 lanes):
//   contraction: wave w, lane l -> element 16 w + l % 16; the B operand of
//     k step kk holds rows KW kk + VPL (l / 16) + v (v < VPL = KW / 4) and
//     the accumulator rows 16 mb + 4 (l / 16) + r of that element (the lane
//     layouts of both instruction shapes, checked on the device);
//   residual: thread t -> element t % EB, rows t / EB + 4 i.
template <typename LP> struct LpMfma;
template <> struct LpMfma<float> {
    static constexpr int KW = 4;
    typedef float operand;
    static __device__ __forceinline__ v4f mma(operand a, operand b, v4f c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ operand load_a(const void *frags, size_t idx) {
        return ((const float *)frags)[idx];
    }
    template <typename F> static __device__ __forceinline__ operand make_b(F f) {
        return (float)f(0);
    }
};
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
template <> struct LpMfma<__bf16> {
    static constexpr int KW = 32;
    typedef bf16x8 operand;
    static __device__ __forceinline__ v4f mma(operand a, operand b, v4f c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ operand load_a(const void *frags, size_t idx) {
        return ((const bf16x8 *)frags)[idx];
    }
    template <typename F> static __device__ __forceinline__ operand make_b(F f) {
        operand b;
#pragma unroll
        for (int v = 0; v < 8; ++v) b[v] = (__bf16)(float)f(v);
        return b;
    }
};

template <int K, typename LP> struct LocalLp {
    static constexpr int NL = 3 * K * K;
    static constexpr int KW = LpMfma<LP>::KW, VPL = KW / 4;
    static constexpr int NMB = (NL + 15) / 16;          // accumulator row blocks
    static constexpr int KS = (NL + KW - 1) / KW;       // k steps
    static constexpr int NLK = KS * KW;                 // padded k range
    static constexpr int EB = K <= 4 ? 64 : K <= 5 ? 32 : 16;   // elements per block
    static constexpr int SPLIT = 64 / EB;               // blocks per 64-element volume block
    static constexpr int THREADS = 4 * EB;
};

template <int K, typename LP, int NDC>
__global__ __launch_bounds__((LocalLp<K, LP>::THREADS)) void k_local_lp(
    const double *__restrict__ R, const double *__restrict__ qh, const Geom g, const Batch bt,
    double aii, double *__restrict__ out,
    const KrylovState *fks, const double *fpart, int fstride, StageStatus *fout) {
    using L = LocalLp<K, LP>;
    using M = LpMfma<LP>;
    constexpr int NL = L::NL, EB = L::EB, KW = L::KW, VPL = L::VPL, NMB = L::NMB, KS = L::KS;
    constexpr int NLK = L::NLK, TH = L::THREADS;
    __shared__ double sQ[NMB * 16][EB];       // the FP64 iterate, [row][element]
    __shared__ double sP[NL][EB];             // R' = R - B Qhat in FP64
    __shared__ LP sR[NLK][EB];                // the residual as B operand
    __shared__ double sD[K * K];              // the weak derivative weights Dw
    int lb;
    const int mi = member_of<CV>(bt, blockIdx.x / L::SPLIT, lb);
    const Member mb = load_member(bt, mi);
    if (fout != nullptr && lb == 0 && blockIdx.x % L::SPLIT == 0)
        stage_finish_block(mb, fks + mi, fpart, fstride, fout + mi);
    const size_t nel = mb.nel;
    R += mb.vo;
    out += mb.vo;
    if (qh != nullptr) qh += mb.to;
    const void *frags = mb.Alp;
    const int e0 = lb * 64 + (blockIdx.x % L::SPLIT) * EB;   // first element of the block
    const double c = mb.dt * aii, tau = g.tau, phiB = g.phiB;
    const double sw = mb.sx * g.winv0, se = mb.sx * g.winvk;
    const double ss = mb.sy * g.winv0, sn = mb.sy * g.winvk;
    // contraction role
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, q4 = lane >> 4;
    const int ce = w * 16 + (lane & 15);                     // element within the block
    const bool cact = e0 + ce < mb.nel;
    // residual role
    const int re = threadIdx.x % EB, rg = threadIdx.x / EB;
    const bool ract = e0 + re < mb.nel;
    const Nbr rnb = neighbours(ract ? e0 + re : 0, mb.nx, mb.ny);

    // R' at local row t of the element with neighbour set nb: R plus the
    // lift c tau s_f Qhat of each face the node lies on
    auto rhs = [&](const Nbr &nb, int t) -> double {
        double r = R[(size_t)t * nel + nb.e];
        if (qh == nullptr) return r;
        const int comp = t / (K * K), ij = t - comp * K * K, j = ij / K, i = ij - j * K;
        const size_t TT = (size_t)3 * K * nel, cb = (size_t)comp * K * nel;
        double lift = 0.0;
        if (i == 0) lift += sw * qh[cb + (size_t)j * nel + nb.e];
        if (i == K - 1) lift += se * qh[cb + (size_t)j * nel + nb.east];
        if (j == 0) lift += ss * qh[TT + cb + (size_t)i * nel + nb.e];
        if (j == K - 1) lift += sn * qh[TT + cb + (size_t)i * nel + nb.north];
        return r + c * tau * lift;
    };

    // Dw is indexed by lane-dependent rows in the residual: LDS, not the
    // kernel-argument segment
    for (int i = threadIdx.x; i < K * K; i += TH) sD[i] = g.Dw[i];
    // R' of the block's elements into LDS: thread (re, rg) loads rows rg,
    // rg + 4, ... of element re (consecutive threads, consecutive elements:
    // coalesced), eight rows' loads in flight at a time
    {
        constexpr int PER = (NL + 3) / 4, CH = 8;
#pragma unroll 1
        for (int i0 = 0; i0 < PER; i0 += CH) {
            double v[CH];
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int t = rg + 4 * (i0 + u);
                v[u] = (t < NL && ract) ? rhs(rnb, t) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < CH; ++u) {
                const int t = rg + 4 * (i0 + u);
                if (t < NL) sP[t][re] = v[u];
            }
        }
    }
    __syncthreads();
    // first solve: Q = A_lp^-1 R'
    v4f acc[NMB];
#pragma unroll
    for (int m = 0; m < NMB; ++m) acc[m] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
    for (int kk = 0; kk < KS; ++kk) {
        const typename M::operand b = M::make_b([&](int v) {
            const int row = KW * kk + VPL * q4 + v;
            return row < NL ? sP[row][ce] : 0.0;
        });
#pragma unroll
        for (int m = 0; m < NMB; ++m)
            acc[m] = M::mma(M::load_a(frags, ((size_t)m * KS + kk) * 64 + lane), b, acc[m]);
    }
#pragma unroll
    for (int m = 0; m < NMB; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) sQ[16 * m + 4 * q4 + r][ce] = (double)acc[m][r];
    // rows of the padded k range past NL stay zero
    for (int i = threadIdx.x; i < (NLK - NL) * EB; i += TH) sR[NL + i / EB][i % EB] = LP(0.f);
    __syncthreads();

#pragma unroll 1
    for (int sweep = 0; sweep < NDC; ++sweep) {
        // residual R' - Q + c Lq Q of this thread's rows, in FP64
#pragma unroll 1
        for (int t = rg; t < NL; t += 4) {
            const int comp = t / (K * K), ij = t - comp * K * K, j = ij / K, i = ij - j * K;
            const double *Qp = &sQ[0][re], *QU = &sQ[K * K][re], *QV = &sQ[2 * K * K][re];
            auto at = [&](const double *b, int ii, int jj) { return b[(jj * K + ii) * EB]; };
            double lq = 0.0;
            if (comp == 0) {
                double sx_ = 0.0, sy_ = 0.0;
#pragma unroll
                for (int m = 0; m < K; ++m) {
                    sx_ += sD[m * K + i] * at(QU, m, j);
                    sy_ += sD[m * K + j] * at(QV, i, m);
                }
                lq = mb.sx * sx_ + mb.sy * sy_;
                const double p = at(Qp, i, j), U = at(QU, i, j), V = at(QV, i, j);
                if (i == 0) lq += sw * U - sw * tau * p;
                if (i == K - 1) lq += -se * U - se * tau * p;
                if (j == 0) lq += ss * V - ss * tau * p;
                if (j == K - 1) lq += -sn * V - sn * tau * p;
            } else if (comp == 1) {
                double sx_ = 0.0;
#pragma unroll
                for (int m = 0; m < K; ++m) sx_ += sD[m * K + i] * at(Qp, m, j);
                lq = mb.sx * phiB * sx_;
                const double p = at(Qp, i, j), U = at(QU, i, j);
                if (i == 0) lq += sw * phiB * p - sw * tau * U;
                if (i == K - 1) lq += -se * phiB * p - se * tau * U;
                if (j == 0) lq += -ss * tau * U;
                if (j == K - 1) lq += -sn * tau * U;
            } else {
                double sy_ = 0.0;
#pragma unroll
                for (int m = 0; m < K; ++m) sy_ += sD[m * K + j] * at(Qp, i, m);
                lq = mb.sy * phiB * sy_;
                const double p = at(Qp, i, j), V = at(QV, i, j);
                if (i == 0) lq += -sw * tau * V;
                if (i == K - 1) lq += -se * tau * V;
                if (j == 0) lq += ss * phiB * p - ss * tau * V;
                if (j == K - 1) lq += -sn * phiB * p - sn * tau * V;
            }
            const double res = ract ? sP[t][re] - sQ[t][re] + c * lq : 0.0;
            sR[t][re] = LP((float)res);
        }
        __syncthreads();
        // correction d = A_lp^-1 (R' - A Q), added to the iterate in FP64
#pragma unroll
        for (int m = 0; m < NMB; ++m) acc[m] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
        for (int kk = 0; kk < KS; ++kk) {
            const typename M::operand b =
                M::make_b([&](int v) { return (float)sR[KW * kk + VPL * q4 + v][ce]; });
#pragma unroll
            for (int m = 0; m < NMB; ++m)
                acc[m] = M::mma(M::load_a(frags, ((size_t)m * KS + kk) * 64 + lane), b, acc[m]);
        }
        if (sweep + 1 < NDC) {
#pragma unroll
            for (int m = 0; m < NMB; ++m)
#pragma unroll
                for (int r = 0; r < 4; ++r) sQ[16 * m + 4 * q4 + r][ce] += (double)acc[m][r];
            __syncthreads();
        }
    }
    if (!cact) return;
#pragma unroll
    for (int m = 0; m < NMB; ++m)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * m + 4 * q4 + r;
            if (row < NL) out[(size_t)row * nel + e0 + ce] = sQ[row][ce] + (double)acc[m][r];
        }
}

// Workgroups per CU the matrix-core kernels are compiled for (8 waves
// each): the register budget that keeps them free of scratch spills.
template <int K> struct MFOcc {
    static constexpr int value = K <= 5 ? 2 : 1;
};
// The bounded-mesh variants (BND) hold the boundary-row state on top: at
// K <= 5 they are held to 128 VGPRs (four waves per SIMD) where that costs
// no spill, so that they keep the periodic kernels' two blocks per CU (K1f;
// the FP32 K1 and refinement check).
template <int K, typename T, bool BND, bool K1F> struct FaceOcc {
    static constexpr int value =
        (BND && K <= 5 && (K1F || sizeof(T) == 4)) ? 4 : MFOcc<K>::value;
};
// The residual kernel at K <= 5 must keep two 512-thread blocks per CU
// (at most 128 VGPRs: four waves per SIMD).
template <int K> struct ResidOcc {
    static constexpr int value = K <= 5 ? 4 : 1;
};

// Packed A fragments: frag[dir][mb][kk][lane] (see element-side packing).
__device__ __forceinline__ size_t frag_off(int d, int mb, int kk, int lane, int NMB, int NKK) {
    return (((size_t)d * NMB + mb) * NKK + kk) * 64 + lane;
}

// Tiles of 64 elements; block b walks tiles so that the blocks resident on
// one XCD (b mod 8, as the dispatcher deals workgroups round robin over
// the eight XCDs) cover one contiguous band of the mesh and share its
// neighbour faces in their L2.
struct TileWalk {
    int first, step, end;
};

// Block `lb` of the G blocks of one member (G a multiple of 8 and the
// member's first block a multiple of 8 keep lb mod 8 = the block's XCD).
__device__ __forceinline__ TileWalk tile_walk(int lb, int G, int ntiles) {
    if (G % 8 != 0 || G < 8) return TileWalk{lb, G, ntiles};
    const int xcd = lb % 8, local = lb / 8, per = G / 8;
    const int chunk = (ntiles + 7) / 8;
    const int begin = xcd * chunk;
    const int end = min(ntiles, begin + chunk);
    return TileWalk{begin + local, per, end};
}

template <typename T> struct FragMatsT {
    const T *A0, *A1;        // packed fragments of one or two matrices
};
typedef FragMatsT<double> FragMats;

// ------------------------------------------------------------ face blocks
// A face kernel runs blocks of 8 waves over 64-element tiles: wave w takes
// face set w / 4 (0: the x-faces, 1: the y-faces of the elements) of the 16
// elements in row w % 4 of the tile, so every wave runs one accumulation
// chain and the two sets proceed in parallel.
constexpr int kFaceThreads = 512;
constexpr int kTX = 16, kTY = 4;     // element tile (below)

struct WaveFaces {
    int set, sub;            // face set (wave-uniform), tile row
    int e;                   // element (= face index) of this lane
    bool active;             // e < nel, and an unknown of a bounded mesh
    int bt;                  // boundary side of this lane's face (bounded mesh): 0 W, 1 E,
                             // 2 S, 3 N, -1 none
    const void *dfr;         // boundary-row corrections of the wave's operator, or nullptr
};


// Boundary-row corrections of the preconditioned row blocks in precision T.
template <typename T> __device__ __forceinline__ const void *delta_hat(const Member &g);
template <> __device__ __forceinline__ const void *delta_hat<double>(const Member &g) {
    return g.dGh;
}
template <> __device__ __forceinline__ const void *delta_hat<float>(const Member &g) {
    return g.dGhf;
}

// Tiles of 16 x 4 elements cover the mesh (partial tiles at the high
// edges, their lanes past the mesh inactive).
__device__ __forceinline__ int tiles_per_row(const Member &g) { return (g.nx + kTX - 1) / kTX; }

// BND: the batch has a bounded member (mask its faces between ghosts, mark
// its boundary faces); false compiles the periodic mapping alone.
template <bool BND>
__device__ __forceinline__ WaveFaces wave_faces(int tile, const Member &g,
                                                const void *dfr = nullptr) {
    WaveFaces wf;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    wf.set = w >> 2;
    wf.sub = w & 3;
    const int tpr = tiles_per_row(g);
    const int ex = (tile % tpr) * kTX + (lane & 15), ey = (tile / tpr) * kTY + wf.sub;
    wf.active = ex < g.nx && ey < g.ny;
    wf.bt = -1;
    wf.dfr = nullptr;
    if constexpr (BND) {
        wf.active = wf.active && !dummy_face(wf.set, ex, ey, g);
        wf.bt = wf.active ? boundary_side(wf.set, ex, ey, g) : -1;
        wf.dfr = g.bx > 0 ? dfr : nullptr;
    }
    wf.e = wf.active ? ey * g.nx + ex : 0;
    return wf;
}

// Trace offset of accumulator element (mb, r) of this lane: row 16 mb +
// row(lane, r) of the row block of face (set, e); valid if that row < 3K.
// Callers load x[valid ? off : 0] and use the value only where valid: a
// load under a divergent branch would be followed by a write of the
// default value to the same register, which waits for every load in
// flight.
template <int K, typename T>
__device__ __forceinline__ uint32_t own_off(const WaveFaces &wf, int mb, int r, uint32_t nel,
                                            bool &valid) {
    const int row = 16 * mb + MfmaT<T>::row(threadIdx.x & 63, r);
    valid = row < MF<K>::B3 && wf.active;
    return (uint32_t)wf.set * MF<K>::B3 * nel + (uint32_t)row * nel + wf.e;
}

// A operands of one slot for this wave's face set, all row blocks and k
// steps, for NM matrices.
template <int K, int NM, typename T> struct FragSlot {
    T v[NM][MF<K>::NMB][MF<K>::KS];
};

template <int K, int NM, typename T>
__device__ __forceinline__ void load_frags(const T *__restrict__ const *frags, int set, int s,
                                           FragSlot<K, NM, T> &b) {
    constexpr int KS = MF<K>::KS, NKK = MF<K>::NKK, NMB = MF<K>::NMB;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int m = 0; m < NM; ++m)
#pragma unroll
        for (int mb = 0; mb < NMB; ++mb)
#pragma unroll
            for (int u = 0; u < KS; ++u)
                b.v[m][mb][u] = frags[m][frag_off(set, mb, s * KS + u, lane, NMB, NKK)];
}

// Double buffer the A operands of the next slot when they fit in 24 VGPRs.
template <int K, int NM, typename T> struct FragPrefetch {
    static constexpr bool value = NM * MF<K>::NMB * MF<K>::KS * (int)sizeof(T) / 4 <= 24;
};

template <int K, int NM, typename T>
__device__ __forceinline__ void zero_acc(typename MfmaT<T>::v4 (&acc)[NM][MF<K>::NMB]) {
#pragma unroll
    for (int m = 0; m < NM; ++m)
#pragma unroll
        for (int mb = 0; mb < MF<K>::NMB; ++mb) acc[m][mb] = typename MfmaT<T>::v4{0, 0, 0, 0};
}

// ------------------------------------- LDS-staged tiles of 16 x 4 elements
// A workgroup stages once into LDS every trace face its tile's row blocks
// read (the union over the 7 slots of the x- and y-faces of its 64
// elements: 18 x 5 x-faces and 17 x 6 y-faces), with coalesced loads of
// whole face rows, and the matrix cores read their B operands from LDS.
// Each trace value then crosses L2 about 1.5 times per launch instead of 7.
// Tiles past the mesh edge are partial: their positions wrap periodically
// and their lanes outside the mesh store nothing.

template <int K> struct Tile {
    static constexpr int B3 = 3 * K;
    static constexpr int XR = kTY + 1, XC = kTX + 2;   // x-faces: rows ey0-1.., cols ex0-1..
    static constexpr int YR = kTY + 2, YC = kTX + 1;   // y-faces
    static constexpr int NX = XR * XC, NY = YR * YC, NF = NX + NY;
};

// LDS row stride of a staged tile of T values.  FP32: 16 words past a
// multiple of the 64 banks, so the four rows that one matrix-core B read
// spans (lane groups l / 16) fall into disjoint banks.  FP64 keeps the
// dense stride (the padded one costs its Krylov kernels their occupancy).
template <int K, typename T> struct TileRow {
    static constexpr int NF = Tile<K>::NF;
    static constexpr int stride = sizeof(T) == 4 ? NF + (80 - NF % 64) % 64 : NF;
    // LDS index of staged value v = cj NF + f
    static __device__ __forceinline__ int lds(int v) { return v + (v / NF) * (stride - NF); }
};

// Staged face f of the tile with corner (ex0, ey0) -> direction, global face
// (element) index, and whether the tile owns it (it is a face of one of the
// tile's own elements).
__device__ __forceinline__ void staged_face(int f, int ex0, int ey0, int nx, int ny, int NX,
                                            int XC, int YC, int &dir, int &elem, bool &own) {
    int r, c;
    if (f < NX) { dir = 0; r = f / XC; c = f % XC; }
    else { dir = 1; r = (f - NX) / YC; c = (f - NX) % YC; }
    // positions past the mesh wrap periodically (a tile wider than the mesh
    // stages a face more than once); only positions of the tile's own
    // elements inside the mesh own their face
    const int gx = ex0 - 1 + c, gy = ey0 - 1 + r;
    int ex = gx < 0 ? gx + nx : gx, ey = gy < 0 ? gy + ny : gy;
    if (ex >= nx) ex = ex - nx < nx ? ex - nx : ex % nx;   // the modulo only on meshes
    if (ey >= ny) ey = ey - ny < ny ? ey - ny : ey % ny;   // narrower than a tile
    elem = ey * nx + ex;
    own = r >= 1 && r <= kTY && c >= 1 && c <= kTX && gx < nx && gy < ny;
}

// LDS face index of slot `s` of face set `set` for tile element (lx, ly).
__device__ __forceinline__ int slot_lds(int set, int s, int lx, int ly, int NX, int XC, int YC) {
    // (dir, dx, dy) of each slot, from the neighbour lists of the row blocks
    int d = 0, dx = 0, dy = 0;
    if (set == 0) {
        switch (s) {
            case 0: d = 0; dx = 0; dy = 0; break;
            case 1: d = 0; dx = 1; dy = 0; break;
            case 2: d = 1; dx = 0; dy = 0; break;
            case 3: d = 1; dx = 0; dy = 1; break;
            case 4: d = 0; dx = -1; dy = 0; break;
            case 5: d = 1; dx = -1; dy = 0; break;
            default: d = 1; dx = -1; dy = 1; break;
        }
    } else {
        switch (s) {
            case 0: d = 1; dx = 0; dy = 0; break;
            case 1: d = 0; dx = 0; dy = 0; break;
            case 2: d = 0; dx = 1; dy = 0; break;
            case 3: d = 1; dx = 0; dy = 1; break;
            case 4: d = 1; dx = 0; dy = -1; break;
            case 5: d = 0; dx = 0; dy = -1; break;
            default: d = 0; dx = 1; dy = -1; break;
        }
    }
    return d == 0 ? (ly + dy + 1) * XC + (lx + dx + 1)
                  : NX + (ly + dy + 1) * YC + (lx + dx + 1);
}

// comb(raw, off, own), or comb(raw, oraw, off, own, li) with NO own-face
// sources (li: the value's LDS index in the staged tile).
template <int NO, typename T, int NA, typename Comb>
__device__ __forceinline__ T apply_comb(Comb &comb, const T (&a)[NA], const T (&o)[NO > 0 ? NO : 1],
                                        uint32_t off, bool own, int li) {
    if constexpr (NO == 0) return comb(a, off, own);
    else return comb(a, o, off, own, li);
}

// Stage the tile: sB[cj stride + f] = comb(raw, o, own) for every staged face
// f and row cj (c' K + j'), where raw holds the NA source arrays at trace
// offset o; comb may store the value at o when the tile owns the face.
// With NO > 0, the NO arrays osrc are also loaded at the faces the tile
// owns (zero elsewhere) and handed to comb.  All loads of a chunk of up to
// 8 values per thread are issued before any is used.
template <int K, typename T, int NA, int NO, typename Comb>
__device__ __forceinline__ void stage_tile(int tile, const Member &g, T *sB,
                                           const T *__restrict__ const (&src)[NA],
                                           const T *const *osrc, Comb comb) {
    using TL = Tile<K>;
    constexpr int NV = TL::B3 * TL::NF, PER = (NV + kFaceThreads - 1) / kFaceThreads;
    constexpr int CH = PER < 8 ? PER : 8;
    const int tpr = tiles_per_row(g);
    const int ex0 = (tile % tpr) * kTX, ey0 = (tile / tpr) * kTY;
    const uint32_t nel = g.nel, TT = TL::B3 * nel;
#pragma unroll
    for (int i0 = 0; i0 < PER; i0 += CH) {
        uint32_t off[CH];
        bool own[CH], ok[CH];
        T raw[CH][NA], oraw[CH][NO > 0 ? NO : 1];
#pragma unroll
        for (int u = 0; u < CH; ++u) {
            const int v = threadIdx.x + kFaceThreads * (i0 + u);
            ok[u] = (i0 + u < PER) && v < NV;
            const int vv = ok[u] ? v : 0;
            const int cj = vv / TL::NF, fc = vv - cj * TL::NF;
            int dir, elem;
            staged_face(fc, ex0, ey0, g.nx, g.ny, TL::NX, TL::XC, TL::YC, dir, elem, own[u]);
            off[u] = (uint32_t)dir * TT + (uint32_t)cj * nel + (uint32_t)elem;
        }
#pragma unroll
        for (int u = 0; u < CH; ++u)
#pragma unroll
            for (int a = 0; a < NA; ++a) raw[u][a] = ok[u] ? src[a][off[u]] : T(0);
#pragma unroll
        for (int u = 0; u < CH; ++u)
#pragma unroll
            for (int b = 0; b < NO; ++b) oraw[u][b] = ok[u] && own[u] ? osrc[b][off[u]] : T(0);
#pragma unroll
        for (int u = 0; u < CH; ++u)
            if (ok[u]) {
                const int li = TileRow<K, T>::lds(threadIdx.x + kFaceThreads * (i0 + u));
                sB[li] = apply_comb<NO>(comb, raw[u], oraw[u], off[u], own[u], li);
            }
    }
}

// A tile's staging split in two: load() issues the loads of every value
// this thread stages (held in registers when there are at most 8 per
// thread), commit() combines them and writes LDS.  The FP32 Krylov kernels
// issue the first tile's loads before their partial-sum reduction, so the
// two memory round trips overlap (FP64 keeps the registers for occupancy).
// With more than 8 values per thread, commit() stages in chunks
// (stage_tile) and load() only records the tile.  NO > 0: own-face sources
// as in stage_tile.
template <int K, typename T, int NA, int NO = 0> struct StagedTile {
    using TL = Tile<K>;
    static constexpr int NV = TL::B3 * TL::NF;
    static constexpr int PER = (NV + kFaceThreads - 1) / kFaceThreads;
    static constexpr bool kHold = PER <= 8;
    static constexpr int H = kHold ? PER : 1;
    T raw[H][NA], oraw[H][NO > 0 ? NO : 1];
    uint32_t off[H];
    bool own[H], ok[H];
    int tile;
    const T *const *os;

    // dummy: every lane reads the member's first values instead (a load
    // that is issued but never committed costs one cache line per wave)
    __device__ __forceinline__ void load(int t, const Member &g,
                                         const T *__restrict__ const (&src)[NA],
                                         const T *const *osrc = nullptr, bool dummy = false) {
        tile = t;
        os = osrc;
        if constexpr (kHold) {
            const int tpr = tiles_per_row(g);
            const int ex0 = (t % tpr) * kTX, ey0 = (t / tpr) * kTY;
            const uint32_t nel = g.nel, TT = TL::B3 * nel;
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int v = threadIdx.x + kFaceThreads * u;
                ok[u] = v < NV;
                const int vv = ok[u] ? v : 0;
                const int cj = vv / TL::NF, fc = vv - cj * TL::NF;
                int dir, elem;
                staged_face(fc, ex0, ey0, g.nx, g.ny, TL::NX, TL::XC, TL::YC, dir, elem, own[u]);
                off[u] = dummy ? 0u : (uint32_t)dir * TT + (uint32_t)cj * nel + (uint32_t)elem;
            }
            // every load is issued and nothing is selected here, so that no
            // wait lands in load() (see EarlyPartials): off[u] is a valid
            // face for every slot (commit() skips the slots past the tile),
            // and the own-face sources of other faces read the member's
            // first value (one cache line per wave; comb ignores them)
#pragma unroll
            for (int u = 0; u < PER; ++u)
#pragma unroll
                for (int a = 0; a < NA; ++a) raw[u][a] = src[a][off[u]];
#pragma unroll
            for (int u = 0; u < PER; ++u)
#pragma unroll
                for (int b = 0; b < NO; ++b) oraw[u][b] = osrc[b][ok[u] && own[u] ? off[u] : 0u];
        }
    }

    template <typename Comb>
    __device__ __forceinline__ void commit(const Member &g, const T *__restrict__ const (&src)[NA],
                                           T *sB, Comb comb) {
        if constexpr (kHold) {
#pragma unroll
            for (int u = 0; u < PER; ++u)
                if (ok[u]) {
                    const int li = TileRow<K, T>::lds(threadIdx.x + kFaceThreads * u);
                    sB[li] = apply_comb<NO>(comb, raw[u], oraw[u], off[u], own[u], li);
                }
        } else {
            stage_tile<K, T, NA, NO>(tile, g, sB, src, os, comb);
        }
    }
};

// This wave's row blocks from the staged tile: the matrix cores read the B
// operands from LDS, slot by slot; the A operands of slot s + 1 are loaded
// while slot s is computed.
template <int K, int NM, typename T>
__device__ __forceinline__ void tile_rows(const T *__restrict__ const *frags, const T *sB,
                                          const WaveFaces &wf,
                                          typename MfmaT<T>::v4 (&acc)[NM][MF<K>::NMB]) {
    using TL = Tile<K>;
    constexpr int B3 = TL::B3, NF = TileRow<K, T>::stride, KS = MF<K>::KS, NMB = MF<K>::NMB;
    constexpr bool PF = FragPrefetch<K, NM, T>::value;
    const int lane = threadIdx.x & 63, q = lane >> 4, lx = lane & 15;
    zero_acc<K, NM, T>(acc);
    FragSlot<K, NM, T> cur, nxt;
    if (PF) load_frags<K, NM, T>(frags, wf.set, 0, cur);
#pragma unroll
    for (int s = 0; s < 7; ++s) {
        if (PF) {
            if (s + 1 < 7) load_frags<K, NM, T>(frags, wf.set, s + 1, nxt);
        } else {
            load_frags<K, NM, T>(frags, wf.set, s, cur);
        }
        const int li = slot_lds(wf.set, s, lx, wf.sub, TL::NX, TL::XC, TL::YC);
#pragma unroll
        for (int u = 0; u < KS; ++u) {
            // rows past 3K meet zero columns of A: any finite staged value
            // serves, so the read is clamped instead of branched around
            const int cj = 4 * u + q;
            const T b = sB[(cj < B3 ? cj : B3 - 1) * NF + li];
#pragma unroll
            for (int m = 0; m < NM; ++m)
#pragma unroll
                for (int mb = 0; mb < NMB; ++mb)
                    acc[m][mb] = MfmaT<T>::mma(cur.v[m][mb][u], b, acc[m][mb]);
        }
        if (PF) cur = nxt;
    }
}

// Row-block slot of entry e of a boundary side's corrections (the real
// element's faces, the boundary face first; see Member): W and S sides, the
// real element is the face's plus element (slots of its west, east, south,
// north faces); E and N, its minus element.
__device__ __forceinline__ int side_slot(int side, int e) {
    switch (side) {
        case 0: return e;                       // W: x-face plus element
        case 1: return e == 0 ? 0 : 3 + e;      // E: 0, 4, 5, 6
        case 2: return e;                       // S: y-face plus element
        default: return e == 0 ? 0 : e == 3 ? 4 : 4 + e;   // N: 0, 5, 6, 4
    }
}

// Bounded mesh: a boundary row adds its side's corrections, each applied to
// the staged face of its slot for the lanes whose face is on that side (the
// B operand is zero for the other lanes): the self slot only with
// exact-solution data (NENT = 1), the real element's four faces with walls
// (NENT = 4).  The entries are unrolled so that the fragment loads of a
// side are in flight together (one round trip per side, not per entry).
template <int K, typename T, int NENT>
__device__ __forceinline__ void boundary_rows_n(const WaveFaces &wf, const T *sB,
                                                typename MfmaT<T>::v4 (&acc)[1][MF<K>::NMB]) {
    using TL = Tile<K>;
    constexpr int B3 = TL::B3, NF = TileRow<K, T>::stride, KS = MF<K>::KS, NMB = MF<K>::NMB;
    const int lane = threadIdx.x & 63, q = lane >> 4, lx = lane & 15;
    const T *dfr = (const T *)wf.dfr;
    for (int h = 0; h < 2; ++h) {
        const int side = 2 * wf.set + h;
        if (!__any(wf.bt == side)) continue;
#pragma unroll
        for (int e = 0; e < NENT; ++e) {
            const int li = slot_lds(wf.set, side_slot(side, e), lx, wf.sub, TL::NX, TL::XC,
                                    TL::YC);
#pragma unroll
            for (int u = 0; u < KS; ++u) {
                const int cj = 4 * u + q;
                const T bv = sB[(cj < B3 ? cj : B3 - 1) * NF + li];
                const T b = wf.bt == side ? bv : T(0);
#pragma unroll
                for (int mb = 0; mb < NMB; ++mb)
                    acc[0][mb] = MfmaT<T>::mma(dfr[frag_off(4 * side + e, mb, u, lane, NMB, KS)],
                                               b, acc[0][mb]);
            }
        }
    }
}

template <int K, typename T>
__device__ __forceinline__ void boundary_rows(const WaveFaces &wf, const T *sB, int nent,
                                              typename MfmaT<T>::v4 (&acc)[1][MF<K>::NMB]) {
    if (wf.dfr == nullptr) return;
    if (nent == 4) boundary_rows_n<K, T, 4>(wf, sB, acc);
    else boundary_rows_n<K, T, 1>(wf, sB, acc);
}

// LDS index of this lane's own face of its wave's set.
template <int K>
__device__ __forceinline__ int own_lds(const WaveFaces &wf) {
    using TL = Tile<K>;
    const int lx = threadIdx.x & 15;
    return wf.set == 0 ? (wf.sub + 1) * TL::XC + (lx + 1)
                       : TL::NX + (wf.sub + 1) * TL::YC + (lx + 1);
}

// Row blocks of this wave for one tile whose staging loads are in flight
// in st: commit the staging, then contract from LDS.
// `next` runs between the staging and the contraction: the FP32 kernels
// issue the next tile's loads there, into the registers commit() freed.
struct NoNext {
    __device__ __forceinline__ void operator()() const {}
};
template <int K, int NM, typename T, int NA, int NO, typename Comb, typename Next = NoNext>
__device__ __forceinline__ void face_rows(const T *__restrict__ const *frags,
                                          StagedTile<K, T, NA, NO> &st, const Member &g,
                                          const WaveFaces &wf, T *sB,
                                          const T *__restrict__ const (&src)[NA], Comb comb,
                                          typename MfmaT<T>::v4 (&acc)[NM][MF<K>::NMB],
                                          Next next = Next()) {
    lds_barrier();   // the previous tile's LDS reads are done
    st.commit(g, src, sB, comb);
    lds_barrier();
    next();
    tile_rows<K, NM, T>(frags, sB, wf, acc);
}

__device__ __forceinline__ int face_tiles(const Member &g) {
    return tiles_per_row(g) * ((g.ny + kTY - 1) / kTY);
}

// LDS of a staged tile.
template <int K, typename T> struct TileLds {
    static constexpr int n = MF<K>::B3 * TileRow<K, T>::stride;
};

// The matrix-core fragments (both face sets, NM matrices) are copied into
// LDS once per block when they fit beside the staged tile in 80 KB (K <= 5:
// two blocks of 8 waves per CU, the register limit, still fit), so the
// matrix-core loop reads its A operands from LDS instead of L2.
template <int K, typename T, int NM = 1> struct FragLds {
    static constexpr int n = 2 * MF<K>::NMB * MF<K>::NKK * 64;
    static constexpr bool value =
        (TileLds<K, T>::n + NM * n) * (int)sizeof(T) <= 80 * 1024;
    static constexpr int alloc = value ? NM * n : 1;
};

// stage_frags split in two: load() issues the fragment loads, store()
// writes LDS and returns the operand pointers.
template <int K, typename T, int NM = 1> struct FragStage {
    static constexpr int n = FragLds<K, T, NM>::n;
    static constexpr int PER = FragLds<K, T, NM>::value ? (n + kFaceThreads - 1) / kFaceThreads : 1;
    T v[NM][PER];
    const T *src[NM];
    __device__ __forceinline__ void load(const T *__restrict__ const *g) {
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            src[m] = g[m];
            if constexpr (FragLds<K, T, NM>::value) {
#pragma unroll
                for (int u = 0; u < PER; ++u) {
                    const int i = threadIdx.x + kFaceThreads * u;
                    const T x = g[m][i < n ? i : 0];   // unconditional (see EarlyPartials)
                    v[m][u] = i < n ? x : T(0);
                }
            }
        }
    }
    __device__ __forceinline__ void store(T *sA, const T **out) {
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            if constexpr (FragLds<K, T, NM>::value) {
#pragma unroll
                for (int u = 0; u < PER; ++u) {
                    const int i = threadIdx.x + kFaceThreads * u;
                    if (i < n) sA[m * n + i] = v[m][u];
                }
                out[m] = sA + m * n;   // read after the staging barrier of the first tile
            } else {
                out[m] = src[m];
            }
        }
    }
};

template <int K, typename T, int NM = 1>
__device__ __forceinline__ void stage_frags(const T *__restrict__ const *g, T *sA,
                                            const T **out) {
    if constexpr (FragLds<K, T, NM>::value) {
        constexpr int n = FragLds<K, T, NM>::n, PER = (n + kFaceThreads - 1) / kFaceThreads;
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            T v[PER];
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int i = threadIdx.x + kFaceThreads * u;
                v[u] = i < n ? g[m][i] : T(0);
            }
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int i = threadIdx.x + kFaceThreads * u;
                if (i < n) sA[m * n + i] = v[u];
            }
            out[m] = sA + m * n;   // read after the staging barrier of the first tile
        }
    } else {
#pragma unroll
        for (int m = 0; m < NM; ++m) out[m] = g[m];
    }
}

// FP64 residuals of the trace system: r = g - G x and rin = P^-1 r (the
// face's block-Jacobi inverse applied to r: ghat - Ghat x, with ghat =
// P^-1 g never stored), rin stored in the inner solve's precision;
// partials of ||r||^2, ||g||^2, ||P^-1 g||^2, ||rin||^2.  The accumulator of
// the G contraction already holds r in the B-operand layout of a further
// matrix-core step (FP64 element e4 of row block mb of lane l is row
// 16 mb + 4 e4 + l/16 of face l % 16: the B operand of k step 4 mb + e4), so
// P^-1 r and P^-1 g are two short contractions on the registers.  With rin
// == nullptr (a check of a finished solve) only ||r||^2 and ||g||^2 are
// formed.
template <int K, typename RT, bool BND>
__global__ __launch_bounds__(kFaceThreads, ResidOcc<K>::value) void k_trace_residual(
    const Batch bt, const double *__restrict__ x, const double *__restrict__ gv,
    RT *__restrict__ rin, double *partials, int stride, const KrylovState *skip) {
    using T = double;
    constexpr int NMB = MF<K>::NMB, B3 = 3 * K;
    arg_now(stride);
    arg_now(skip);
    int lb;
    const int mi = member_of<CF>(bt, blockIdx.x, lb);
    const Member mb = load_member(bt, mi);
    // the member's fields and the flag in one round trip
    const int done = skip ? skip[mi].stage_done : 0;
    arg_now(mb.to);
    arg_now(mb.bf);
    arg_now(mb.G);
    if (done) return;
    const bool want_rin = rin != nullptr;
    x += mb.to; gv += mb.to;
    if (want_rin) rin += mb.to;
    __shared__ double sB[TileLds<K, T>::n];
    __shared__ double sA[FragLds<K, T, 1>::alloc];
    const uint32_t nel = mb.nel;
    const double *gfr[1] = {mb.G};
    const double *fr[1];
    // the first tile's loads are issued with the operand loads (a block
    // without tiles loads tile 0 and never commits it)
    FragStage<K, T, 1> fs;
    fs.load(gfr);
    const double *src[1] = {x};
    const TileWalk tw = tile_walk(lb, mb.nbf, face_tiles(mb));
    StagedTile<K, T, 1> st;
    st.load(tw.first < tw.end ? tw.first : 0, mb, src);
    // P^-1 of this wave's face set as A fragments: pf[mo][kk] = P[16 mo +
    // l % 16][4 kk + l / 16], zero past 3K (P row-major, 3K x 3K)
    const int lane = threadIdx.x & 63;
    const double *P = ((threadIdx.x >> 6) >> 2) == 0 ? mb.Px : mb.Py;
    double pf[NMB][4 * NMB];
#pragma unroll
    for (int mo = 0; mo < NMB; ++mo)
#pragma unroll
        for (int kk = 0; kk < 4 * NMB; ++kk) {
            const int row = 16 * mo + (lane & 15), col = 4 * kk + (lane >> 4);
            const bool in = row < B3 && col < B3;
            const double pv = P[in ? row * B3 + col : 0];
            pf[mo][kk] = in ? pv : 0.0;
        }
    fs.store(sA, fr);
    double acc4[4] = {0.0, 0.0, 0.0, 0.0};
    {
        for (int tile = tw.first; tile < tw.end; tile += tw.step) {
            // this tile's loads were issued above or during the previous
            // tile's contraction
            auto prefetch = [&] {
                const int nt = tile + tw.step;   // unconditional (see EarlyPartials)
                st.load(nt < tw.end ? nt : tile, mb, src, nullptr, nt >= tw.end);
            };
            const WaveFaces wf = wave_faces<BND>(tile, mb, mb.dG);
            // g at the own rows, loaded ahead of the contraction
            double gvv[NMB][4];
            uint32_t o[NMB][4];
            bool ok[NMB][4];
#pragma unroll
            for (int m = 0; m < NMB; ++m)
#pragma unroll
                for (int e4 = 0; e4 < 4; ++e4) {
                    o[m][e4] = own_off<K, T>(wf, m, e4, nel, ok[m][e4]);
                    gvv[m][e4] = gv[ok[m][e4] ? o[m][e4] : 0u];
                }
            v4d acc[1][NMB];
            face_rows<K, 1>(fr, st, mb, wf, sB, src,
                            [](const double (&a)[1], uint32_t, bool) { return a[0]; },
                            acc, prefetch);
            if constexpr (BND) boundary_rows<K, T>(wf, sB, mb.bwall ? 4 : 1, acc);
            // r and g as B operands (zero past row 3K and off the mesh)
            double rb[NMB][4], gb[NMB][4];
#pragma unroll
            for (int m = 0; m < NMB; ++m)
#pragma unroll
                for (int e4 = 0; e4 < 4; ++e4) {
                    gb[m][e4] = ok[m][e4] ? gvv[m][e4] : 0.0;
                    rb[m][e4] = ok[m][e4] ? gvv[m][e4] - acc[0][m][e4] : 0.0;
                }
            if (!want_rin) {
#pragma unroll
                for (int m = 0; m < NMB; ++m)
#pragma unroll
                    for (int e4 = 0; e4 < 4; ++e4) {
                        acc4[0] += rb[m][e4] * rb[m][e4];
                        acc4[1] += gb[m][e4] * gb[m][e4];
                    }
                continue;
            }
            v4d ar[NMB], ag[NMB];
#pragma unroll
            for (int mo = 0; mo < NMB; ++mo) {
                ar[mo] = v4d{0, 0, 0, 0};
                ag[mo] = v4d{0, 0, 0, 0};
#pragma unroll
                for (int kk = 0; kk < 4 * NMB; ++kk) {
                    ar[mo] = MfmaT<double>::mma(pf[mo][kk], rb[kk / 4][kk % 4], ar[mo]);
                    ag[mo] = MfmaT<double>::mma(pf[mo][kk], gb[kk / 4][kk % 4], ag[mo]);
                }
            }
#pragma unroll
            for (int m = 0; m < NMB; ++m)
#pragma unroll
                for (int e4 = 0; e4 < 4; ++e4)
                    if (ok[m][e4]) {
                        const double ri = ar[m][e4];
                        rin[o[m][e4]] = (RT)ri;
                        acc4[0] += rb[m][e4] * rb[m][e4];
                        acc4[1] += gb[m][e4] * gb[m][e4];
                        acc4[2] += ag[m][e4] * ag[m][e4];
                        acc4[3] += ri * ri;
                    }
        }
    }
    store_partials<4, kFaceThreads>(acc4, partials, stride);
}

// ------------------------------------------------------------ BiCGStab
// Left-preconditioned BiCGStab (van der Vorst 1992) on Ghat d = rin, d0 = 0,
// with the block-Jacobi preconditioner folded into Ghat.  A solve is init
// (or, on the fixed schedule, refine_k1) and a first K1, then two launches
// per iteration:
//   K2:  alpha = rho / (rh.v);  s = r - alpha v on the fly, t = Ghat s;
//        partials P2 = (t.s, t.t, rh.t)
//   K1f: omega = (t.s)/(t.t);  d += alpha p + omega s;  r' = s - omega t;
//        p' = r' + beta (p - omega v), v' = Ghat p';
//        partials P1 = (rh.v', rh.r', r'.r')
// r, p and v are double buffered because K1f reads the old values at
// neighbouring faces while writing the new ones.  Convergence (r.r <= tol2)
// is detected at the start of K2; every later kernel returns at entry.
// Elementwise trace kernels: the member's nbe blocks run grid-stride loops
// over its 6 K nel trace values, four values per thread and pass with all
// loads issued before use.
struct ElemRange {
    size_t i0, span, n;
};

__device__ __forceinline__ ElemRange elem_range(const Member &mb, int lb, int K) {
    const size_t bd = blockDim.x;
    return ElemRange{(size_t)lb * bd * 4 + threadIdx.x, (size_t)mb.nbe * bd * 4,
                     (size_t)6 * K * mb.nel};
}

template <typename T>
__global__ void k_bicg_init(const Batch bt, int K, const T *__restrict__ rin,
                            T *__restrict__ r, T *__restrict__ rh, T *__restrict__ p,
                            T *__restrict__ v, T *__restrict__ d, KrylovState *ks_all,
                            double tol2, double *P3, int stride) {
    int lb;
    const int mi = member_of<CE>(bt, blockIdx.x, lb);
    const Member mb = load_member(bt, mi);
    rin += mb.to; r += mb.to; rh += mb.to; p += mb.to; v += mb.to; d += mb.to;
    double acc[2] = {0.0, 0.0};
    const ElemRange er = elem_range(mb, lb, K);
    const size_t bd = blockDim.x;
    for (size_t i0 = er.i0; i0 < er.n; i0 += er.span) {
        T x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = (i0 + u * bd < er.n) ? rin[i0 + u * bd] : T(0);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const size_t i = i0 + u * bd;
            if (i < er.n) {
                r[i] = x[u]; rh[i] = x[u]; p[i] = T(0); v[i] = T(0); d[i] = T(0);
                const double xd = x[u];
                acc[0] += xd * xd;
                acc[1] += xd * xd;
            }
        }
    }
    store_partials<2>(acc, P3, stride);
    if (lb == 0 && threadIdx.x == 0) {
        KrylovState *ks = ks_all + mi;
        ks->rho = 1.0;
        ks->alpha = 1.0;
        ks->omega = 1.0;
        ks->rr = 0.0;
        ks->rv = 0.0;
        ks->tol2 = tol2;
        ks->conv = 0;
        ks->breakdown = 0;
        ks->iters = 0;
    }
}

// Matrix-core fragments of Ghat in the inner solve's precision.
__device__ __forceinline__ const double *ghat_frags(const Member &mb, double) { return mb.Gh; }
__device__ __forceinline__ const float *ghat_frags(const Member &mb, float) { return mb.Ghf; }


// First K1 of an inner solve (after init or a refinement check): beta
// from rh.r and r.r [partials P3 of the elementwise class]; p <- r + beta
// (p - omega v) at the seven faces of each row block (p = v = 0 here), v =
// Ghat p; partials P1 = (rh.v, rh.r, r.r) over the own faces.
template <int K, typename T, bool SCHED, bool BND>
__global__ __launch_bounds__(kFaceThreads, (FaceOcc<K, T, BND, false>::value)) void k_bicg_k1(
    const Batch bt, const T *__restrict__ r, const T *__restrict__ rh,
    const T *__restrict__ pin, const T *__restrict__ vin, T *__restrict__ pout,
    T *__restrict__ vout, KrylovState *ks_all, const double *P3, double *P1, int stride) {
    constexpr int NMB = MF<K>::NMB;
    int lb;
    const int mi = member_of<CF>(bt, blockIdx.x, lb);
    const Member mb = load_member(bt, mi);
    KrylovState *ks = ks_all + mi;
    if (ks->conv) return;
    const double rho = ks->rho, alpha = ks->alpha, omega = ks->omega, tol2 = ks->tol2;
    // issue order: the partial sums, the A operands, the first tile; the
    // partial sums are reduced while the rest is in flight
    EarlyPartials<2> ep;
    ep.load(P3 + mb.be, stride, mb.nbe);
    __shared__ T sA[FragLds<K, T>::alloc];
    const T *gfr[1] = {ghat_frags(mb, T(0))};
    const T *fr[1];
    FragStage<K, T> fs;
    fs.load(gfr);
    r += mb.to; rh += mb.to; pin += mb.to; vin += mb.to; pout += mb.to; vout += mb.to;
    const T *src[3] = {r, pin, vin};
    const TileWalk tw = tile_walk(lb, mb.nbf, face_tiles(mb));
    StagedTile<K, T, 3> st;
    constexpr bool kEarly = sizeof(T) == 4;   // registers allow it for FP32
    // unconditional: a block without tiles loads tile 0 and never commits it
    if (kEarly) st.load(tw.first < tw.end ? tw.first : 0, mb, src);
    double red[2];
    ep.finish(red);
    fs.store(sA, fr);
    const double rho_new = red[0], rr = red[1];
    if (rr <= tol2 || rho_new == 0.0 || omega == 0.0 || !isfinite(rr)) {
        if (lb == 0 && threadIdx.x == 0) {
            ks->rr = rr;
            ks->breakdown = (rr <= tol2) ? 0 : 1;
            ks->conv = 1;
        }
        return;
    }
    const T beta = (T)((rho_new / rho) * (alpha / omega)), om = (T)omega;
    __shared__ T sB[TileLds<K, T>::n];
    const uint32_t nel = mb.nel;
    double acc1[3] = {0.0, 0.0, 0.0};
    {
        for (int tile = tw.first; tile < tw.end; tile += tw.step) {
            // FP32: this tile's loads were issued in the prologue or during
            // the previous tile's contraction
            if (!kEarly) st.load(tile, mb, src);
            auto prefetch = [&] {
                if constexpr (kEarly) {
                    const int nt = tile + tw.step;   // unconditional (see EarlyPartials)
                    st.load(nt < tw.end ? nt : tile, mb, src, nullptr, nt >= tw.end);
                }
            };
            const WaveFaces wf = wave_faces<BND>(tile, mb, delta_hat<T>(mb));
            T rhv[NMB][4], rv[NMB][4];
            uint32_t o[NMB][4];
            bool ok[NMB][4];
#pragma unroll
            for (int m = 0; m < NMB; ++m)
#pragma unroll
                for (int e4 = 0; e4 < 4; ++e4) {
                    o[m][e4] = own_off<K, T>(wf, m, e4, nel, ok[m][e4]);
                    rhv[m][e4] = rh[ok[m][e4] ? o[m][e4] : 0u];
                    rv[m][e4] = r[ok[m][e4] ? o[m][e4] : 0u];
                }
            typename MfmaT<T>::v4 acc[1][NMB];
            face_rows<K, 1>(fr, st, mb, wf, sB, src,
                                   [&](const T (&a)[3], uint32_t off, bool own) {
                                       const T p = a[0] + beta * (a[1] - om * a[2]);
                                       if (own) pout[off] = p;
                                       return p;
                                   },
                                   acc, prefetch);
            if constexpr (BND) boundary_rows<K, T>(wf, sB, mb.bwall ? 4 : 1, acc);
#pragma unroll
            for (int m = 0; m < NMB; ++m)
#pragma unroll
                for (int e4 = 0; e4 < 4; ++e4)
                    if (ok[m][e4]) {
                        const double y = acc[0][m][e4];
                        const double rhd = rhv[m][e4], rd = rv[m][e4];
                        vout[o[m][e4]] = (T)y;
                        acc1[0] += rhd * y;
                        acc1[1] += rhd * rd;
                        acc1[2] += rd * rd;
                    }
        }
    }
    store_partials<3>(acc1, P1, stride);
    if (lb == 0 && threadIdx.x == 0) ks->rr = rr;
}

// A refinement check fused with the first K1 of the sweep's inner solve
// (fixed launch schedule, where it replaces a separate check kernel and K1).  Every
// block reduces the member's FP64 residual norms of the last
// trace_residual (partials [4][face blocks]: ||r||^2, ||g||^2, ||ghat||^2,
// ||rin||^2).  Once relres = ||r|| / ||g|| <= refine_rtol the member's
// stage solve is done and the launch returns.  Otherwise the inner solve on
// Ghat d = rin starts from d = 0, so r = rh = p = rin, and v = Ghat rin; the
// own faces receive r, rh, p, v and d = 0, P1 = (rh.v, rh.r, r.r), and the
// tolerance is max(inner_rtol^2 ||rin||^2, (0.1 refine_rtol)^2 ||ghat||^2)
// (an inner solve that starts below it is converged at once).
template <int K, typename T, bool BND>
__global__ __launch_bounds__(kFaceThreads, (FaceOcc<K, T, BND, false>::value)) void k_refine_k1(
    const Batch bt, const T *__restrict__ rin, T *__restrict__ r, T *__restrict__ rh,
    T *__restrict__ pout, T *__restrict__ vout, T *__restrict__ d, KrylovState *ks_all,
    const double *res_partials, int rstride, double refine_rtol, double inner_rtol,
    double *P1, int stride) {
    constexpr int NMB = MF<K>::NMB;
    arg_now(ks_all);
    arg_now(rstride);
    arg_now(stride);
    int lb;
    const int mi = member_of<CF>(bt, blockIdx.x, lb);
    KrylovState *ks = ks_all + mi;
    const Member mb = load_member(bt, mi);
    // the member's fields and the flag in one round trip
    const int done = ks->stage_done;
    arg_now(mb.to);
    arg_now(mb.bf);
    if (done) return;
    // issue order: the residual norms, the A operands, the first tile
    EarlyPartials<4> ep;
    ep.load(res_partials + mb.bf, rstride, mb.nbf);
    __shared__ T sA[FragLds<K, T>::alloc];
    const T *gfr[1] = {ghat_frags(mb, T(0))};
    const T *fr[1];
    FragStage<K, T> fs;
    fs.load(gfr);
    rin += mb.to; r += mb.to; rh += mb.to; pout += mb.to; vout += mb.to; d += mb.to;
    const T *src[1] = {rin};
    const TileWalk tw = tile_walk(lb, mb.nbf, face_tiles(mb));
    StagedTile<K, T, 1> st;
    // unconditional: a block without tiles loads tile 0 and never commits it
    st.load(tw.first < tw.end ? tw.first : 0, mb, src);
    double nrm[4];
    ep.finish(nrm);
    fs.store(sA, fr);
    const double rr = nrm[0], gg = nrm[1], ghh = nrm[2], rinrin = nrm[3];
    const double relres = gg > 0.0 ? sqrt(rr / gg) : sqrt(rr);
    const bool finite = isfinite(rr) && isfinite(gg) && isfinite(rinrin);
    if (!finite || relres <= refine_rtol) {
        if (lb == 0 && threadIdx.x == 0) {
            ks->relres = finite ? relres : NAN;
            ks->stage_done = 1;
            ks->conv = 1;
        }
        return;
    }
    const double fl = 0.1 * refine_rtol;
    const double tol2 = fmax(inner_rtol * inner_rtol * rinrin, fl * fl * ghh);
    __shared__ T sB[TileLds<K, T>::n];
    const uint32_t nel = mb.nel;
    double acc1[3] = {0.0, 0.0, 0.0};
    for (int tile = tw.first; tile < tw.end; tile += tw.step) {
        auto prefetch = [&] {
            const int nt = tile + tw.step;   // unconditional (see EarlyPartials)
            st.load(nt < tw.end ? nt : tile, mb, src, nullptr, nt >= tw.end);
        };
        const WaveFaces wf = wave_faces<BND>(tile, mb, delta_hat<T>(mb));
        T rv[NMB][4];
        uint32_t o[NMB][4];
        bool ok[NMB][4];
#pragma unroll
        for (int m = 0; m < NMB; ++m)
#pragma unroll
            for (int e4 = 0; e4 < 4; ++e4) {
                o[m][e4] = own_off<K, T>(wf, m, e4, nel, ok[m][e4]);
                rv[m][e4] = rin[ok[m][e4] ? o[m][e4] : 0u];
            }
        typename MfmaT<T>::v4 acc[1][NMB];
        face_rows<K, 1>(fr, st, mb, wf, sB, src,
                        [&](const T (&a)[1], uint32_t off, bool own) {
                            if (own) {
                                r[off] = a[0];
                                rh[off] = a[0];
                                pout[off] = a[0];
                                d[off] = T(0);
                            }
                            return a[0];
                        },
                        acc, prefetch);
        if constexpr (BND) boundary_rows<K, T>(wf, sB, mb.bwall ? 4 : 1, acc);
#pragma unroll
        for (int m = 0; m < NMB; ++m)
#pragma unroll
            for (int e4 = 0; e4 < 4; ++e4)
                if (ok[m][e4]) {
                    const double y = acc[0][m][e4], rd = rv[m][e4];
                    vout[o[m][e4]] = (T)y;
                    acc1[0] += rd * y;
                    acc1[1] += rd * rd;
                    acc1[2] += rd * rd;
                }
    }
    store_partials<3>(acc1, P1, stride);
    if (lb == 0 && threadIdx.x == 0) {
        const bool done = rinrin <= tol2;
        ks->relres = relres;
        ks->rho = 1.0;
        ks->alpha = 1.0;
        ks->omega = 1.0;
        ks->rr = rinrin;
        ks->rv = 0.0;
        ks->tol2 = tol2;
        ks->conv = done ? 1 : 0;
        ks->breakdown = 0;
        ks->iters = 0;
        ks->sweep += 1;
    }
}

// s = r - alpha v, formed identically (one fused multiply-add) by K2, which
// applies Ghat to it, and by K1f, which recomputes it instead of K2 storing
// it.
__device__ __forceinline__ float s_of(float r, float al, float v) {
    return __builtin_fmaf(-al, v, r);
}
__device__ __forceinline__ double s_of(double r, double al, double v) {
    return __builtin_fma(-al, v, r);
}

// K2: rho = rh.r, rr = r.r and rv = rh.v from partials P1 (exact dot
// products of the last K1); stop when rr <= tol2; alpha = rho / rv;
// s = r - alpha v at the seven faces, t = Ghat s; partials P2 = (t.s, t.t,
// rh.t) over the own faces.
template <int K, typename T, bool SCHED, bool BND>
__global__ __launch_bounds__(kFaceThreads, MFOcc<K>::value) void k_bicg_k2(
    const Batch bt, const T *__restrict__ r, const T *__restrict__ v,
    const T *__restrict__ rh, T *__restrict__ t, KrylovState *ks_all,
    const double *P1, double *P2, int stride) {
    constexpr int NMB = MF<K>::NMB;
    arg_now(stride);
    arg_now(ks_all);
    int lb;
    const int mi = member_of<CF>(bt, blockIdx.x, lb);
    const Member mb = load_member(bt, mi);
    KrylovState *ks = ks_all + mi;
    // the member's fields and the flags in one round trip
    const int conv = ks->conv, brk = ks->breakdown;
    arg_now(mb.to);
    arg_now(mb.bf);
    if (conv) return;
    // a breakdown in the last K1f (which completed its iteration) ends the
    // solve here: the flag was written by an earlier launch, so every block
    // of this one decides alike
    if (brk) {
        if (lb == 0 && threadIdx.x == 0) ks->conv = 1;
        return;
    }
    const double tol2 = ks->tol2;
    // issue order: the partial sums, the A operands, the first tile; the
    // partial sums are reduced while the rest is in flight
    EarlyPartials<3, kFaceThreads> ep;
    ep.load(P1 + mb.bf, stride, mb.nbf);
    __shared__ T sA[FragLds<K, T>::alloc];
    const T *gfr[1] = {ghat_frags(mb, T(0))};
    const T *fr[1];
    FragStage<K, T> fs;
    fs.load(gfr);
    r += mb.to; v += mb.to; rh += mb.to; t += mb.to;
    const T *src[2] = {r, v};
    const TileWalk tw = tile_walk(lb, mb.nbf, face_tiles(mb));
    StagedTile<K, T, 2> st;
    constexpr bool kEarly = sizeof(T) == 4;   // registers allow it for FP32
    // unconditional: a block without tiles loads tile 0 and never commits it
    if (kEarly) st.load(tw.first < tw.end ? tw.first : 0, mb, src);
    double red1[3];
    ep.finish(red1);
    fs.store(sA, fr);
    const double rv = red1[0], rho = red1[1], rr = red1[2];
    if (rr <= tol2 || !isfinite(rr) || rv == 0.0 || !isfinite(rv)) {
        if (lb == 0 && threadIdx.x == 0) {
            ks->rr = rr;
            ks->breakdown = (rr <= tol2) ? 0 : 1;
            ks->conv = 1;
        }
        return;
    }
    const double alpha = rho / rv;
    const T al = (T)alpha;
    __shared__ T sB[TileLds<K, T>::n];
    const uint32_t nel = mb.nel;
    double acc2[3] = {0.0, 0.0, 0.0};
    {
        for (int tile = tw.first; tile < tw.end; tile += tw.step) {
            // FP32: this tile's loads were issued in the prologue or during
            // the previous tile's contraction
            if (!kEarly) st.load(tile, mb, src);
            auto prefetch = [&] {
                if constexpr (kEarly) {
                    const int nt = tile + tw.step;   // unconditional (see EarlyPartials)
                    st.load(nt < tw.end ? nt : tile, mb, src, nullptr, nt >= tw.end);
                }
            };
            const WaveFaces wf = wave_faces<BND>(tile, mb, delta_hat<T>(mb));
            uint32_t o[NMB][4];
            bool ok[NMB][4];
            T sown[NMB][4], rhv[NMB][4];
#pragma unroll
            for (int m = 0; m < NMB; ++m)
#pragma unroll
                for (int e4 = 0; e4 < 4; ++e4) {
                    o[m][e4] = own_off<K, T>(wf, m, e4, nel, ok[m][e4]);
                    rhv[m][e4] = rh[ok[m][e4] ? o[m][e4] : 0u];
                    sown[m][e4] = T(0);
                }
            typename MfmaT<T>::v4 acc[1][NMB];
            face_rows<K, 1>(fr, st, mb, wf, sB, src,
                                   [&](const T (&a)[2], uint32_t, bool) {
                                       return s_of(a[0], al, a[1]);
                                   },
                                   acc, prefetch);
            if constexpr (BND) boundary_rows<K, T>(wf, sB, mb.bwall ? 4 : 1, acc);
            {
                const int li = own_lds<K>(wf);
#pragma unroll
                for (int m = 0; m < NMB; ++m)
#pragma unroll
                    for (int e4 = 0; e4 < 4; ++e4) {
                        const int row = 16 * m + MfmaT<T>::row(threadIdx.x & 63, e4);
                        if (ok[m][e4]) sown[m][e4] = sB[row * TileRow<K, T>::stride + li];
                    }
            }
#pragma unroll
            for (int m = 0; m < NMB; ++m)
#pragma unroll
                for (int e4 = 0; e4 < 4; ++e4)
                    if (ok[m][e4]) {
                        const double y = acc[0][m][e4];
                        const double sval = sown[m][e4];
                        t[o[m][e4]] = (T)y;
                        acc2[0] += y * sval;
                        acc2[1] += y * y;
                        acc2[2] += (double)rhv[m][e4] * y;
                    }
        }
    }
    store_partials<3, kFaceThreads>(acc2, P2, stride);
    if (lb == 0 && threadIdx.x == 0) {
        ks->rho = rho;
        ks->alpha = alpha;
        ks->rv = rv;
        ks->rr = rr;
    }
}

// K1 of the next iteration fused with the d and r updates of this one:
//   omega = (t.s)/(t.t) and rh.t from partials P2 of K2;
//   rho' = rh.(s - omega t) = (rho - alpha rv) - omega rh.t;
//   beta = (rho'/rho)(alpha/omega);
//   s = r - alpha v (recomputed as in K2), r' = s - omega t,
//   p' = r' + beta (p - omega v) at the seven faces of each row block,
//   v' = Ghat p';  d += alpha p + omega s, r', p', v' stored at the own
//   faces (r', p' and v' into the other buffer of each pair: neighbouring
//   blocks still read r, p and v);  partials P1 = (rh.v', rh.r', r'.r').
// On breakdown (omega or rho' zero or not finite) the d and r updates still
// complete the iteration in every block, and the solve stops at the next K2:
// this launch only flags it (a flag read at entry and written in the same
// launch would let a block that starts after block 0 has finished skip its
// updates).
template <int K, typename T, bool SCHED, bool BND>
__global__ __launch_bounds__(kFaceThreads, (FaceOcc<K, T, BND, true>::value)) void k_bicg_k1f(
    const Batch bt, const T *__restrict__ rin, const T *__restrict__ t,
    const T *__restrict__ rh, const T *__restrict__ pin, const T *__restrict__ vin,
    T *__restrict__ pout, T *__restrict__ vout, T *__restrict__ r, T *__restrict__ d,
    KrylovState *ks_all, const double *P2, double *P1, int stride) {
    constexpr int NMB = MF<K>::NMB;
    arg_now(stride);
    arg_now(ks_all);
    int lb;
    const int mi = member_of<CF>(bt, blockIdx.x, lb);
    const Member mb = load_member(bt, mi);
    KrylovState *ks = ks_all + mi;
    // the member's fields and the flags in one round trip
    const int conv = ks->conv, fbrk = ks->force_brk;
    arg_now(mb.to);
    arg_now(mb.bf);
    if (conv) return;
    const double rho = ks->rho, alpha = ks->alpha, rvv = ks->rv;
    // issue order: the partial sums, the A operands, the first tile; the
    // partial sums are reduced while the rest is in flight
    EarlyPartials<3, kFaceThreads> ep;
    ep.load(P2 + mb.bf, stride, mb.nbf);
    __shared__ T sA[FragLds<K, T>::alloc];
    const T *gfr[1] = {ghat_frags(mb, T(0))};
    const T *fr[1];
    FragStage<K, T> fs;
    fs.load(gfr);
    rin += mb.to; t += mb.to; rh += mb.to; pin += mb.to; vin += mb.to;
    pout += mb.to; vout += mb.to; r += mb.to; d += mb.to;
    const T *src[4] = {rin, t, pin, vin};
    // With the tile held in registers (K <= 7): the staging thread of an
    // own face also reads d there and updates r, p and d, and leaves r' in
    // LDS for the matrix-core lanes (which hold rh) to sum rh.r' and r'.r'.
    // FP32 always; FP64 where one block runs per CU anyway (K >= 6).  FP64
    // at K <= 5 keeps its registers for two blocks per CU and updates the
    // own faces after the contraction, reading them again.
    constexpr bool kOwnStage =
        (sizeof(T) == 4 || MFOcc<K>::value == 1) && StagedTile<K, T, 4>::kHold;
    const T *osrc[1] = {d};
    const TileWalk tw = tile_walk(lb, mb.nbf, face_tiles(mb));
    StagedTile<K, T, 4, kOwnStage ? 1 : 0> st;
    constexpr bool kEarly = sizeof(T) == 4;   // registers allow it for FP32
    // unconditional: a block without tiles loads tile 0 and never commits it
    if (kEarly) st.load(tw.first < tw.end ? tw.first : 0, mb, src, osrc);
    double red[3];
    ep.finish(red);
    fs.store(sA, fr);
    const double ts = red[0], tt = red[1], rht = red[2];
    const double omega = tt > 0.0 ? ts / tt : 0.0;
    const double rho_new = (rho - alpha * rvv) - omega * rht;
    const bool brk = !(omega != 0.0) || !isfinite(omega) || !(rho_new != 0.0) ||
                     !isfinite(rho_new) || fbrk != 0;
    const double beta = brk ? 0.0 : (rho_new / rho) * (alpha / omega);
    const T be = (T)beta, om = (T)omega, al = (T)alpha;
    __shared__ T sB[TileLds<K, T>::n];
    __shared__ T sR[kOwnStage ? TileLds<K, T>::n : 1];   // r' at the own faces
    const uint32_t nel = mb.nel;
    auto rnew = [&](T s_, T t_) { return (T)((double)s_ - omega * (double)t_); };
    auto pnew = [&](T r_, T p_, T v_) { return r_ + be * (p_ - om * v_); };
    double acc1[3] = {0.0, 0.0, 0.0};
    {
        for (int tile = tw.first; tile < tw.end; tile += tw.step) {
            // FP32: this tile's loads were issued in the prologue or during
            // the previous tile's contraction
            if (!kEarly) st.load(tile, mb, src, osrc);
            auto prefetch = [&] {
                if constexpr (kEarly) {
                    const int nt = tile + tw.step;   // unconditional (see EarlyPartials)
                    st.load(nt < tw.end ? nt : tile, mb, src, osrc, nt >= tw.end);
                }
            };
            const WaveFaces wf = wave_faces<BND>(tile, mb, delta_hat<T>(mb));
            T rhv[NMB][4];
            uint32_t o[NMB][4];
            bool ok[NMB][4];
#pragma unroll
            for (int m = 0; m < NMB; ++m)
#pragma unroll
                for (int e4 = 0; e4 < 4; ++e4) {
                    o[m][e4] = own_off<K, T>(wf, m, e4, nel, ok[m][e4]);
                    rhv[m][e4] = rh[ok[m][e4] ? o[m][e4] : 0u];
                }
            typename MfmaT<T>::v4 acc[1][NMB];
            // r_ is r at the face; s = r - alpha v as in K2
            auto own_update = [&](T r_, T t_, T p_, T v_, T d_, T rh_, uint32_t oo) {
                const T s_ = s_of(r_, al, v_);
                const T rn = rnew(s_, t_);
                r[oo] = rn;
                pout[oo] = pnew(rn, p_, v_);
                d[oo] = (T)((double)d_ + alpha * (double)p_ + omega * (double)s_);
                const double rd = rn;
                acc1[1] += (double)rh_ * rd;
                acc1[2] += rd * rd;
            };
            if constexpr (kOwnStage) {
                face_rows<K, 1>(fr, st, mb, wf, sB, src,
                                [&](const T (&a)[4], const T (&ov)[1], uint32_t off, bool own,
                                    int li) {
                                    const T s_ = s_of(a[0], al, a[3]);
                                    const T rn = rnew(s_, a[1]);
                                    const T pn = pnew(rn, a[2], a[3]);
                                    if (own) {
                                        r[off] = rn;
                                        pout[off] = pn;
                                        d[off] = (T)((double)ov[0] + alpha * (double)a[2] +
                                                     omega * (double)s_);
                                        sR[li] = rn;
                                    }
                                    return pn;
                                },
                                acc, prefetch);
                if constexpr (BND) boundary_rows<K, T>(wf, sB, mb.bwall ? 4 : 1, acc);
                const int li = own_lds<K>(wf);
#pragma unroll
                for (int m = 0; m < NMB; ++m)
#pragma unroll
                    for (int e4 = 0; e4 < 4; ++e4)
                        if (ok[m][e4]) {
                            const int row = 16 * m + MfmaT<T>::row(threadIdx.x & 63, e4);
                            const double rd = sR[row * TileRow<K, T>::stride + li];
                            acc1[1] += (double)rhv[m][e4] * rd;
                            acc1[2] += rd * rd;
                        }
            } else {
                face_rows<K, 1>(fr, st, mb, wf, sB, src,
                                [&](const T (&a)[4], uint32_t, bool) {
                                    return pnew(rnew(s_of(a[0], al, a[3]), a[1]), a[2], a[3]);
                                },
                                acc, prefetch);
                if constexpr (BND) boundary_rows<K, T>(wf, sB, mb.bwall ? 4 : 1, acc);
                // own faces: all loads first, then the updates
                T sv_[NMB][4], tv_[NMB][4], pv_[NMB][4], vv_[NMB][4], dv_[NMB][4];
#pragma unroll
                for (int m = 0; m < NMB; ++m)
#pragma unroll
                    for (int e4 = 0; e4 < 4; ++e4) {
                        const bool k_ = ok[m][e4];
                        const uint32_t oo = o[m][e4];
                        sv_[m][e4] = rin[k_ ? oo : 0u];
                        tv_[m][e4] = t[k_ ? oo : 0u];
                        pv_[m][e4] = pin[k_ ? oo : 0u];
                        vv_[m][e4] = vin[k_ ? oo : 0u];
                        dv_[m][e4] = d[k_ ? oo : 0u];
                    }
#pragma unroll
                for (int m = 0; m < NMB; ++m)
#pragma unroll
                    for (int e4 = 0; e4 < 4; ++e4)
                        if (ok[m][e4])
                            own_update(sv_[m][e4], tv_[m][e4], pv_[m][e4], vv_[m][e4],
                                       dv_[m][e4], rhv[m][e4], o[m][e4]);
            }
            // the matrix-core lanes store v' = Ghat p' and sum rh.v'
#pragma unroll
            for (int m = 0; m < NMB; ++m)
#pragma unroll
                for (int e4 = 0; e4 < 4; ++e4)
                    if (ok[m][e4]) {
                        const double y = acc[0][m][e4];
                        vout[o[m][e4]] = (T)y;
                        acc1[0] += (double)rhv[m][e4] * y;
                    }
        }
    }
    store_partials<3, kFaceThreads>(acc1, P1, stride);
    if (lb == 0 && threadIdx.x == 0) {
        ks->omega = omega;
        ks->iters += 1;
        if (brk) ks->breakdown = 1;
    }
}

template <typename T>
__global__ void k_axpy(double *__restrict__ y, const T *__restrict__ x, double a, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += a * x[i];
}

// ------------------------------------- device-driven refinement sweeps
// A stage solve on a fixed launch schedule: the host enqueues every sweep
// and a budget of inner iterations up front (so the whole step can be
// captured in a graph); the decisions the host-driven loop takes after a
// read-back are taken here on the device, and launches past convergence
// return at entry.
// x += d after a sweep, unless the member's stage solve had already
// converged.
template <typename T>
__global__ void k_axpy_guarded(const Batch bt, int K, double *__restrict__ y,
                               const T *__restrict__ x, KrylovState *ks_all) {
    int lb;
    const int mi = member_of<CE>(bt, blockIdx.x, lb);
    KrylovState *ks = ks_all + mi;
    if (ks->stage_done) return;
    const Member mb = load_member(bt, mi);
    y += mb.to;
    x += mb.to;
    const ElemRange er = elem_range(mb, lb, K);
    const size_t bd = blockDim.x;
    for (size_t i0 = er.i0; i0 < er.n; i0 += er.span) {
        T xv[4];
        double yv[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const bool ok = i0 + u * bd < er.n;
            xv[u] = ok ? x[i0 + u * bd] : T(0);
            yv[u] = ok ? y[i0 + u * bd] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (i0 + u * bd < er.n) y[i0 + u * bd] = yv[u] + (double)xv[u];
    }
    if (lb == 0 && threadIdx.x == 0) {
        const int sw = ks->sweep - 1;
        if (sw >= 0 && sw < 8) ks->sweep_iters[sw] = ks->iters;
    }
}


// ------------------------------------------- variable bathymetry
// DG residuals over nodal phi_B (pB, one value per node in the volume
// layout of one variable).  LIN = false: M^-1 NL(q), the nonlinear flux
// F_NL = (0, U U / phi + phi_eta^2 / 2, U V / phi | ...) with phi = phi_eta
// + phi_B at the node and the flux F* - F*_L (Sec. 4.3), tau* = max of
// |u.n| + sqrt(phi) and tau_L* = max of sqrt(phi_B) over the two sides;
// the stage combination `comb` as in k_nl.  LIN = true: the stage
// residual out = R - (Q - c M^-1 L(Q)) of the linear part, L with F_L =
// (U, phi_B phi_eta I), the Lax-Friedrichs flux with tau_L* and the source
// (0, phi_eta grad phi_B) (grad of the element's interpolant of phi_B),
// c = a~_ii dt of the member; partials [2][blocks] of ||out||^2, ||R||^2.
// One thread per (element, node row j); the y fluxes through LDS.
template <bool LIN>
__device__ __forceinline__ void var_flux(double p, double U, double V, double b, double F[2][3]) {
    if (LIN) {
        F[0][0] = U; F[0][1] = b * p; F[0][2] = 0.0;
        F[1][0] = V; F[1][1] = 0.0; F[1][2] = b * p;
    } else {
        const double inv = 1.0 / (p + b), hp = 0.5 * p * p;
        F[0][0] = 0.0; F[0][1] = U * U * inv + hp; F[0][2] = U * V * inv;
        F[1][0] = 0.0; F[1][1] = V * U * inv; F[1][2] = V * V * inv + hp;
    }
}

template <bool LIN>
__device__ __forceinline__ void var_numflux(const double qm[3], const double qp[3], double bm,
                                            double bp, double nx, double ny, double f[3]) {
    double Fm[2][3], Fp[2][3];
    var_flux<LIN>(qm[0], qm[1], qm[2], bm, Fm);
    var_flux<LIN>(qp[0], qp[1], qp[2], bp, Fp);
    const double tl = fmax(sqrt(bm), sqrt(bp));
    double diss = tl;
    if (!LIN) {
        const double sm = fabs((qm[1] * nx + qm[2] * ny) / (qm[0] + bm)) + sqrt(qm[0] + bm);
        const double sp = fabs((qp[1] * nx + qp[2] * ny) / (qp[0] + bp)) + sqrt(qp[0] + bp);
        diss = fmax(sm, sp) - tl;
    }
    for (int c = 0; c < 3; ++c)
        f[c] = 0.5 * ((Fm[0][c] + Fp[0][c]) * nx + (Fm[1][c] + Fp[1][c]) * ny) +
               0.5 * diss * (qm[c] - qp[c]);
}

template <int K, bool LIN>
__global__ __launch_bounds__(64 * K) void k_dg_var(const double *__restrict__ q,
                                                   const double *__restrict__ pB, const Geom g,
                                                   const Batch bt, const Comb comb, int scale_dt,
                                                   const double *__restrict__ R,
                                                   double *__restrict__ out, double cst,
                                                   double *partials, int stride) {
    __shared__ double sF[3][K][K][64];
    const int lane = threadIdx.x & 63;
    const int j = wave_id();
    int lb;
    const Member mb = load_member(bt, member_of<CV>(bt, blockIdx.x, lb));
    q += mb.vo;
    pB += mb.vo / 3;
    const int e = lb * 64 + lane;
    // a bounded member's ghost elements carry boundary states only: no
    // residual, no contribution to the norms
    const bool ghost = mb.bx > 0 && (e % mb.nx >= mb.bx || e / mb.nx >= mb.by);
    const bool active = e < mb.nel && !ghost;
    const Nbr nb = neighbours(active ? e : 0, mb.nx, mb.ny);
    const size_t nel = mb.nel, NN = (size_t)K * K * nel;
    auto at = [&](int row, int i, int el, double v[3], double &b) {
        const size_t o = (size_t)(row * K + i) * nel + el;
        v[0] = q[o]; v[1] = q[NN + o]; v[2] = q[2 * NN + o];
        b = pB[o];
    };
    double p[K], U[K], V[K], b[K], o[3][K];
    for (int i = 0; i < K; ++i) {
        double v[3];
        at(j, i, nb.e, v, b[i]);
        p[i] = v[0]; U[i] = v[1]; V[i] = v[2];
    }
    double Fx[3][K];
    for (int i = 0; i < K; ++i) {
        double F[2][3];
        var_flux<LIN>(p[i], U[i], V[i], b[i], F);
        for (int c = 0; c < 3; ++c) {
            Fx[c][i] = F[0][c];
            sF[c][j][i][lane] = F[1][c];
        }
    }
    const double sx = mb.sx, sy = mb.sy;
    for (int a = 0; a < K; ++a)
        for (int c = 0; c < 3; ++c) {
            double sacc = 0.0;
            for (int m = 0; m < K; ++m) sacc += g.Dw[m * K + a] * Fx[c][m];
            o[c][a] = sx * sacc;
        }
    {   // east and west faces of row j
        double qm[3], qp[3], bp, f[3];
        qm[0] = p[K - 1]; qm[1] = U[K - 1]; qm[2] = V[K - 1];
        at(j, 0, nb.east, qp, bp);
        var_numflux<LIN>(qm, qp, b[K - 1], bp, 1.0, 0.0, f);
        for (int c = 0; c < 3; ++c) o[c][K - 1] -= sx * g.winvk * f[c];
        qm[0] = p[0]; qm[1] = U[0]; qm[2] = V[0];
        at(j, K - 1, nb.west, qp, bp);
        var_numflux<LIN>(qm, qp, b[0], bp, -1.0, 0.0, f);
        for (int c = 0; c < 3; ++c) o[c][0] -= sx * g.winv0 * f[c];
    }
    __syncthreads();
    for (int i = 0; i < K; ++i)
        for (int c = 0; c < 3; ++c) {
            double sacc = 0.0;
            for (int m = 0; m < K; ++m) sacc += g.Dw[m * K + j] * sF[c][m][i][lane];
            o[c][i] += sy * sacc;
        }
    if (j == K - 1 || j == 0) {
        const bool north = j == K - 1;
        const int other = north ? nb.north : nb.south, orow = north ? 0 : K - 1;
        const double ny = north ? 1.0 : -1.0, sc = sy * (north ? g.winvk : g.winv0);
        for (int i = 0; i < K; ++i) {
            double qm[3] = {p[i], U[i], V[i]}, qp[3], bp, f[3];
            at(orow, i, other, qp, bp);
            var_numflux<LIN>(qm, qp, b[i], bp, 0.0, ny, f);
            for (int c = 0; c < 3; ++c) o[c][i] -= sc * f[c];
        }
    }
    if (LIN) {
        // source (0, phi_eta d_x phi_B, phi_eta d_y phi_B) with the
        // derivatives of the element's interpolant of phi_B at the node
        for (int i = 0; i < K; ++i) {
            double dx = 0.0, dy = 0.0;
            for (int m = 0; m < K; ++m) {
                double bm_;
                double v[3];
                at(m, i, nb.e, v, bm_);
                dx += g.D[i * K + m] * b[m];
                dy += g.D[j * K + m] * bm_;
            }
            o[1][i] += p[i] * sx * dx;
            o[2][i] += p[i] * sy * dy;
        }
    }
    double acc[2] = {0.0, 0.0};
    if (active) {
        const size_t o0 = mb.vo + (size_t)(j * K) * nel + e;
        if (LIN) {
            for (int i = 0; i < K; ++i) {
                const size_t oi = o0 + (size_t)i * nel;
                const double Qv[3] = {p[i], U[i], V[i]};
                for (int c = 0; c < 3; ++c) {
                    const double r = R[c * NN + oi];
                    const double v = r - (Qv[c] - cst * mb.dt * o[c][i]);
                    out[c * NN + oi] = v;
                    acc[0] += v * v;
                    acc[1] += r * r;
                }
            }
        } else {
            const double scl = scale_dt ? mb.dt : 1.0;
            for (int i = 0; i < K; ++i) {
                const size_t oi = o0 + (size_t)i * nel;
                for (int c = 0; c < 3; ++c) {
                    const double x = o[c][i] * scl;
                    if (comb.store) comb.store[c * NN + oi] = x;
                    double v = comb.self * x;
                    for (int t = 0; t < comb.n; ++t) v += comb.coef[t] * comb.in[t][c * NN + oi];
                    comb.out[c * NN + oi] = v;
                }
            }
        }
    }
    if (LIN) store_partials<2>(acc, partials, stride);
}

// ------------------------------------------------ boundary states
// The exact translating vortex of Sec. 6.1 (eq. tc_vortex_ic) at (x, y, t)
// in the geopotential variables: depth h = H - beta^2 / (32 pi^2)
// exp(-2 (r^2 - 1)), velocity (u_inf - beta / (2 pi) exp(-(r^2 - 1)) y_t,
// v_inf + beta / (2 pi) exp(-(r^2 - 1)) x_t), x_t = x - xc - u_inf t,
// y_t = y - yc - v_inf t; (phi_eta, U, V) = (g (h - H), g h u, g h v).
__device__ __forceinline__ void vortex_state(const Vortex &v, double x, double y, double t,
                                             double &p, double &U, double &V) {
    const double xt = x - v.xc - v.uinf * t, yt = y - v.yc - v.vinf * t;
    const double r2 = xt * xt + yt * yt;
    const double e = exp(-(r2 - 1.0));
    const double pi = 3.141592653589793;
    const double h = v.H - v.beta * v.beta / (32.0 * (pi * pi)) * e * e;
    const double u = v.uinf - v.beta / (2.0 * pi) * e * yt;
    const double w = v.vinf + v.beta / (2.0 * pi) * e * xt;
    p = v.g * (h - v.H);
    U = v.g * (h * u);
    V = v.g * (h * w);
}

// Ghost elements of a bounded member (see Member): every node of a ghost
// takes the boundary state at the point of the domain boundary it faces
// (only the nodes on the shared face are read: by the explicit flux, and
// by the trace right-hand side from Z).  One thread per (element, node
// row j, node i): block = 64 elements x K rows.
__global__ __launch_bounds__(64 * kMaxK) void k_bc_fill(double *__restrict__ q, const Geom g,
                                                        const Batch bt, const double *tstep,
                                                        double toff, double *tnext,
                                                        const Vortex vx) {
    const int K = g.K;
    const int lane = threadIdx.x & 63, j = threadIdx.x >> 6;
    int lb;
    const Member mb = load_member(bt, member_of<CV>(bt, blockIdx.x, lb));
    if (mb.bx == 0) return;
    if (tnext != nullptr && lb == 0 && threadIdx.x == 0) tnext[0] = tstep[0] + 1.0;
    const int e = lb * 64 + lane;
    if (e >= mb.nel) return;
    const int ex = e % mb.nx, ey = e / mb.nx;
    const bool gx = ex >= mb.bx, gy = ey >= mb.by;
    if (!gx && !gy) return;
    q += mb.vo;
    const size_t nel = mb.nel, NN = (size_t)K * K * nel;
    if (mb.bwall) {
        // the real element across the boundary face and its node on that
        // face; the normal momentum (U across x-walls, V across y-walls)
        // changes sign
        for (int i = 0; i < K; ++i) {
            double p = 0.0, U = 0.0, V = 0.0;
            if (gx != gy) {
                int se, sn;
                if (gx) {
                    se = ey * mb.nx + (ex == mb.bx ? mb.bx - 1 : 0);
                    sn = j * K + (ex == mb.bx ? K - 1 : 0);
                } else {
                    se = (ey == mb.by ? mb.by - 1 : 0) * mb.nx + ex;
                    sn = (ey == mb.by ? K - 1 : 0) * K + i;
                }
                const size_t so = (size_t)sn * nel + se;
                p = q[so];
                U = gx ? -q[NN + so] : q[NN + so];
                V = gx ? q[2 * NN + so] : -q[2 * NN + so];
            }
            const size_t o = (size_t)(j * K + i) * nel + e;
            q[o] = p;
            q[NN + o] = U;
            q[2 * NN + o] = V;
        }
        return;
    }
    const double t = tstep[0] * mb.dt + toff;
    const double hx = 2.0 / mb.sx, hy = 2.0 / mb.sy;
    for (int i = 0; i < K; ++i) {
        double p = 0.0, U = 0.0, V = 0.0;
        if (gx != gy) {
            double x, y;
            if (gx) {   // east (bx) or west (bx + 1) ghost: boundary x, the node's y
                x = ex == mb.bx ? mb.bx * hx : 0.0;
                y = (ey + (g.xi[j] + 1.0) * 0.5) * hy;
            } else {    // north (by) or south (by + 1) ghost: the node's x, boundary y
                x = (ex + (g.xi[i] + 1.0) * 0.5) * hx;
                y = ey == mb.by ? mb.by * hy : 0.0;
            }
            vortex_state(vx, x, y, t, p, U, V);
        }
        const size_t o = (size_t)(j * K + i) * nel + e;
        q[o] = p;
        q[NN + o] = U;
        q[2 * NN + o] = V;
    }
}

__global__ void k_put_f64(double *p, double v) { p[0] = v; }

// --------------------------------------------------------- diagnostics
// Partials of (mass phi_eta, mass U, mass V, energy, non-finite count).
template <int K>
__global__ __launch_bounds__(64 * K) void k_diag(const double *__restrict__ q, const Geom g,
                                                 const Batch bt, double *partials,
                                                 int stride) {
    const int lane = threadIdx.x & 63;
    const int j = wave_id();
    int lb;
    const Member mb = load_member(bt, member_of<CD>(bt, blockIdx.x, lb));
    q += mb.vo;
    const size_t nel = mb.nel, NN = (size_t)K * K * nel;
    double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int e = lb * 64 + lane; e < mb.nel; e += mb.nbd * 64) {
        if (mb.bx > 0 && (e % mb.nx >= mb.bx || e / mb.nx >= mb.by)) continue;   // ghost
        for (int i = 0; i < K; ++i) {
            const size_t o = (size_t)(j * K + i) * nel + e;
            const double m = mb.area * g.w[i] * g.w[j];
            const double p = q[o], U = q[NN + o], V = q[2 * NN + o];
            acc[0] += m * p;
            acc[1] += m * U;
            acc[2] += m * V;
            acc[3] += m * (p * p + (U * U + V * V) / g.phiB);
            if (!isfinite(p) || !isfinite(U) || !isfinite(V)) acc[4] += 1.0;
        }
    }
    store_partials<5>(acc, partials, stride);
}

// State in from a caller's device array (see launch_state_in).  Each thread
// reads consecutive host-ordered values (coalesced) and scatters them to the
// element-fastest device layout; the checks are those of the host path.
template <typename T>
__global__ void k_state_in(const T *__restrict__ src, int depth, double g, double H,
                           double phiB, const double *__restrict__ pBn, int nel, int KK,
                           double *__restrict__ dst, double *partials, int stride, int bx,
                           int nxp) {
    const size_t nn = (size_t)nel * KK;
    // bounded member: real element e = ey bx + ex sits at ey nxp + ex of the
    // padded layout of nxp (nel / bx + 2) elements
    const size_t nd = bx > 0 ? (size_t)nxp * (nel / bx + 2) : (size_t)nel;
    double bad[1] = {0.0};
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nn;
         i += (size_t)gridDim.x * blockDim.x) {
        const double a = (double)src[i], b = (double)src[nn + i], c = (double)src[2 * nn + i];
        const size_t e = i / KK, n = i - e * KK;
        const size_t ed = bx > 0 ? (e / bx) * nxp + e % bx : e;
        const size_t o = n * nd + ed, nnd = nd * KK;
        // the node's phi_B: nodal with a variable depth, else g H
        const double pb = pBn ? pBn[o] : phiB;
        // g h rounded before the subtraction (no fused multiply-add), as the
        // host conversion rounds it
        double p;
        {
#pragma clang fp contract(off)
            p = depth ? (pBn ? g * a - pb : g * (a - H)) : a;
        }
        const double U = depth ? g * b : b;
        const double V = depth ? g * c : c;
        const double phi = p + pb;
        const bool ok = isfinite(p) && isfinite(U) && isfinite(V) && phi > 0.0;
        if (!ok) bad[0] += 1.0;
        dst[o] = p;
        dst[nnd + o] = U;
        dst[2 * nnd + o] = V;
    }
    store_partials<1>(bad, partials, stride);
}

inline unsigned grid1(size_t n, unsigned b) { return (unsigned)((n + b - 1) / b); }

template <template <int> class F, typename... Args>
hipError_t dispatch(int K, Args &&...args) {
    switch (K) {
        case 2: return F<2>::run(args...);
        case 3: return F<3>::run(args...);
        case 4: return F<4>::run(args...);
        case 5: return F<5>::run(args...);
        case 6: return F<6>::run(args...);
        case 7: return F<7>::run(args...);
        case 8: return F<8>::run(args...);
        case 9: return F<9>::run(args...);
        default: return hipErrorInvalidValue;
    }
}

template <int K> struct RunNL {
    static hipError_t run(const Geom &g, const Batch &b, const double *q, const Comb &c,
                          bool scale_dt, bool fp32, hipStream_t s) {
        if (fp32)
            KLAUNCH((k_nl<K, float>), dim3(b.nbv), dim3(64 * K), 0, s, q, g, b, c,
                    scale_dt ? 1 : 0);
        else
            KLAUNCH((k_nl<K, double>), dim3(b.nbv), dim3(64 * K), 0, s, q, g, b, c,
                    scale_dt ? 1 : 0);
        return hipGetLastError();
    }
};
template <int K> struct RunLinres {
    static hipError_t run(const Geom &g, const Batch &b, const double *Q, const double *qh,
                          double *out, hipStream_t s) {
        KLAUNCH(k_linres<K>, dim3(b.nbv), dim3(64 * K), 0, s, Q, qh, g, b, out);
        return hipGetLastError();
    }
};
template <int K> struct RunLocal {
    static hipError_t run(const Batch &b, const double *R, double *Z, hipStream_t s) {
        // measured: the LDS variant wins at K <= 4; at K = 5 the streamed
        // one is faster (its 48 KB matrix costs the LDS variant occupancy)
        if constexpr (K <= 4 && LocalLds<3 * K * K, 3 * K * K>::value)
            KLAUNCH(k_local_apply_lds<K>, dim3(b.nbv), dim3(256), 0, s, R, b, Z);
        else
            KLAUNCH(k_local_apply<K>, dim3(b.nbv), dim3(256), 0, s, R, b, Z);
        return hipGetLastError();
    }
};
template <int K> struct RunRecover {
    static hipError_t run(const Batch &b, const double *Z, const double *qh, double *Q,
                          const KrylovState *ks, const double *part, int stride,
                          StageStatus *status, hipStream_t s) {
        if constexpr (LocalLds<3 * K * K, 12 * K>::value)
            KLAUNCH(k_recover_lds<K>, dim3(b.nbv), dim3(256), 0, s, Z, qh, b, Q, ks, part,
                    stride, status);
        else
            KLAUNCH(k_recover<K>, dim3(b.nbv), dim3(256), 0, s, Z, qh, b, Q, ks, part, stride,
                    status);
        return hipGetLastError();
    }
};
template <int K> struct RunLocalLp {
    template <typename LP, int NDC>
    static hipError_t go(const Geom &g, const Batch &b, const double *R, const double *qh,
                         double aii, double *out, const KrylovState *ks, const double *part,
                         int stride, StageStatus *status, hipStream_t s) {
        using L = LocalLp<K, LP>;
        KLAUNCH((k_local_lp<K, LP, NDC>), dim3(b.nbv * L::SPLIT), dim3(L::THREADS), 0, s, R, qh,
                g, b, aii, out, ks, part, stride, status);
        return hipGetLastError();
    }
    static hipError_t run(const Geom &g, const Batch &b, const double *R, const double *qh,
                          double aii, double *out, bool bf16, int ndc, const KrylovState *ks,
                          const double *part, int stride, StageStatus *status, hipStream_t s) {
        if (bf16)
            return ndc == 1   ? go<__bf16, 1>(g, b, R, qh, aii, out, ks, part, stride, status, s)
                   : ndc == 2 ? go<__bf16, 2>(g, b, R, qh, aii, out, ks, part, stride, status, s)
                              : go<__bf16, 3>(g, b, R, qh, aii, out, ks, part, stride, status, s);
        return ndc == 1 ? go<float, 1>(g, b, R, qh, aii, out, ks, part, stride, status, s)
                        : go<float, 2>(g, b, R, qh, aii, out, ks, part, stride, status, s);
    }
};
template <int K> struct RunTraceRhs {
    static hipError_t run(const Geom &g, const Batch &b, const double *Z, double *gv,
                          KrylovState *begin, double *x, double *xp, double xc,
                          hipStream_t s) {
        KLAUNCH(k_trace_rhs<K>, dim3(2 * b.nbv), dim3(64 * K), 0, s, Z, g, b, gv, begin, x,
                xp, xc);
        return hipGetLastError();
    }
};
// The face kernels exist in a periodic (BND = false) and a bounded-mesh
// variant; the batch's box flag picks one.
template <typename RT> struct RunTraceResidual {
    template <int K> struct F {
        static hipError_t run(const Batch &b, const double *x, const double *gv, RT *rin,
                              double *partials, int stride, const KrylovState *skip,
                              hipStream_t s) {
            if (b.box)
                KLAUNCH((k_trace_residual<K, RT, true>), dim3(b.nbf), dim3(kFaceThreads), 0, s,
                        b, x, gv, rin, partials, stride, skip);
            else
                KLAUNCH((k_trace_residual<K, RT, false>), dim3(b.nbf), dim3(kFaceThreads), 0, s,
                        b, x, gv, rin, partials, stride, skip);
            return hipGetLastError();
        }
    };
};
template <typename T> struct RunK1 {
    template <int K, bool SCHED, bool BND>
    static void go(const Batch &b, const T *r, const T *rh, const T *pin, const T *vin, T *pout,
                   T *vout, KrylovState *ks, const KrylovBufs &kb, hipStream_t s) {
        KLAUNCH((k_bicg_k1<K, T, SCHED, BND>), dim3(b.nbf), dim3(kFaceThreads), 0, s, b, r, rh,
                pin, vin, pout, vout, ks, kb.P3, kb.P1, kb.stride);
    }
    template <int K> struct F {
        static hipError_t run(const Batch &b, const T *r, const T *rh, const T *pin,
                              const T *vin, T *pout, T *vout, KrylovState *ks,
                              const KrylovBufs &kb, hipStream_t s) {
            if (kb.sched && b.box) go<K, true, true>(b, r, rh, pin, vin, pout, vout, ks, kb, s);
            else if (kb.sched) go<K, true, false>(b, r, rh, pin, vin, pout, vout, ks, kb, s);
            else if (b.box) go<K, false, true>(b, r, rh, pin, vin, pout, vout, ks, kb, s);
            else go<K, false, false>(b, r, rh, pin, vin, pout, vout, ks, kb, s);
            return hipGetLastError();
        }
    };
};
template <typename T> struct RunRefineK1 {
    template <int K> struct F {
        static hipError_t run(const Batch &b, const T *rin, T *r, T *rh, T *p, T *v, T *d,
                              KrylovState *ks, const double *partials, int pstride,
                              double refine_rtol, double inner_rtol, const KrylovBufs &kb,
                              hipStream_t s) {
            if (b.box)
                KLAUNCH((k_refine_k1<K, T, true>), dim3(b.nbf), dim3(kFaceThreads), 0, s, b, rin,
                        r, rh, p, v, d, ks, partials, pstride, refine_rtol, inner_rtol, kb.P1,
                        kb.stride);
            else
                KLAUNCH((k_refine_k1<K, T, false>), dim3(b.nbf), dim3(kFaceThreads), 0, s, b,
                        rin, r, rh, p, v, d, ks, partials, pstride, refine_rtol, inner_rtol,
                        kb.P1, kb.stride);
            return hipGetLastError();
        }
    };
};
template <typename T> struct RunK2 {
    template <int K, bool SCHED, bool BND>
    static void go(const Batch &b, const T *r, const T *v, const T *rh, T *t, KrylovState *ks,
                   const KrylovBufs &kb, hipStream_t s) {
        KLAUNCH((k_bicg_k2<K, T, SCHED, BND>), dim3(b.nbf), dim3(kFaceThreads), 0, s, b, r, v,
                rh, t, ks, kb.P1, kb.P2, kb.stride);
    }
    template <int K> struct F {
        static hipError_t run(const Batch &b, const T *r, const T *v, const T *rh, T *t,
                              KrylovState *ks, const KrylovBufs &kb, hipStream_t s) {
            if (kb.sched && b.box) go<K, true, true>(b, r, v, rh, t, ks, kb, s);
            else if (kb.sched) go<K, true, false>(b, r, v, rh, t, ks, kb, s);
            else if (b.box) go<K, false, true>(b, r, v, rh, t, ks, kb, s);
            else go<K, false, false>(b, r, v, rh, t, ks, kb, s);
            return hipGetLastError();
        }
    };
};
template <typename T> struct RunK1F {
    template <int K, bool SCHED, bool BND>
    static void go(const Batch &b, const T *rin, const T *t, const T *rh, const T *pin,
                   const T *vin, T *pout, T *vout, T *r, T *d, KrylovState *ks,
                   const KrylovBufs &kb, hipStream_t s) {
        KLAUNCH((k_bicg_k1f<K, T, SCHED, BND>), dim3(b.nbf), dim3(kFaceThreads), 0, s, b, rin,
                t, rh, pin, vin, pout, vout, r, d, ks, kb.P2, kb.P1, kb.stride);
    }
    template <int K> struct F {
        static hipError_t run(const Batch &b, const T *rin, const T *t, const T *rh,
                              const T *pin, const T *vin, T *pout, T *vout, T *r, T *d,
                              KrylovState *ks, const KrylovBufs &kb, hipStream_t s) {
            if (kb.sched && b.box)
                go<K, true, true>(b, rin, t, rh, pin, vin, pout, vout, r, d, ks, kb, s);
            else if (kb.sched)
                go<K, true, false>(b, rin, t, rh, pin, vin, pout, vout, r, d, ks, kb, s);
            else if (b.box)
                go<K, false, true>(b, rin, t, rh, pin, vin, pout, vout, r, d, ks, kb, s);
            else
                go<K, false, false>(b, rin, t, rh, pin, vin, pout, vout, r, d, ks, kb, s);
            return hipGetLastError();
        }
    };
};
template <int K> struct RunDiag {
    static hipError_t run(const Geom &g, const Batch &b, const double *q, double *partials,
                          int stride, hipStream_t s) {
        KLAUNCH(k_diag<K>, dim3(b.nbd), dim3(64 * K), 0, s, q, g, b, partials,
                           stride);
        return hipGetLastError();
    }
};

}  // namespace

int member_tiles(int nx, int ny) { return ((nx + kTX - 1) / kTX) * ((ny + kTY - 1) / kTY); }

int member_face_blocks(int nx, int ny, int fgrid, int tpb) {
    // a multiple of 8 blocks when there are enough tiles, so that every XCD
    // gets the same number of blocks
    const int tiles = member_tiles(nx, ny);
    const int want = tpb > 0 ? (tiles + tpb - 1) / tpb : tiles;
    const int n = std::min(want, std::min(fgrid, kMaxLaunchGrid));
    return n >= 8 ? n & ~7 : n;
}

int member_elem_blocks(int nel, int K, int egrid) {
    const size_t n = (size_t)6 * K * nel;
    return (int)std::min<size_t>(grid1(n, 256 * 4), (size_t)std::min(egrid, kMaxLaunchGrid));
}

int member_vol_blocks(int nel) { return (int)grid1(nel, 64); }

int member_diag_blocks(int nel) { return (int)std::min<unsigned>(grid1(nel, 64), 1024u); }

hipError_t launch_nl(const Geom &g, const Batch &b, const double *q, const Comb &comb,
                     bool scale_dt, hipStream_t s, bool fp32) {
    return dispatch<RunNL>(g.K, g, b, q, comb, scale_dt, fp32, s);
}

hipError_t launch_combine(const Comb &comb, size_t n, hipStream_t s) {
    KLAUNCH(k_combine, dim3(grid1(n, 256)), dim3(256), 0, s, comb, n);
    return hipGetLastError();
}

hipError_t launch_linear_residual(const Geom &g, const Batch &b, const double *Q,
                                  const double *qhat, double *out, hipStream_t s) {
    return dispatch<RunLinres>(g.K, g, b, Q, qhat, out, s);
}

hipError_t launch_local_apply(const Geom &g, const Batch &b, const double *R, double *Z,
                              hipStream_t s) {
    return dispatch<RunLocal>(g.K, b, R, Z, s);
}

int local_lp_kw(bool bf16) { return bf16 ? LpMfma<__bf16>::KW : LpMfma<float>::KW; }

hipError_t launch_local_lp(const Geom &g, const Batch &b, const double *R, const double *qhat,
                           double aii, double *out, bool bf16, int ndc, hipStream_t s,
                           const KrylovState *ks, const double *partials, int stride,
                           StageStatus *status) {
    if (ndc < 1 || ndc > (bf16 ? 3 : 2)) return hipErrorInvalidValue;
    return dispatch<RunLocalLp>(g.K, g, b, R, qhat, aii, out, bf16, ndc, ks, partials, stride,
                                status, s);
}

hipError_t launch_trace_rhs(const Geom &g, const Batch &b, const double *Z, double *gvec,
                            hipStream_t s, KrylovState *begin, double *x, double *xprev,
                            double xcoef) {
    return dispatch<RunTraceRhs>(g.K, g, b, Z, gvec, begin, x, xprev, xcoef, s);
}

hipError_t launch_recover(const Geom &g, const Batch &b, const double *Z, const double *qhat,
                          double *Q, hipStream_t s, const KrylovState *ks,
                          const double *partials, int stride, StageStatus *status) {
    return dispatch<RunRecover>(g.K, b, Z, qhat, Q, ks, partials, stride, status, s);
}

#define IMEXHDG_KRYLOV_LAUNCHERS(T)                                                            \
    hipError_t launch_trace_residual(const Geom &g, const Batch &b, const double *x,          \
                                     const double *gvec, T *rin, double *partials,            \
                                     int stride, const KrylovState *skip, hipStream_t s) {    \
        return dispatch<RunTraceResidual<T>::template F>(g.K, b, x, gvec, rin, partials,      \
                                                         stride, skip, s);                    \
    }                                                                                          \
    hipError_t launch_bicg_init(const Geom &g, const Batch &b, const T *rin, T *r, T *rh,     \
                                T *p, T *v, T *d, KrylovState *ks, double tol2,               \
                                const KrylovBufs &kb, hipStream_t s) {                        \
        KLAUNCH(k_bicg_init<T>, dim3(b.nbe), dim3(256), 0, s, b, g.K, rin, r, rh, \
                           p, v, d, ks, tol2, kb.P3, kb.stride);                              \
        return hipGetLastError();                                                              \
    }                                                                                          \
    hipError_t launch_bicg_k1(const Geom &g, const Batch &b, const T *r, const T *rh,         \
                              const T *pin, const T *vin, T *pout, T *vout, KrylovState *ks,  \
                              const KrylovBufs &kb, hipStream_t s) {                          \
        return dispatch<RunK1<T>::template F>(g.K, b, r, rh, pin, vin, pout, vout, ks, kb,    \
                                              s);                                             \
    }                                                                                          \
    hipError_t launch_bicg_k2(const Geom &g, const Batch &b, const T *r, const T *v,          \
                              const T *rh, T *t, KrylovState *ks, const KrylovBufs &kb,       \
                              hipStream_t s) {                                                \
        return dispatch<RunK2<T>::template F>(g.K, b, r, v, rh, t, ks, kb, s);                \
    }                                                                                          \
    hipError_t launch_bicg_k1f(const Geom &g, const Batch &b, const T *rin, const T *t,       \
                               const T *rh, const T *pin, const T *vin, T *pout, T *vout,     \
                               T *r, T *d, KrylovState *ks, const KrylovBufs &kb,             \
                               hipStream_t s) {                                               \
        return dispatch<RunK1F<T>::template F>(g.K, b, rin, t, rh, pin, vin, pout, vout, r, d,\
                                               ks, kb, s);                                    \
    }                                                                                          \
    hipError_t launch_axpy(double *y, const T *x, double a, size_t n, hipStream_t s) {        \
        KLAUNCH(k_axpy<T>, dim3(grid1(n, 256)), dim3(256), 0, s, y, x, a, n);     \
        return hipGetLastError();                                                              \
    }                                                                                          \
    hipError_t launch_refine_k1(const Geom &g, const Batch &b, const T *rin, T *r, T *rh,     \
                                T *p, T *v, T *d, KrylovState *ks, const double *partials,    \
                                int stride, double refine_rtol, double inner_rtol,            \
                                const KrylovBufs &kb, hipStream_t s) {                        \
        return dispatch<RunRefineK1<T>::template F>(g.K, b, rin, r, rh, p, v, d, ks, partials, \
                                                    stride, refine_rtol, inner_rtol, kb, s);  \
    }                                                                                          \
    hipError_t launch_axpy_guarded(const Geom &g, const Batch &b, double *y, const T *x,      \
                                   KrylovState *ks, hipStream_t s) {                          \
        KLAUNCH(k_axpy_guarded<T>, dim3(b.nbe), dim3(256), 0, s, b, g.K, y, x, ks); \
        return hipGetLastError();                                                              \
    }

IMEXHDG_KRYLOV_LAUNCHERS(double)
IMEXHDG_KRYLOV_LAUNCHERS(float)
#undef IMEXHDG_KRYLOV_LAUNCHERS

hipError_t launch_diag(const Geom &g, const Batch &b, const double *q, double *partials,
                       int stride, hipStream_t s) {
    return dispatch<RunDiag>(g.K, g, b, q, partials, stride, s);
}

// ------------------------------------------------------------ scratch
// Device memory of the allocation-free stage solve.  Each GPU the library
// runs on holds its own copy at its own address until the process ends.
// Host code never uses the array's name as an address (on the host it is
// a stand-in, not device memory): it uses the pointer that
// hipGetSymbolAddress returned on that device.
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t scratch_init(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
    return hipSuccess;
}

__global__ void k_zero(uint32_t *p, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

hipError_t launch_zero(void *p, size_t n32, hipStream_t s) {
    if (n32 == 0) return hipSuccess;
    KLAUNCH(k_zero, dim3((unsigned)((n32 + 255) / 256)), dim3(256), 0, s, (uint32_t *)p, n32);
    return hipGetLastError();
}

void *scratch_base(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[dev];
}

int state_in_blocks(int nel, int K, int cap) {
    return (int)std::max<unsigned>(1u, std::min<unsigned>(grid1((size_t)nel * K * K, 256),
                                                          (unsigned)cap));
}

hipError_t launch_state_in(const void *src, bool f32, bool depth, double g, double H,
                           int nel, int K, double *dst, double *partials, int blocks,
                           hipStream_t s, int bx, int nxp, const double *pBn) {
    const double phiB = g * H;
    if (f32)
        KLAUNCH(k_state_in<float>, dim3(blocks), dim3(256), 0, s, (const float *)src,
                depth ? 1 : 0, g, H, phiB, pBn, nel, K * K, dst, partials, blocks, bx, nxp);
    else
        KLAUNCH(k_state_in<double>, dim3(blocks), dim3(256), 0, s, (const double *)src,
                depth ? 1 : 0, g, H, phiB, pBn, nel, K * K, dst, partials, blocks, bx, nxp);
    return hipGetLastError();
}

template <int K> struct RunDgVar {
    static hipError_t run(const Geom &g, const Batch &b, const double *q, const double *pB,
                          const Comb &comb, bool scale_dt, const double *R, double *out,
                          double cst, double *partials, int stride, bool lin, hipStream_t s) {
        if (lin)
            KLAUNCH((k_dg_var<K, true>), dim3(b.nbv), dim3(64 * K), 0, s, q, pB, g, b, comb,
                    scale_dt ? 1 : 0, R, out, cst, partials, stride);
        else
            KLAUNCH((k_dg_var<K, false>), dim3(b.nbv), dim3(64 * K), 0, s, q, pB, g, b, comb,
                    scale_dt ? 1 : 0, R, out, cst, partials, stride);
        return hipGetLastError();
    }
};

hipError_t launch_nl_var(const Geom &g, const Batch &b, const double *q, const double *pB,
                         const Comb &comb, bool scale_dt, hipStream_t s) {
    return dispatch<RunDgVar>(g.K, g, b, q, pB, comb, scale_dt, nullptr, nullptr, 0.0,
                              nullptr, 0, false, s);
}

hipError_t launch_stage_res_var(const Geom &g, const Batch &b, const double *Q,
                                const double *pB, const double *R, double aii, double *out,
                                double *partials, int stride, hipStream_t s) {
    Comb none{};
    return dispatch<RunDgVar>(g.K, g, b, Q, pB, none, false, R, out, aii, partials, stride,
                              true, s);
}

hipError_t launch_put(double *p, double v, hipStream_t s) {
    KLAUNCH(k_put_f64, dim3(1), dim3(1), 0, s, p, v);
    return hipGetLastError();
}

hipError_t launch_bc_fill(const Geom &g, const Batch &b, double *q, const double *tstep,
                          double toff, double *tnext, const Vortex &vx, hipStream_t s) {
    KLAUNCH(k_bc_fill, dim3(b.nbv), dim3(64 * g.K), 0, s, q, g, b, tstep, toff, tnext, vx);
    return hipGetLastError();
}

}  // namespace imexhdg
