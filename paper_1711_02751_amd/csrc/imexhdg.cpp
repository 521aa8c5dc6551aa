// C ABI of the IMEX HDG-DG step: context, workspace, stage orchestration.
//
// The engine runs a batch of members (independent periodic meshes sharing
// the degree, the physical constants, the scheme and the solver settings):
// a context is the batch of one member, an ensemble the batch of many.
// Every launch covers all members; see kernels.hpp.
#include "../../include/imexhdg.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstddef>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "element.hpp"
#include "kernels.hpp"

using namespace imexhdg;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

#define HIP_TRY(expr)                                                            \
    do {                                                                         \
        hipError_t _e = (expr);                                                  \
        if (_e != hipSuccess)                                                    \
            return fail(IMEXHDG_E_DEVICE, std::string(#expr) + ": " +            \
                                              hipGetErrorString(_e));            \
    } while (0)

// IMEX tableau: explicit A (strictly lower), implicit At (SDIRK), b, bt.
struct Tableau {
    int s = 0;
    std::vector<double> A, At, b, bt;   // s x s row-major, s
    double a(int i, int j) const { return A[i * s + j]; }
    double at(int i, int j) const { return At[i * s + j]; }
};

Tableau make_tableau(int scheme) {
    Tableau t;
    if (scheme == IMEXHDG_SCHEME_ARS232) {
        // ARS(2,3,2): gamma = 1 - 1/sqrt(2), delta = -2 sqrt(2)/3
        const double g = 1.0 - 1.0 / std::sqrt(2.0), d = -2.0 * std::sqrt(2.0) / 3.0;
        t.s = 3;
        t.A = {0, 0, 0, g, 0, 0, d, 1 - d, 0};
        t.At = {0, 0, 0, 0, g, 0, 0, 1 - g, g};
        t.b = {0, 1 - g, g};
        t.bt = {0, 1 - g, g};
    } else {
        // ARS(4,4,3), both parts stiffly accurate
        t.s = 5;
        t.A = {0, 0, 0, 0, 0,  0.5, 0, 0, 0, 0,  11.0 / 18, 1.0 / 18, 0, 0, 0,
               5.0 / 6, -5.0 / 6, 0.5, 0, 0,  0.25, 1.75, 0.75, -1.75, 0};
        t.At = {0, 0, 0, 0, 0,  0, 0.5, 0, 0, 0,  0, 1.0 / 6, 0.5, 0, 0,
                0, -0.5, 0.5, 0.5, 0,  0, 1.5, -1.5, 0.5, 0.5};
        t.b = {0.25, 1.75, 0.75, -1.75, 0};
        t.bt = {0, 1.5, -1.5, 0.5, 0.5};
    }
    return t;
}

// A linear combination over the step's vectors.  Vector ids:
//   QN (q^n), NLV+j (dt NL_j), QV+j (Q_j), RV+j (Res0_j), SELF (kernel result).
// The NL kernel returns dt NL (the member's dt), so no coefficient holds dt
// and one plan serves members with different time steps.
enum { QN = 0, NLV = 1, QV = 17, RV = 33, SELF = 49 };
struct Term { int id; double coef; };
using Plan = std::vector<Term>;

void add(Plan &p, int id, double c) {
    if (c == 0.0) return;
    for (Term &t : p)
        if (t.id == id) { t.coef += c; return; }
    p.push_back({id, c});
}

void cleanup(Plan &p) {
    Plan out;
    for (const Term &t : p)
        if (t.coef != 0.0) out.push_back(t);
    p.swap(out);
}

// Element operators of one (hx, hy, dt) on the device.
struct OpSet {
    double hx = 0, hy = 0, dt = 0;
    double *Ainv = nullptr, *W = nullptr, *G = nullptr, *Gh = nullptr, *Px = nullptr,
           *Py = nullptr;
    float *Ghf = nullptr;
    void *Alp = nullptr;      // reduced-precision A^-1 fragments (launch_local_lp)
    // boundary-row corrections of G and Ghat (bounded meshes), see Member
    double *dG = nullptr, *dGh = nullptr;
    float *dGhf = nullptr;
};

// nx, ny, nel: the device mesh (a bounded one padded by two ghost columns
// and rows); bx, by: the bounded mesh's own elements (0: periodic).
struct MemberHost {
    int nx = 0, ny = 0, nel = 0;
    int bx = 0, by = 0;
    double hx = 0, hy = 0;
    double Lx = 0, Ly = 0, dt = 0;
    size_t N = 0, T = 0, vo = 0, to = 0;
    int op = 0;
};

}  // namespace

struct imexhdg_ctx {
    imexhdg_config cfg{};             // shared settings (the first member's config)
    int nm = 1;
    std::vector<MemberHost> mh;
    std::vector<Member> mtab;         // host copy of the device member table
    Member *dmem = nullptr;
    Batch bt{};
    int fgrid = 1024, egrid = 1024;   // launch-geometry caps
    int ftpb = 0;                     // > 0: face blocks per member = tiles / ftpb (ensembles)
    int pstride = 0;                  // stride of every partial-sum array
    hipStream_t stream = nullptr;
    int device = 0;
    bool own_ws = false;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    LGL ref;
    Geom geom{};
    std::vector<OpSet> ops;
    Tableau tab;
    double aii = 0.0;
    size_t N = 0, T = 0, nnodes = 0;  // over all members
    // device buffers; the state lives in a ring of three buffers, q is
    // qbuf[cur] and a step from qbuf[a] writes qbuf[(a + 1) % 3]
    double *qbuf[3] = {nullptr, nullptr, nullptr};
    int cur = 0;
    double *q = nullptr, *Z = nullptr, *save = nullptr;   // save: autotuner's copy of q
    const double *qin = nullptr;      // q^n of the step being enqueued
    std::vector<double *> NLb, Qb, Rb;
    double *x = nullptr, *gv = nullptr;
    double *xp = nullptr;             // trace of the stage solve before the last
    std::vector<double> xcoef;        // per stage: trace-guess extrapolation coefficient
    double *xsave = nullptr;          // autotuner's copy of the trace guess
    // inner-solve vectors, FP64 or FP32 (every precision but IMEXHDG_PREC_FP64)
    bool mixed = false;
    // reduced-precision local solves (IMEXHDG_PREC_FP32 / _BF16) with
    // lp_ndc defect-correction sweeps, and the FP32 DG residual
    bool lp = false, lp_bf16 = false, nl32 = false;
    int lp_ndc = 0;
    void *rin = nullptr, *kr[2] = {nullptr, nullptr}, *krh = nullptr,
         *kp[2] = {nullptr, nullptr}, *kv[2] = {nullptr, nullptr}, *kt = nullptr,
         *kd = nullptr;
    KrylovState *ks = nullptr;        // [nm]
    KrylovBufs kb{};
    // bounded mesh: boundary states of the exact vortex at the stage times;
    // tstep[a] is the step count of the state in qbuf[a] (device, so that
    // captured steps read it), tcur the ring position of the step being
    // enqueued, cst[i] the abscissa of stage i
    bool box = false, wall = false;
    Vortex vx{};
    double *tstep = nullptr;
    int tcur = 0;
    std::vector<double> cst;
    // variable depth: nodal phi_B (device), the host depth for state
    // conversions, the stage residual and correction, their partial sums
    bool vdepth = false;
    double *pB = nullptr, *dres = nullptr, *ddel = nullptr, *dcpart = nullptr;
    double *hcpart = nullptr;         // pinned host mirror of dcpart
    int nvb = 0;
    std::vector<double> hB;
    int64_t dcorr = 0;
    double *dpart = nullptr;          // [5][pstride] residual / diagnostics partials
    // host mirrors
    KrylovState *hks = nullptr;
    double *hpart = nullptr;
    bool have_state = false;
    std::vector<bool> member_set;
    // plans: after stage i the NL kernel writes plan_out[i]
    std::vector<Plan> plans;
    std::vector<bool> store_nl;
    // counters
    int64_t steps = 0, kiters = 0, solves = 0, sweeps = 0;
    double step_ms = 0.0;             // host wall time inside step calls since set_state
    double last_relres = 0.0, max_relres = 0.0;
    int iter_pred = 0;      // inner iterations of the last first sweep
    int dbg_brk = 0;        // debug (IMEXHDG_DEBUG_BREAKDOWN_AT): host-driven inner solves
                            // take the breakdown branch in this K1f iteration (1-based)
    // fixed-schedule stepping: sweeps and inner-iteration budget per sweep,
    // what the last host-driven solves needed, one graph per ring position
    int sched_sweeps = 0, sched_budget[kMaxSweeps] = {};
    int margin = 2;                   // schedule slack: +2 per redone step, -1 per clean window
    int learn_sweeps = 0, learn_iters[kMaxSweeps] = {};
    int win_sweeps = 0, win_iters[kMaxSweeps] = {};   // graph steps since capture
    int64_t win_steps = 0;
    bool cold = true;                 // next step starts from a fresh trace guess
    bool gready = false;
    hipStream_t gstream = nullptr;    // capture stream
    hipGraphExec_t gexec[3] = {nullptr, nullptr, nullptr};
    hipEvent_t gev[3] = {nullptr, nullptr, nullptr};
    StageStatus *dstat = nullptr;     // [3][s][nm], device
    StageStatus *hstat = nullptr;     // [3][s][nm], pinned host mirror
    int64_t graph_steps = 0, redos = 0, captures = 0;
    // event profiler
    int prof_target = -2;
    std::vector<hipEvent_t> ev0, ev1;
    std::vector<int> ev_id;
    int ev_used = 0;
    double prof_ms[IMEXHDG_K_COUNT] = {};
    std::vector<float> prof_dur[IMEXHDG_K_COUNT];   // per-launch times (ms) of the timed classes
    int64_t prof_n[IMEXHDG_K_COUNT] = {};
};

struct imexhdg_ens {
    imexhdg_ctx *c = nullptr;
};

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Device mesh of a config: a bounded rectangle is padded by two ghost
// columns and rows.
void device_dims(const imexhdg_config &c, int &nx, int &ny) {
    const int pad = c.boundary != IMEXHDG_BOUNDARY_PERIODIC ? 2 : 0;
    nx = c.nx + pad;
    ny = c.ny + pad;
}

// Boundary-row corrections (bounded meshes): per side [W, E, S, N] four
// entries, one per local face of the side's real element (entry 0 its
// boundary face, the self slot of the row), each a 3K x 3K matrix packed
// like one slot of G: frag[4 side + e][mb][kk][lane] = D[16 mb + lane % 16]
// [4 kk + lane / 16], KS = ceil(3K / 4) k steps, zero past 3K.
constexpr int kSideEntries = 4;
size_t side_frag_count(int K) {
    const int B3 = 3 * K, KS = (B3 + 3) / 4, NMB = (B3 + 15) / 16;
    return (size_t)4 * kSideEntries * NMB * KS * 64;
}

std::vector<double> pack_sides(const std::vector<double> (&D)[4][kSideEntries], int K) {
    const int B3 = 3 * K, KS = (B3 + 3) / 4, NMB = (B3 + 15) / 16;
    std::vector<double> f(side_frag_count(K), 0.0);
    for (int sd = 0; sd < 4; ++sd)
        for (int e = 0; e < kSideEntries; ++e)
            for (int mb = 0; mb < NMB; ++mb)
                for (int u = 0; u < KS; ++u)
                    for (int l = 0; l < 64; ++l) {
                        const int row = 16 * mb + l % 16, col = 4 * u + l / 16;
                        if (row < B3 && col < B3)
                            f[((((size_t)sd * kSideEntries + e) * NMB + mb) * KS + u) * 64 + l] =
                                D[sd][e][(size_t)row * B3 + col];
                    }
    return f;
}

// A boundary face has one element and the imaginary neighbour (Sec. 4.3,
// eqs. reflection / reflectionBC; the exact-solution data of Sec. 6.1 enter
// the same way).  Its conservation condition keeps 2 tau I and the real
// element's C W; the neighbour adds C_g Q_g at the face nodes, C_g Q =
// F_L(Q) . n_g + tau Q with n_g = -n the neighbour's outward normal.
//   * Exact-solution data: Q_g is data (the ghost element holds it there,
//     so the right-hand side kernel adds C_g Q_g as for an interior face).
//   * Wall: Q_g = R E Q, the reflection R of the real element's face values
//     E Q, Q = Z - W qhat: the right-hand side gains C_g R E Z (the ghost
//     holds R E Z) and the row gains + C_g R E W over the real element's
//     four faces.
// The interior row the face kernels apply has instead C_g' W_g' of the ghost
// element at the face (its other faces hold zero), so every side's entry 0
// (the self slot) removes it, -S(f_g, f_g) with f_g the ghost's local face
// (W: the ghost lies west, its east face 1; E: 0; S: 3; N: 2), and with a
// wall entries 0..3 add C_g R E W for the real element's faces in the order
// side_faces below.  With the interior block-Jacobi inverse P^-1 kept as
// the boundary rows' preconditioner, dGh = P^-1 dG.
void boundary_deltas(const StageOperators &op, int K, bool wall,
                     std::vector<double> (&dG)[4][kSideEntries],
                     std::vector<double> (&dGh)[4][kSideEntries]) {
    const int B3 = 3 * K, NT = 12 * K, k = K - 1;
    const int ghost_face[4] = {1, 0, 3, 2};
    const int real_face[4] = {0, 1, 2, 3};   // the boundary face as a face of the real element
    const double nrm[4][2] = {{-1, 0}, {1, 0}, {0, -1}, {0, 1}};   // its outward normal
    // the real element's faces in entry order (entry 0: the boundary face)
    const int side_faces[4][4] = {{0, 1, 2, 3}, {1, 0, 2, 3}, {2, 0, 1, 3}, {3, 0, 1, 2}};
    auto face_node = [k](int f, int j, int &a, int &b) {
        if (f == 0) { a = 0; b = j; }
        else if (f == 1) { a = k; b = j; }
        else if (f == 2) { a = j; b = 0; }
        else { a = j; b = k; }
    };
    for (int sd = 0; sd < 4; ++sd) {
        for (int e = 0; e < kSideEntries; ++e) dG[sd][e].assign((size_t)B3 * B3, 0.0);
        const int fg = ghost_face[sd];
        for (int r = 0; r < B3; ++r)
            for (int cc = 0; cc < B3; ++cc)
                dG[sd][0][(size_t)r * B3 + cc] = -op.S[(size_t)(fg * B3 + r) * NT + fg * B3 + cc];
        if (wall) {
            const double gx = -nrm[sd][0], gy = -nrm[sd][1];   // the neighbour's normal
            const int refl = sd < 2 ? 1 : 2;                    // the normal momentum
            for (int e = 0; e < kSideEntries; ++e) {
                const int f = side_faces[sd][e];
                for (int j = 0; j < K; ++j) {
                    int a, b;
                    face_node(real_face[sd], j, a, b);
                    // R E W restricted to face f's traces: rows (c, j), cols (c', j')
                    double rew[3][3 * kMaxK];
                    for (int c = 0; c < 3; ++c)
                        for (int col = 0; col < B3; ++col) {
                            const int v = c * K * K + b * K + a;
                            const double w = op.W[(size_t)v * NT + f * B3 + col];
                            rew[c][col] = c == refl ? -w : w;
                        }
                    for (int col = 0; col < B3; ++col) {
                        const double p = rew[0][col], U = rew[1][col], V = rew[2][col];
                        const double cg[3] = {op.tau * p + gx * U + gy * V,
                                              op.phiB * gx * p + op.tau * U,
                                              op.phiB * gy * p + op.tau * V};
                        for (int c = 0; c < 3; ++c)
                            dG[sd][e][(size_t)(c * K + j) * B3 + col] += cg[c];
                    }
                }
            }
        }
        const std::vector<double> &P = sd < 2 ? op.Pxinv : op.Pyinv;
        for (int e = 0; e < kSideEntries; ++e) {
            dGh[sd][e].assign((size_t)B3 * B3, 0.0);
            for (int r = 0; r < B3; ++r)
                for (int m = 0; m < B3; ++m) {
                    const double pv = P[(size_t)r * B3 + m];
                    for (int cc = 0; cc < B3; ++cc)
                        dGh[sd][e][(size_t)r * B3 + cc] += pv * dG[sd][e][(size_t)m * B3 + cc];
                }
        }
    }
}

// Sizes of the packed matrix-core operands of the trace row blocks.
size_t frag_count(int K) {
    const int B3 = 3 * K, KS = (B3 + 3) / 4, NKK = 7 * KS, NMB = (B3 + 15) / 16;
    return (size_t)2 * NMB * NKK * 64;
}

// Pack the 7-slot row blocks of G for x- and y-faces into the A-operand
// order of the 16x16x4 matrix-core step: frag[dir][mb][kk][lane] holds row
// 16 mb + lane % 16 (face row (c, j)) and column 4 (kk mod KS) + lane / 16
// (c' K + j') of slot kk / KS, KS = ceil(3K / 4) k-steps per slot; rows and
// columns past 3K are zero.
std::vector<double> pack_frags(const std::vector<double> &Gx, const std::vector<double> &Gy,
                               int K) {
    const int B3 = 3 * K, KS = (B3 + 3) / 4, NKK = 7 * KS, NMB = (B3 + 15) / 16;
    std::vector<double> f(frag_count(K), 0.0);
    for (int d = 0; d < 2; ++d) {
        const std::vector<double> &G = d ? Gy : Gx;
        for (int mb = 0; mb < NMB; ++mb)
            for (int kk = 0; kk < NKK; ++kk)
                for (int l = 0; l < 64; ++l) {
                    const int row = 16 * mb + l % 16;
                    const int slot = kk / KS, col = 4 * (kk % KS) + l / 16;
                    if (row >= B3 || col >= B3) continue;
                    f[(((size_t)d * NMB + mb) * NKK + kk) * 64 + l] =
                        G[(size_t)slot * B3 * B3 + (size_t)row * B3 + col];
                }
    }
    return f;
}

// Local matrix-core operand of an nr x nc row-major matrix M:
// frag[mb][kk][lane] = M[16 mb + lane % 16][4 kk + lane / 16], zero past M.
size_t local_frag_count(int nr, int nc) {
    return (size_t)((nr + 15) / 16) * ((nc + 3) / 4) * 64;
}

std::vector<double> pack_local(const std::vector<double> &M, int nr, int nc) {
    const int NMB = (nr + 15) / 16, KS = (nc + 3) / 4;
    std::vector<double> f(local_frag_count(nr, nc), 0.0);
    for (int mb = 0; mb < NMB; ++mb)
        for (int kk = 0; kk < KS; ++kk)
            for (int l = 0; l < 64; ++l) {
                const int row = 16 * mb + l % 16, col = 4 * kk + l / 16;
                if (row < nr && col < nc)
                    f[((size_t)mb * KS + kk) * 64 + l] = M[(size_t)row * nc + col];
            }
    return f;
}

// A^-1 fragments of the reduced-precision local solve (launch_local_lp):
// frag[mb][kk][lane][v] = M[16 mb + lane % 16][kw kk + (kw / 4)(lane / 16) + v],
// zero past the n x n matrix; FP32 values, or BF16 bit patterns rounded to
// nearest even.
size_t lp_frag_count(int n, bool bf16) {
    const int kw = local_lp_kw(bf16);
    return (size_t)((n + 15) / 16) * ((n + kw - 1) / kw) * 64 * (kw / 4);
}

size_t lp_frag_bytes(int n, bool bf16) { return lp_frag_count(n, bf16) * (bf16 ? 2 : 4); }

uint16_t bf16_bits(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest, ties to even (finite values)
    return (uint16_t)(u >> 16);
}

std::vector<uint8_t> pack_lp(const std::vector<double> &M, int n, bool bf16) {
    const int kw = local_lp_kw(bf16), vpl = kw / 4;
    const int NMB = (n + 15) / 16, KS = (n + kw - 1) / kw;
    std::vector<uint8_t> out(lp_frag_bytes(n, bf16), 0);
    size_t idx = 0;
    for (int mb = 0; mb < NMB; ++mb)
        for (int kk = 0; kk < KS; ++kk)
            for (int l = 0; l < 64; ++l)
                for (int v = 0; v < vpl; ++v, ++idx) {
                    const int row = 16 * mb + l % 16, col = kw * kk + vpl * (l / 16) + v;
                    const float x = (row < n && col < n) ? (float)M[(size_t)row * n + col] : 0.f;
                    if (bf16) {
                        const uint16_t b = bf16_bits(x);
                        std::memcpy(&out[idx * 2], &b, 2);
                    } else {
                        std::memcpy(&out[idx * 4], &x, 4);
                    }
                }
    return out;
}

// Worst-case partial-sum stride of a batch: every class at its largest caps.
int partial_stride(const std::vector<imexhdg_config> &cf) {
    int64_t f = 0, e = 0, d = 0;
    for (const imexhdg_config &c : cf) {
        int nx, ny;
        device_dims(c, nx, ny);
        const int nel = nx * ny;
        f += member_face_blocks(nx, ny, kMaxLaunchGrid);
        e += member_elem_blocks(nel, c.degree + 1, kMaxLaunchGrid);
        d += member_diag_blocks(nel);
    }
    const int64_t m = std::max<int64_t>(std::max(f, e), std::max<int64_t>(d, 1));
    return (int)((m + 63) / 64 * 64);
}

// Distinct (hx, hy, dt) of a batch.
int count_opsets(const std::vector<imexhdg_config> &cf) {
    std::vector<std::vector<double>> seen;
    for (const imexhdg_config &c : cf) {
        const std::vector<double> key = {c.Lx / c.nx, c.Ly / c.ny, c.dt};
        if (std::find(seen.begin(), seen.end(), key) == seen.end()) seen.push_back(key);
    }
    return (int)seen.size();
}

struct Layout {
    size_t N = 0, T = 0, total = 0;
    int s = 0, nops = 0, pstride = 0;
};

Layout layout_of(const std::vector<imexhdg_config> &cf) {
    Layout L{};
    const imexhdg_config &c0 = cf[0];
    const size_t K = (size_t)c0.degree + 1;
    for (const imexhdg_config &c : cf) {
        int nx, ny;
        device_dims(c, nx, ny);
        const size_t nel = (size_t)nx * ny;
        L.N += 3 * K * K * nel;
        L.T += 6 * K * nel;
    }
    const size_t n_loc = 3 * K * K, n_tr = 12 * K;
    L.s = (c0.scheme == IMEXHDG_SCHEME_ARS443) ? 5 : 3;
    L.nops = count_opsets(cf);
    L.pstride = partial_stride(cf);
    const size_t nm = cf.size();
    size_t t = 0;
    t += 5 * align256(L.N * 8);                       // q ring (3), Z, save
    t += 3 * (size_t)L.s * align256(L.N * 8);          // NL, Q, R per stage
    const size_t isz = (c0.precision != IMEXHDG_PREC_FP64) ? 4 : 8;
    t += 4 * align256(L.T * 8);                        // FP64 trace vectors
    t += 10 * align256(L.T * isz);                     // inner-solve vectors
    if (c0.precision == IMEXHDG_PREC_FP32 || c0.precision == IMEXHDG_PREC_BF16)
        t += (size_t)L.nops * align256(lp_frag_bytes((int)n_loc,
                                                     c0.precision == IMEXHDG_PREC_BF16));
    t += (size_t)L.nops * (align256(local_frag_count((int)n_loc, (int)n_loc) * 8) +
                           align256(local_frag_count((int)n_loc, (int)n_tr) * 8) +
                           2 * align256(frag_count((int)K) * 8) +
                           align256(frag_count((int)K) * 4) + 2 * align256(9 * K * K * 8) +
                           2 * align256(side_frag_count((int)K) * 8) +
                           align256(side_frag_count((int)K) * 4));
    t += align256(3 * 8);                              // step counts of the state ring
    if (c0.variable_depth) {                           // phi_B, residual, correction, partials
        size_t nvb = 0;
        for (const imexhdg_config &c : cf) {
            int nx, ny;
            device_dims(c, nx, ny);
            nvb += (size_t)member_vol_blocks(nx * ny);
        }
        t += align256(L.N / 3 * 8) + 2 * align256(L.N * 8) + align256(2 * nvb * 8);
    }
    t += 8 * align256((size_t)L.pstride * 8) + align256(5 * (size_t)L.pstride * 8);
    t += align256(nm * sizeof(KrylovState));
    t += align256(nm * sizeof(Member));
    t += align256(3 * (size_t)L.s * nm * sizeof(StageStatus));
    L.total = t;
    return L;
}

int validate(const imexhdg_config *c) {
    if (!c) return fail(IMEXHDG_E_INVAL, "config is NULL");
    if (c->nx < 1 || c->ny < 1) return fail(IMEXHDG_E_INVAL, "nx and ny must be >= 1");
    if ((int64_t)c->nx * c->ny > (int64_t)1 << 28)
        return fail(IMEXHDG_E_INVAL, "too many elements");
    if (c->degree < 1 || c->degree > 8) return fail(IMEXHDG_E_INVAL, "degree must be in [1, 8]");
    if ((int64_t)6 * (c->degree + 1) * c->nx * c->ny >= ((int64_t)1 << 31))
        return fail(IMEXHDG_E_INVAL, "trace system too large (6 (k+1) nx ny >= 2^31)");
    if (!(c->Lx > 0) || !(c->Ly > 0) || !std::isfinite(c->Lx) || !std::isfinite(c->Ly))
        return fail(IMEXHDG_E_INVAL, "domain lengths must be positive and finite");
    if (!(c->g > 0) || !(c->H > 0) || !std::isfinite(c->g * c->H))
        return fail(IMEXHDG_E_INVAL, "g and H must be positive (phi_B = g H > 0)");
    if (!(c->dt > 0) || !std::isfinite(c->dt)) return fail(IMEXHDG_E_INVAL, "dt must be > 0");
    if (c->scheme != IMEXHDG_SCHEME_ARS232 && c->scheme != IMEXHDG_SCHEME_ARS443)
        return fail(IMEXHDG_E_INVAL, "unknown scheme");
    if (c->physics != IMEXHDG_PHYSICS_LINEARIZED && c->physics != IMEXHDG_PHYSICS_NONLINEAR)
        return fail(IMEXHDG_E_INVAL, "unknown physics");
    if (c->precision < IMEXHDG_PREC_FP64 || c->precision > IMEXHDG_PREC_BF16)
        return fail(IMEXHDG_E_INVAL, "unknown precision");
    if (c->local_sweeps < 0 || c->local_sweeps > 3 ||
        (c->local_sweeps == 3 && c->precision != IMEXHDG_PREC_BF16))
        return fail(IMEXHDG_E_INVAL, "local_sweeps must be 0 (default), 1 or 2, or 3 with BF16");
    if (!(c->krylov_rtol > 0) || !(c->krylov_rtol < 1))
        return fail(IMEXHDG_E_INVAL, "krylov_rtol must be in (0, 1)");
    if (!(c->refine_rtol > 0) || !(c->refine_rtol < 1))
        return fail(IMEXHDG_E_INVAL, "refine_rtol must be in (0, 1)");
    if (c->krylov_max_iter < 1 || c->check_every < 1 || c->refine_max < 1)
        return fail(IMEXHDG_E_INVAL, "iteration budgets must be >= 1");
    if (c->launch != IMEXHDG_LAUNCH_GRAPH && c->launch != IMEXHDG_LAUNCH_HOST)
        return fail(IMEXHDG_E_INVAL, "unknown launch mode");
    if (c->trace_guess != IMEXHDG_GUESS_EXTRAPOLATE && c->trace_guess != IMEXHDG_GUESS_LAST)
        return fail(IMEXHDG_E_INVAL, "unknown trace guess");
    if (c->boundary != IMEXHDG_BOUNDARY_PERIODIC && c->boundary != IMEXHDG_BOUNDARY_VORTEX &&
        c->boundary != IMEXHDG_BOUNDARY_WALL)
        return fail(IMEXHDG_E_INVAL, "unknown boundary");
    if (c->variable_depth != 0 && c->variable_depth != 1)
        return fail(IMEXHDG_E_INVAL, "variable_depth must be 0 or 1");
    if (c->variable_depth && c->boundary == IMEXHDG_BOUNDARY_VORTEX)
        return fail(IMEXHDG_E_INVAL,
                    "variable depth takes periodic meshes or walls (the vortex is a flat-bottom "
                    "solution)");
    if (c->boundary != IMEXHDG_BOUNDARY_PERIODIC) {
        if (c->boundary == IMEXHDG_BOUNDARY_VORTEX)
            for (double v : c->vortex)
                if (!std::isfinite(v))
                    return fail(IMEXHDG_E_INVAL, "vortex parameters must be finite");
        if ((int64_t)(c->nx + 2) * (c->ny + 2) > (int64_t)1 << 28 ||
            (int64_t)6 * (c->degree + 1) * (c->nx + 2) * (c->ny + 2) >= ((int64_t)1 << 31))
            return fail(IMEXHDG_E_INVAL, "bounded mesh too large");
    }
    return IMEXHDG_OK;
}

// Members of one batch share everything but the mesh and the time step.
int validate_batch(const imexhdg_config *cfgs, int n) {
    if (!cfgs) return fail(IMEXHDG_E_INVAL, "configs are NULL");
    if (n < 1) return fail(IMEXHDG_E_INVAL, "an ensemble needs at least one member");
    for (int m = 0; m < n; ++m) {
        int rc = validate(cfgs + m);
        if (rc) return fail(rc, "member " + std::to_string(m) + ": " + g_last_error);
        const imexhdg_config &a = cfgs[0], &b = cfgs[m];
        if (a.degree != b.degree || a.g != b.g || a.H != b.H || a.scheme != b.scheme ||
            a.physics != b.physics || a.precision != b.precision ||
            a.local_sweeps != b.local_sweeps ||
            a.krylov_rtol != b.krylov_rtol || a.krylov_max_iter != b.krylov_max_iter ||
            a.check_every != b.check_every || a.refine_rtol != b.refine_rtol ||
            a.refine_max != b.refine_max || a.launch != b.launch ||
            a.trace_guess != b.trace_guess || a.boundary != b.boundary ||
            a.variable_depth != b.variable_depth)
            return fail(IMEXHDG_E_INVAL, "member " + std::to_string(m) +
                                             " differs from member 0 in more than nx, ny, "
                                             "Lx, Ly and dt");
    }
    if (n > 1 && cfgs[0].launch != IMEXHDG_LAUNCH_GRAPH)
        return fail(IMEXHDG_E_INVAL, "an ensemble steps on the fixed launch schedule only");
    if (n > 1 && cfgs[0].boundary != IMEXHDG_BOUNDARY_PERIODIC)
        return fail(IMEXHDG_E_INVAL, "ensemble members must be periodic");
    if (n > 1 && cfgs[0].variable_depth)
        return fail(IMEXHDG_E_INVAL, "ensemble members must have a flat bottom");
    return IMEXHDG_OK;
}

// Build the combination plans of Algorithm 1 for the configured tableau.
// After stage i (0-based) the NL kernel (or a plain combination when the
// physics is linearized) writes Res0_{i+1}, or q^{n+1} after the last stage.
// The implicit residual of an implicit stage j is taken from its local
// equation (eq. IMEXRKDiscretizedForm_localSolver):
//   dt M^-1 L_j = (Q_j - Res0_j) / a~_jj.
// NL terms carry no dt: the NL kernel's output is dt M^-1 NL.
// Trace-guess extrapolation per implicit stage i: the guess is the last
// stage solution x_b plus (tau_i - tau_b) / (tau_b - tau_a) (x_b - x_a), a
// straight line in time through the last two solutions (tau = c~ of the
// stage, one step earlier for the previous step's stages).  Used only where
// tau_a < tau_b < tau_i (ARS(2,3,2): 2.414 for its second stage, 0.414 for
// its first; ARS(4,4,3) has non-monotone stage times, where the guess stays
// the last solution, coefficient 0).
std::vector<double> guess_coefficients(const Tableau &t) {
    std::vector<int> imp;
    for (int i = 0; i < t.s; ++i)
        if (t.at(i, i) != 0.0) imp.push_back(i);
    std::vector<double> ct(t.s, 0.0), coef(t.s, 0.0);
    for (int i = 0; i < t.s; ++i)
        for (int j = 0; j < t.s; ++j) ct[i] += t.at(i, j);
    const int n = (int)imp.size();
    // time (in steps, from the current step's start) of the solve m places
    // before implicit stage k in the sequence of solves
    auto tau = [&](int k, int m) {
        const int p = k - m;
        const int q = ((p % n) + n) % n;
        const int step = (p - q) / n;   // 0, -1, -2, ...
        return ct[imp[q]] + step;
    };
    for (int k = 0; k < n; ++k) {
        const double ti = tau(k, 0), tb = tau(k, 1), ta = tau(k, 2);
        if (ta < tb && tb < ti) coef[imp[k]] = (ti - tb) / (tb - ta);
    }
    return coef;
}

int build_plans(imexhdg_ctx *c) {
    const Tableau &t = c->tab;
    const int s = t.s;
    for (int j = 0; j < s; ++j)
        if (t.at(j, j) == 0.0 && j != 0)
            return fail(IMEXHDG_E_INVAL, "explicit-only stage after the first");
    for (int i = 1; i < s; ++i)
        if (t.at(i, 0) != 0.0)
            return fail(IMEXHDG_E_INVAL, "tableau needs L(q^n) (a~_i1 != 0)");
    c->plans.assign(s, Plan());
    for (int i = 0; i < s; ++i) {
        Plan p;
        if (i + 1 < s) {
            const int m = i + 1;   // Res0_m
            add(p, QN, 1.0);
            for (int j = 0; j <= i; ++j) {
                add(p, j == i ? SELF : NLV + j, t.a(m, j));
                if (j > 0) {
                    const double r = t.at(m, j) / t.at(j, j);
                    add(p, QV + j, r);
                    add(p, RV + j, -r);
                }
            }
        } else {
            // q^{n+1}; if the implicit weights equal the last implicit row
            // (stiffly accurate), q^{n+1} = Q_s + dt sum (b_j - a_sj) NL_j.
            bool stiff = s > 1;
            for (int j = 0; j < s; ++j)
                if (std::fabs(t.bt[j] - t.at(s - 1, j)) > 1e-15) stiff = false;
            if (stiff) {
                add(p, QV + (s - 1), 1.0);
                for (int j = 0; j < s; ++j)
                    add(p, j == s - 1 ? SELF : NLV + j, t.b[j] - t.a(s - 1, j));
            } else {
                add(p, QN, 1.0);
                for (int j = 0; j < s; ++j) {
                    add(p, j == s - 1 ? SELF : NLV + j, t.b[j]);
                    if (j > 0) {
                        add(p, QV + j, t.bt[j] / t.at(j, j));
                        add(p, RV + j, -t.bt[j] / t.at(j, j));
                    }
                }
            }
        }
        cleanup(p);
        c->plans[i] = p;
    }
    c->store_nl.assign(s, false);
    for (const Plan &p : c->plans)
        for (const Term &tm : p)
            if (tm.id >= NLV && tm.id < QV) c->store_nl[tm.id - NLV] = true;
    return IMEXHDG_OK;
}

// Block ranges of every member for the current grid caps; uploads the
// member table (not captured: call outside graph capture).
int build_batch(imexhdg_ctx *c) {
    const int K = c->geom.K;
    int bv = 0, bf = 0, be = 0, bd = 0;
    c->mtab.assign(c->nm, Member{});
    for (int m = 0; m < c->nm; ++m) {
        const MemberHost &h = c->mh[m];
        const OpSet &o = c->ops[h.op];
        Member &d = c->mtab[m];
        d.nx = h.nx;
        d.ny = h.ny;
        d.nel = h.nel;
        const int rx = h.bx > 0 ? h.bx : h.nx, ry = h.by > 0 ? h.by : h.ny;
        d.sx = 2.0 * rx / h.Lx;
        d.sy = 2.0 * ry / h.Ly;
        d.area = (h.Lx / rx / 2.0) * (h.Ly / ry / 2.0);
        d.bx = h.bx;
        d.by = h.by;
        d.bwall = c->wall ? 1 : 0;
        d.dG = o.dG;
        d.dGh = o.dGh;
        d.dGhf = o.dGhf;
        d.dt = h.dt;
        d.vo = h.vo;
        d.to = h.to;
        d.bv = bv;
        d.nbv = member_vol_blocks(h.nel);
        d.bf = bf;
        d.nbf = member_face_blocks(h.nx, h.ny, c->fgrid, c->ftpb);
        d.be = be;
        d.nbe = member_elem_blocks(h.nel, K, c->egrid);
        d.bd = bd;
        d.nbd = member_diag_blocks(h.nel);
        d.Ainv = o.Ainv;
        d.W = o.W;
        d.G = o.G;
        d.Gh = o.Gh;
        d.Px = o.Px;
        d.Py = o.Py;
        d.Ghf = o.Ghf;
        d.Alp = o.Alp;
        bv += d.nbv;
        bf += d.nbf;
        be += d.nbe;
        bd += d.nbd;
    }
    if (std::max(std::max(bf, be), bd) > c->pstride)
        return fail(IMEXHDG_E_INVAL, "internal: partial-sum stride too small");
    c->bt.m = c->dmem;
    c->bt.nm = c->nm;
    c->bt.nbv = bv;
    c->bt.nbf = bf;
    c->bt.nbe = be;
    c->bt.nbd = bd;
    c->bt.box = c->box ? 1 : 0;
    HIP_TRY(hipMemcpyAsync(c->dmem, c->mtab.data(), c->nm * sizeof(Member),
                           hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return IMEXHDG_OK;
}

// ---- event profiler: events are read back at the library's own stream
// synchronisations, so timing adds no extra host-device round trips.
constexpr int kEventPool = 1024;

void prof_harvest(imexhdg_ctx *c) {
    for (int i = 0; i < c->ev_used; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev0[i], c->ev1[i]) == hipSuccess) {
            c->prof_ms[c->ev_id[i]] += ms;
            c->prof_n[c->ev_id[i]] += 1;
            c->prof_dur[c->ev_id[i]].push_back(ms);
        }
    }
    c->ev_used = 0;
}

bool prof_on(const imexhdg_ctx *c, int id) {
    return c->prof_target == -1 || c->prof_target == id;
}

// The events go with the launch itself (set_launch_events), so they time
// the kernel's execution, not the event packets around it.
hipError_t prof_begin(imexhdg_ctx *c, int id) {
    if (!prof_on(c, id)) return hipSuccess;
    if (c->ev_used == kEventPool) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return e;
        prof_harvest(c);
    }
    set_launch_events(c->ev0[c->ev_used], c->ev1[c->ev_used]);
    return hipSuccess;
}

hipError_t prof_end(imexhdg_ctx *c, int id) {
    if (!prof_on(c, id)) return hipSuccess;
    set_launch_events(nullptr, nullptr);
    c->ev_id[c->ev_used] = id;
    c->ev_used += 1;
    return hipSuccess;
}

hipError_t stream_sync(imexhdg_ctx *c) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) prof_harvest(c);
    return e;
}

#define LAUNCH(id, expr)                \
    do {                                \
        HIP_TRY(prof_begin(c, id));     \
        HIP_TRY(expr);                  \
        HIP_TRY(prof_end(c, id));       \
    } while (0)

const double *vec_of(imexhdg_ctx *c, int id) {
    if (id == QN) return c->qin;
    if (id >= NLV && id < QV) return c->NLb[id - NLV];
    if (id >= QV && id < RV) return c->Qb[id - QV];
    return c->Rb[id - RV];
}

int sync_read_ks(imexhdg_ctx *c) {
    HIP_TRY(hipMemcpyAsync(c->hks, c->ks, sizeof(KrylovState), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(stream_sync(c));
    return IMEXHDG_OK;
}

// Sum partials [nq][first, first + n) on the host in a fixed order.
int read_partials(imexhdg_ctx *c, int nq, int first, int n, double *out) {
    HIP_TRY(hipMemcpy2DAsync(c->hpart, (size_t)c->pstride * 8, c->dpart + first,
                             (size_t)c->pstride * 8, (size_t)n * 8, nq, hipMemcpyDeviceToHost,
                             c->stream));
    HIP_TRY(stream_sync(c));
    for (int q = 0; q < nq; ++q) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += c->hpart[(size_t)q * c->pstride + i];
        out[q] = s;
    }
    return IMEXHDG_OK;
}

// ------------------------------------------------ host-driven trace solve
// (one member: the host reads the Krylov state of member 0)

// Inner BiCGStab on Ghat d = rin in precision T, d0 = 0.  The operator is
// the same for every stage and step, so the first sweep's iteration count
// is predictable: run one less than last time before the first convergence
// check, then check every two iterations (a converged solve turns the
// remaining launches into no-ops, so few are wasted).  One iteration is K2
// then K1f (the next K1 fused with this iteration's d and r updates).
template <typename T>
int inner_solve(imexhdg_ctx *c, double tol2, int sweep) {
    const imexhdg_config &cf = c->cfg;
    const Geom &g = c->geom;
    const Batch &b = c->bt;
    T *rin = (T *)c->rin, *rh = (T *)c->krh, *t = (T *)c->kt, *d = (T *)c->kd;
    T *p[2] = {(T *)c->kp[0], (T *)c->kp[1]}, *v[2] = {(T *)c->kv[0], (T *)c->kv[1]};
    T *r[2] = {(T *)c->kr[0], (T *)c->kr[1]};
    int rc;
    LAUNCH(IMEXHDG_K_BICG_INIT,
           launch_bicg_init(g, b, (const T *)rin, r[0], rh, p[0], v[0], d, c->ks, tol2, c->kb,
                            c->stream));
    int par = 0;     // p, v of the current iteration live in p[par], v[par]
    int rp = 0;      // r in r[rp]
    LAUNCH(IMEXHDG_K_BICG_K1, launch_bicg_k1(g, b, r[rp], rh, p[par], v[par], p[1 - par],
                                             v[1 - par], c->ks, c->kb, c->stream));
    par = 1 - par;
    int done = 0;
    int chunk = (sweep == 0 && c->iter_pred > 1) ? c->iter_pred - 1 : cf.check_every;
    while (done < cf.krylov_max_iter) {
        const int n = std::min(chunk, cf.krylov_max_iter - done);
        chunk = std::min(2, cf.check_every);
        for (int it = 0; it < n; ++it) {
            LAUNCH(IMEXHDG_K_BICG_K2,
                   launch_bicg_k2(g, b, r[rp], v[par], rh, t, c->ks, c->kb, c->stream));
            // debug knob: force the breakdown branch of this K1f (the flag is
            // set and cleared between launches, so every block sees one value)
            const bool force = c->dbg_brk > 0 && done + it + 1 == c->dbg_brk;
            if (force)
                HIP_TRY(hipMemsetD32Async((hipDeviceptr_t)&c->ks->force_brk, 1, 1, c->stream));
            LAUNCH(IMEXHDG_K_BICG_K1F,
                   launch_bicg_k1f(g, b, r[rp], t, rh, p[par], v[par], p[1 - par], v[1 - par],
                                   r[1 - rp], d, c->ks, c->kb, c->stream));
            if (force)
                HIP_TRY(hipMemsetD32Async((hipDeviceptr_t)&c->ks->force_brk, 0, 1, c->stream));
            par = 1 - par;
            rp = 1 - rp;
        }
        done += n;
        if ((rc = sync_read_ks(c))) return rc;
        if (c->hks->conv) break;
    }
    if (sweep == 0) c->iter_pred = c->hks->iters;
    LAUNCH(IMEXHDG_K_AXPY, launch_axpy(c->x, (const T *)d, 1.0, c->T, c->stream));
    return IMEXHDG_OK;
}

// Trace solve by FP64 iterative refinement around block-Jacobi BiCGStab.
// x holds the initial guess and receives the solution.  Each sweep: FP64
// residual r = g - G x (and its preconditioned form rin), stop if
// ||r|| <= refine_rtol ||g||, else solve Ghat d = rin and set x += d.
int trace_solve(imexhdg_ctx *c, int32_t *iters_out, double *relres_out) {
    const imexhdg_config &cf = c->cfg;
    const Geom &g = c->geom;
    const Batch &b = c->bt;
    int iters = 0;
    double relres = 0.0;
    for (int sweep = 0;; ++sweep) {
        int rc;
        LAUNCH(IMEXHDG_K_TRACE_RESID,
               c->mixed ? launch_trace_residual(g, b, c->x, c->gv, (float *)c->rin, c->dpart,
                                                c->pstride, nullptr, c->stream)
                        : launch_trace_residual(g, b, c->x, c->gv, (double *)c->rin, c->dpart,
                                                c->pstride, nullptr, c->stream));
        double nrm[4];
        if ((rc = read_partials(c, 4, 0, c->mtab[0].nbf, nrm))) return rc;
        const double rr = nrm[0], gg = nrm[1], ghh = nrm[2], rinrin = nrm[3];
        if (!std::isfinite(gg) || !std::isfinite(rr) || !std::isfinite(rinrin)) {
            c->last_relres = NAN;
            return fail(IMEXHDG_E_NONFINITE, "non-finite trace residual");
        }
        relres = gg > 0.0 ? std::sqrt(rr / gg) : std::sqrt(rr);
        if (relres <= cf.refine_rtol || sweep >= cf.refine_max) break;
        c->sweeps += 1;
        // inner tolerance: krylov_rtol relative to the sweep's right-hand
        // side, floored at 0.1 refine_rtol relative to ||ghat||
        // (an FP32 inner solve is held to at least 1e-6, its attainable
        // accuracy; the FP64 sweeps recover the rest)
        const double fl = 0.1 * cf.refine_rtol;
        const double irt = c->mixed ? std::max(cf.krylov_rtol, 1e-6) : cf.krylov_rtol;
        const double tol2 = std::max(irt * irt * rinrin, fl * fl * ghh);
        rc = c->mixed ? inner_solve<float>(c, tol2, sweep) : inner_solve<double>(c, tol2, sweep);
        if (rc) return rc;
        iters += c->hks->iters;
        if (sweep < kMaxSweeps) {
            c->learn_iters[sweep] = std::max(c->learn_iters[sweep], (int)c->hks->iters);
            c->learn_sweeps = std::max(c->learn_sweeps, sweep + 1);
        }
    }
    c->kiters += iters;
    c->solves += 1;
    c->last_relres = relres;
    if (relres > c->max_relres) c->max_relres = relres;
    if (iters_out) *iters_out = iters;
    if (relres_out) *relres_out = relres;
    if (relres > cf.refine_rtol)
        return fail(IMEXHDG_E_NOCONV, "trace solve above refine_rtol after refine_max sweeps");
    return IMEXHDG_OK;
}

// Bounded mesh: boundary states at stage i's time into the ghost elements of
// v (the state ring position of the step being enqueued gives its step
// count); `last`: also advance the step count of the output position.
int fill_ghosts(imexhdg_ctx *c, double *v, int i, bool last) {
    if (!c->box) return IMEXHDG_OK;
    const int a = c->tcur;
    HIP_TRY(launch_bc_fill(c->geom, c->bt, v, c->tstep + a, c->cst[i] * c->mh[0].dt,
                           last ? c->tstep + (a + 1) % 3 : nullptr, c->vx, c->stream));
    return IMEXHDG_OK;
}

// Ring position of a step's input state (bounded meshes step from the ring only).
void begin_step(imexhdg_ctx *c, const double *qin) {
    c->qin = qin;
    c->tcur = 0;
    for (int a = 0; a < 3; ++a)
        if (c->qbuf[a] == qin) c->tcur = a;
}

// One implicit stage: Z = A^-1 R, g = C Z, solve G x = g, Q = Z - W x.
// stage >= 0 (a step's stage i): the trace guess is extrapolated from the
// last two solutions; stage < 0: x is the guess as it is.
int stage_solve_const(imexhdg_ctx *c, const double *R, double *Q, int32_t *iters,
                      double *relres, int stage) {
    if (c->lp) {
        LAUNCH(IMEXHDG_K_LOCAL_APPLY, launch_local_lp(c->geom, c->bt, R, nullptr, c->aii, c->Z,
                                                      c->lp_bf16, c->lp_ndc, c->stream));
    } else {
        LAUNCH(IMEXHDG_K_LOCAL_APPLY, launch_local_apply(c->geom, c->bt, R, c->Z, c->stream));
    }
    // the ghosts of Z: the boundary data of the step's stage (exact-solution
    // boundary), or the reflection of Z (walls: part of the operator, so
    // also for the corrections of a variable-depth stage, stage < 0)
    if (stage >= 0 || c->wall) {
        int rf = fill_ghosts(c, c->Z, stage >= 0 ? stage : 0, false);
        if (rf) return rf;
    }
    LAUNCH(IMEXHDG_K_TRACE_RHS,
           launch_trace_rhs(c->geom, c->bt, c->Z, c->gv, c->stream, nullptr,
                            stage >= 0 ? c->x : nullptr, c->xp,
                            stage >= 0 ? c->xcoef[stage] : 0.0));
    int rc = trace_solve(c, iters, relres);
    if (rc && rc != IMEXHDG_E_NOCONV) return rc;
    if (c->lp) {
        LAUNCH(IMEXHDG_K_RECOVER, launch_local_lp(c->geom, c->bt, R, c->x, c->aii, Q, c->lp_bf16,
                                                  c->lp_ndc, c->stream));
    } else {
        LAUNCH(IMEXHDG_K_RECOVER, launch_recover(c->geom, c->bt, c->Z, c->x, Q, c->stream));
    }
    return rc;
}

// Stage solve with variable depth: the stage system (I - dt a~_ii M^-1 L) Q
// = R with the nodal phi_B (its DG-LF form, equal to the HDG stage: Sec.
// 4.3, footnote to eq. linear_hdgflux3) by defect correction, each
// correction the constant-depth HDG stage solve of the FP64 residual, Q <-
// Q + S^-1 (R - A Q), until ||R - A Q|| <= refine_rtol ||R||.  Converges
// at a rate set by how far phi_B strays from g H.  The constant-depth
// solves need only be accurate to well below that rate: their trace solves
// stop at kDepthInnerRtol relative to their own right-hand side (or
// refine_rtol if looser), the outer loop reaching refine_rtol.  The trace
// of the stage (the next stage's guess) accumulates the corrections'
// traces.
constexpr int kMaxDepthCorrections = 60;
constexpr double kDepthInnerRtol = 1e-6;
int stage_solve(imexhdg_ctx *c, const double *R, double *Q, int32_t *iters, double *relres,
                int stage) {
    if (!c->vdepth) return stage_solve_const(c, R, Q, iters, relres, stage);
    const double outer = c->cfg.refine_rtol;
    struct Restore {
        imexhdg_ctx *c;
        double v;
        ~Restore() { c->cfg.refine_rtol = v; }
    } restore{c, outer};
    c->cfg.refine_rtol = std::max(outer, kDepthInnerRtol);
    int rc = stage_solve_const(c, R, Q, iters, relres, stage);
    if (rc && rc != IMEXHDG_E_NOCONV) return rc;
    int status = IMEXHDG_OK;
    HIP_TRY(hipMemcpyAsync(c->xsave, c->x, c->T * 8, hipMemcpyDeviceToDevice, c->stream));
    for (int it = 0;; ++it) {
        // walls: the residual's boundary flux reads the reflection of Q
        if (int rf = fill_ghosts(c, Q, stage >= 0 ? stage : 0, false)) return rf;
        HIP_TRY(launch_stage_res_var(c->geom, c->bt, Q, c->pB, R, c->aii, c->dres, c->dcpart,
                                     c->nvb, c->stream));
        HIP_TRY(hipMemcpyAsync(c->hcpart, c->dcpart, 2 * (size_t)c->nvb * 8,
                               hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(stream_sync(c));
        double rr = 0.0, RR = 0.0;
        for (int b = 0; b < c->nvb; ++b) {
            rr += c->hcpart[b];
            RR += c->hcpart[c->nvb + b];
        }
        if (!std::isfinite(rr)) return fail(IMEXHDG_E_NONFINITE, "non-finite stage residual");
        const double rel = RR > 0.0 ? std::sqrt(rr / RR) : std::sqrt(rr);
        if (relres) *relres = rel;
        if (rel <= outer) break;
        if (it >= kMaxDepthCorrections) {
            status = IMEXHDG_E_NOCONV;
            break;
        }
        HIP_TRY(hipMemsetAsync(c->x, 0, c->T * 8, c->stream));
        rc = stage_solve_const(c, c->dres, c->ddel, nullptr, nullptr, -1);
        if (rc && rc != IMEXHDG_E_NOCONV) return rc;
        if (rc == IMEXHDG_E_NOCONV) status = rc;
        HIP_TRY(launch_axpy(Q, (const double *)c->ddel, 1.0, c->N, c->stream));
        HIP_TRY(launch_axpy(c->xsave, (const double *)c->x, 1.0, c->T, c->stream));
        c->dcorr += 1;
    }
    HIP_TRY(hipMemcpyAsync(c->x, c->xsave, c->T * 8, hipMemcpyDeviceToDevice, c->stream));
    return status;
}

int run_plan(imexhdg_ctx *c, int i, const double *Qi, double *out) {
    Comb cb{};
    cb.n = 0;
    cb.self = 0.0;
    cb.out = out;
    cb.store = c->store_nl[i] ? c->NLb[i] : nullptr;
    const bool nonlinear = c->cfg.physics == IMEXHDG_PHYSICS_NONLINEAR;
    for (const Term &t : c->plans[i]) {
        if (t.id == SELF) { cb.self = t.coef; continue; }
        if (!nonlinear && t.id >= NLV && t.id < QV) continue;
        if (cb.n >= kMaxComb) return fail(IMEXHDG_E_INVAL, "combination too long");
        cb.in[cb.n] = vec_of(c, t.id);
        cb.coef[cb.n] = t.coef;
        cb.n += 1;
    }
    // bounded mesh: the explicit flux reads the boundary states from the
    // ghosts of Q_i (Qi is the step's input or a stage buffer, both workspace)
    if (int rf = fill_ghosts(c, const_cast<double *>(Qi), i, i + 1 == c->tab.s)) return rf;
    if (nonlinear && c->vdepth) {
        LAUNCH(IMEXHDG_K_NL, launch_nl_var(c->geom, c->bt, Qi, c->pB, cb, true, c->stream));
    } else if (nonlinear) {
        LAUNCH(IMEXHDG_K_NL, launch_nl(c->geom, c->bt, Qi, cb, true, c->stream, c->nl32));
    } else {
        LAUNCH(IMEXHDG_K_COMBINE, launch_combine(cb, c->N, c->stream));
    }
    return IMEXHDG_OK;
}

// ------------------------------------------------ host-driven step
// One step of Algorithm 1 from qin to qout; the trace solves are driven by
// host reads of the residual and the Krylov state (one member).
int step_host(imexhdg_ctx *c, const double *qin, double *qout, int *status) {
    const int s = c->tab.s;
    begin_step(c, qin);
    for (int i = 0; i < s; ++i) {
        const double *Qi = qin;
        if (i > 0) {
            int rc = stage_solve(c, c->Rb[i], c->Qb[i], nullptr, nullptr, i);
            if (rc == IMEXHDG_E_NOCONV) *status = rc;
            else if (rc) return rc;
            Qi = c->Qb[i];
        }
        double *out = (i + 1 < s) ? c->Rb[i + 1] : qout;
        int rc = run_plan(c, i, Qi, out);
        if (rc) return rc;
    }
    return IMEXHDG_OK;
}

// ------------------------------------------------ fixed launch schedule
// The same trace solve as trace_solve(), with every decision taken on the
// device, per member: per sweep the FP64 residual, the refinement check
// fused with the first K1 (it ends the member's stage solve once
// refine_rtol is met and otherwise opens an inner solve), `budget` rounds
// of K2 and K1f, and x += d.  Launches after convergence return at entry.
template <typename T>
int sched_sweep(imexhdg_ctx *c, int budget, double inner_rtol) {
    const Geom &g = c->geom;
    const Batch &b = c->bt;
    T *rin = (T *)c->rin, *rh = (T *)c->krh, *t = (T *)c->kt, *d = (T *)c->kd;
    T *p[2] = {(T *)c->kp[0], (T *)c->kp[1]}, *v[2] = {(T *)c->kv[0], (T *)c->kv[1]};
    T *r[2] = {(T *)c->kr[0], (T *)c->kr[1]};
    KrylovBufs kb = c->kb;
    kb.sched = 1;
    HIP_TRY(launch_trace_residual(g, b, c->x, c->gv, rin, c->dpart, c->pstride,
                                  c->ks, c->stream));
    // the refinement check and the first K1 of the inner solve in one launch
    HIP_TRY(launch_refine_k1(g, b, (const T *)rin, r[0], rh, p[1], v[1], d, c->ks, c->dpart,
                             c->pstride, c->cfg.refine_rtol, inner_rtol, kb, c->stream));
    int par = 1, rp = 0;
    for (int it = 0; it < budget; ++it) {
        HIP_TRY(launch_bicg_k2(g, b, r[rp], v[par], rh, t, c->ks, kb, c->stream));
        HIP_TRY(launch_bicg_k1f(g, b, r[rp], t, rh, p[par], v[par], p[1 - par], v[1 - par],
                                r[1 - rp], d, c->ks, kb, c->stream));
        par = 1 - par;
        rp = 1 - rp;
    }
    HIP_TRY(launch_axpy_guarded(g, b, c->x, (const T *)d, c->ks, c->stream));
    return IMEXHDG_OK;
}

int stage_solve_sched(imexhdg_ctx *c, const double *R, double *Q, StageStatus *st, int stage) {
    const Geom &g = c->geom;
    const Batch &b = c->bt;
    const imexhdg_config &cf = c->cfg;
    if (c->lp) {
        LAUNCH(IMEXHDG_K_LOCAL_APPLY, launch_local_lp(g, b, R, nullptr, c->aii, c->Z,
                                                      c->lp_bf16, c->lp_ndc, c->stream));
    } else {
        LAUNCH(IMEXHDG_K_LOCAL_APPLY, launch_local_apply(g, b, R, c->Z, c->stream));
    }
    if (int rf = fill_ghosts(c, c->Z, stage, false)) return rf;
    // trace_rhs also resets each member's stage-solve state and extrapolates
    // the trace guess
    LAUNCH(IMEXHDG_K_TRACE_RHS, launch_trace_rhs(g, b, c->Z, c->gv, c->stream, c->ks, c->x,
                                                 c->xp, c->xcoef[stage]));
    const double irt = c->mixed ? std::max(cf.krylov_rtol, 1e-6) : cf.krylov_rtol;
    for (int sw = 0; sw < c->sched_sweeps; ++sw) {
        const int bud = c->sched_budget[sw];
        int rc = c->mixed ? sched_sweep<float>(c, bud, irt) : sched_sweep<double>(c, bud, irt);
        if (rc) return rc;
    }
    // the final check needs ||r|| and ||g|| only (no rin)
    HIP_TRY(c->mixed ? launch_trace_residual(g, b, c->x, c->gv, (float *)nullptr, c->dpart,
                                             c->pstride, c->ks, c->stream)
                     : launch_trace_residual(g, b, c->x, c->gv, (double *)nullptr, c->dpart,
                                             c->pstride, c->ks, c->stream));
    // recover also records each member's stage-solve outcome
    if (c->lp) {
        LAUNCH(IMEXHDG_K_RECOVER, launch_local_lp(g, b, R, c->x, c->aii, Q, c->lp_bf16,
                                                  c->lp_ndc, c->stream, c->ks, c->dpart,
                                                  c->pstride, st));
    } else {
        LAUNCH(IMEXHDG_K_RECOVER, launch_recover(g, b, c->Z, c->x, Q, c->stream, c->ks, c->dpart,
                                                 c->pstride, st));
    }
    return IMEXHDG_OK;
}

// One step on the fixed schedule from qin to qout; stage i records the
// outcome of member m in st[i nm + m].  Nothing here reads from the device.
int step_sched(imexhdg_ctx *c, const double *qin, double *qout, StageStatus *st) {
    const int s = c->tab.s;
    begin_step(c, qin);
    for (int i = 0; i < s; ++i) {
        const double *Qi = qin;
        if (i > 0) {
            int rc = stage_solve_sched(c, c->Rb[i], c->Qb[i], st + (size_t)i * c->nm, i);
            if (rc) return rc;
            Qi = c->Qb[i];
        }
        double *out = (i + 1 < s) ? c->Rb[i + 1] : qout;
        int rc = run_plan(c, i, Qi, out);
        if (rc) return rc;
    }
    return IMEXHDG_OK;
}

void drop_graphs(imexhdg_ctx *c) {
    for (hipGraphExec_t &e : c->gexec)
        if (e) {
            (void)hipGraphExecDestroy(e);
            e = nullptr;
        }
    c->gready = false;
}

void reset_learn(imexhdg_ctx *c) {
    c->learn_sweeps = 0;
    for (int &v : c->learn_iters) v = 0;
}

void reset_window(imexhdg_ctx *c) {
    c->win_sweeps = 0;
    c->win_steps = 0;
    for (int &v : c->win_iters) v = 0;
}

int max_sweeps(const imexhdg_ctx *c) { return std::min((int)c->cfg.refine_max, kMaxSweeps); }

// Schedule from observed sweeps / per-sweep iterations plus the margin.
void schedule_from(imexhdg_ctx *c, int sweeps, const int *iters, bool widen_only) {
    const imexhdg_config &cf = c->cfg;
    int ns = std::min(std::max(sweeps, 1), max_sweeps(c));
    int b[kMaxSweeps];
    for (int i = 0; i < kMaxSweeps; ++i)
        b[i] = std::min(iters[i] + c->margin, (int)cf.krylov_max_iter);
    if (widen_only) {
        ns = std::max(ns, c->sched_sweeps);
        for (int i = 0; i < kMaxSweeps; ++i) b[i] = std::max(b[i], c->sched_budget[i]);
    }
    c->sched_sweeps = ns;
    for (int i = 0; i < kMaxSweeps; ++i) c->sched_budget[i] = i < ns ? b[i] : 0;
}

// Capture one step per ring position (input qbuf[a], output qbuf[a + 1]).
// The capture runs on the library's own stream, so that the caller's
// stream may be the null stream.
int capture(imexhdg_ctx *c) {
    drop_graphs(c);
    if (!c->gstream) HIP_TRY(hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
    const int s = c->tab.s;
    hipStream_t user = c->stream;
    const int prof = c->prof_target;
    for (int a = 0; a < 3; ++a) {
        HIP_TRY(hipStreamBeginCapture(c->gstream, hipStreamCaptureModeThreadLocal));
        c->stream = c->gstream;
        c->prof_target = -2;
        const int rc = step_sched(c, c->qbuf[a], c->qbuf[(a + 1) % 3],
                                  c->dstat + (size_t)a * s * c->nm);
        c->stream = user;
        c->prof_target = prof;
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(c->gstream, &graph);
        if (rc || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            drop_graphs(c);
            if (rc) return rc;
            return fail(IMEXHDG_E_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
        }
        const hipError_t ei = hipGraphInstantiate(&c->gexec[a], graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) {
            c->gexec[a] = nullptr;
            drop_graphs(c);
            return fail(IMEXHDG_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(ei));
        }
    }
    c->gready = true;
    c->captures += 1;
    reset_window(c);
    return IMEXHDG_OK;
}

bool implicit_stage(const imexhdg_ctx *c, int i) { return i > 0 && c->tab.at(i, i) != 0.0; }

void advance(imexhdg_ctx *c) {
    c->cur = (c->cur + 1) % 3;
    c->q = c->qbuf[c->cur];
    c->steps += 1;
}

// Stage outcomes of one step (st = [s][nm]): did every member meet
// refine_rtol?  If so and `record`, adds them to the counters and window.
bool check_step(imexhdg_ctx *c, const StageStatus *st, bool record) {
    const imexhdg_config &cf = c->cfg;
    const int s = c->tab.s;
    bool ok = true;
    for (int i = 0; i < s; ++i)
        if (implicit_stage(c, i))
            for (int m = 0; m < c->nm; ++m) {
                const StageStatus &x = st[(size_t)i * c->nm + m];
                ok = ok && std::isfinite(x.relres) && x.relres <= cf.refine_rtol;
            }
    if (!ok || !record) return ok;
    for (int i = 0; i < s; ++i) {
        if (!implicit_stage(c, i)) continue;
        for (int m = 0; m < c->nm; ++m) {
            const StageStatus &x = st[(size_t)i * c->nm + m];
            c->kiters += x.iters_total;
            c->sweeps += x.sweeps;
            c->last_relres = x.relres;
            c->max_relres = std::max(c->max_relres, x.relres);
            c->win_sweeps = std::max(c->win_sweeps, (int)x.sweeps);
            for (int w = 0; w < kMaxSweeps; ++w)
                c->win_iters[w] = std::max(c->win_iters[w], (int)x.sweep_iters[w]);
        }
        c->solves += 1;
    }
    return true;
}

// Observations of a step that may have failed (all members, all stages).
void observe(imexhdg_ctx *c, const StageStatus *st, int *sweeps, int *iters) {
    *sweeps = 0;
    for (int w = 0; w < kMaxSweeps; ++w) iters[w] = 0;
    for (int i = 0; i < c->tab.s; ++i)
        if (implicit_stage(c, i))
            for (int m = 0; m < c->nm; ++m) {
                const StageStatus &x = st[(size_t)i * c->nm + m];
                *sweeps = std::max(*sweeps, (int)x.sweeps);
                for (int w = 0; w < kMaxSweeps; ++w)
                    iters[w] = std::max(iters[w], (int)x.sweep_iters[w]);
            }
}

// Step on the fixed schedule, eagerly, from ring position a; widens the
// schedule and repeats until every member meets refine_rtol or the schedule
// is at refine_max sweeps of krylov_max_iter iterations.  Then sets the
// schedule to what the step used plus the margin.
int step_sched_eager(imexhdg_ctx *c, int a, int *status) {
    const imexhdg_config &cf = c->cfg;
    const int s = c->tab.s;
    StageStatus *dst = c->dstat + (size_t)a * s * c->nm;
    StageStatus *hst = c->hstat + (size_t)a * s * c->nm;
    for (;;) {
        int rc = step_sched(c, c->qbuf[a], c->qbuf[(a + 1) % 3], dst);
        if (rc) return rc;
        HIP_TRY(hipMemcpyAsync(hst, dst, (size_t)s * c->nm * sizeof(StageStatus),
                               hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(stream_sync(c));
        for (int i = 0; i < s; ++i)
            for (int m = 0; m < c->nm; ++m)
                if (implicit_stage(c, i) && !std::isfinite(hst[(size_t)i * c->nm + m].relres))
                    return fail(IMEXHDG_E_NONFINITE, "non-finite trace residual");
        const bool full = c->sched_sweeps >= max_sweeps(c) &&
                          c->sched_budget[c->sched_sweeps - 1] >= cf.krylov_max_iter;
        const bool ok = check_step(c, hst, true);
        if (ok || full) {
            if (!ok) *status = IMEXHDG_E_NOCONV;
            int sw, it[kMaxSweeps];
            observe(c, hst, &sw, it);
            schedule_from(c, sw, it, false);
            return IMEXHDG_OK;
        }
        // widen: one more sweep and half again the budget of every sweep
        c->redos += 1;
        const int ns = std::min(c->sched_sweeps + 1, max_sweeps(c));
        for (int w = 0; w < ns; ++w) {
            const int b0 = w < c->sched_sweeps ? c->sched_budget[w] : c->sched_budget[0];
            c->sched_budget[w] = std::min((int)cf.krylov_max_iter, std::max(b0 + 4, b0 * 3 / 2));
        }
        c->sched_sweeps = ns;
    }
}

// Graph stepping.  One member: after a cold start (fresh trace guess) one
// host-driven step; then, once, a host-driven step that measures the
// schedule, and the capture.  Several members: cold and learning steps run
// eagerly on a probe schedule (widened until every member converges).
// Graph steps are verified one step behind: before step m + 2 is launched
// (it overwrites the input of step m), step m's stage outcomes are read.
// A failed step is redone (host-driven for one member, on a widened eager
// schedule for several) and the schedule widened (the margin grows by 2);
// after 64 verified steps the margin shrinks by 1 (down to 2) and a
// schedule that has become loose by at least two iterations is tightened.
int step_graph(imexhdg_ctx *c, int nsteps, int *status) {
    const imexhdg_config &cf = c->cfg;
    const int s = c->tab.s;
    const size_t slot = (size_t)s * c->nm;
    int done = 0;
    while (done < nsteps && (c->cold || !c->gready)) {
        const int a = c->cur;
        const bool learn = !c->cold;
        int rc;
        if (c->nm == 1) {
            if (learn) reset_learn(c);
            rc = step_host(c, c->qbuf[a], c->qbuf[(a + 1) % 3], status);
            if (rc) return rc;
            if (learn) schedule_from(c, c->learn_sweeps, c->learn_iters, false);
        } else {
            if (c->sched_sweeps == 0) {
                // probe schedule for the first step
                c->sched_sweeps = max_sweeps(c);
                for (int w = 0; w < kMaxSweeps; ++w)
                    c->sched_budget[w] =
                        w < c->sched_sweeps ? std::min((int)cf.krylov_max_iter, 64) : 0;
            }
            rc = step_sched_eager(c, a, status);
            if (rc) return rc;
        }
        advance(c);
        ++done;
        c->cold = false;
        if (learn && (rc = capture(c))) return rc;
    }
    int inflight[2] = {0, 0}, nin = 0, next = c->cur, launched = done;
    bool want = false;
    while (done < nsteps) {
        if (want && nin == 0) {
            schedule_from(c, c->win_sweeps, c->win_iters, false);
            int rc = capture(c);
            if (rc) return rc;
            want = false;
        }
        if (!want && launched < nsteps && nin < 2) {
            const int a = next;
            HIP_TRY(hipGraphLaunch(c->gexec[a], c->stream));
            HIP_TRY(hipMemcpyAsync(c->hstat + a * slot, c->dstat + a * slot,
                                   slot * sizeof(StageStatus), hipMemcpyDeviceToHost,
                                   c->stream));
            HIP_TRY(hipEventRecord(c->gev[a], c->stream));
            inflight[nin++] = a;
            next = (a + 1) % 3;
            ++launched;
            continue;
        }
        const int a = inflight[0];
        inflight[0] = inflight[1];
        --nin;
        HIP_TRY(hipEventSynchronize(c->gev[a]));
        if (check_step(c, c->hstat + a * slot, true)) {
            c->graph_steps += 1;
            c->win_steps += 1;
            advance(c);
            ++done;
            if (c->win_steps >= 64 && !want) {
                // 64 verified steps without a redo: give back one iteration
                // of the slack a redo added (never below the initial 2)
                if (c->margin > 2) c->margin -= 1;
                int loose = 0;
                for (int w = 0; w < c->sched_sweeps; ++w)
                    loose += c->sched_budget[w] -
                             (w < c->win_sweeps ? std::min(c->win_iters[w] + c->margin,
                                                           (int)cf.krylov_max_iter)
                                                : 0);
                if (loose >= 2) want = true;
                else reset_window(c);
            }
            continue;
        }
        // the step missed refine_rtol on the schedule: redo it
        HIP_TRY(stream_sync(c));
        nin = 0;
        want = false;
        c->redos += 1;
        c->margin = std::min(c->margin + 2, 16);
        int rc;
        if (c->nm == 1) {
            reset_learn(c);
            rc = step_host(c, c->qbuf[a], c->qbuf[(a + 1) % 3], status);
            if (rc) return rc;
            schedule_from(c, c->learn_sweeps, c->learn_iters, true);
        } else {
            rc = step_sched_eager(c, a, status);
            if (rc) return rc;
        }
        c->cur = a;
        advance(c);
        ++done;
        launched = done;
        next = c->cur;
        if ((rc = capture(c))) return rc;
    }
    return IMEXHDG_OK;
}

// Convert a member's host state (user ordering [ey][ex][j][i]) to the device
// layout in h (3 K^2 nel values).
// Element e of the host ordering (over the mesh's own elements) in the
// device layout: a bounded mesh's element (ex, ey) sits at ey (bx + 2) + ex.
int device_elem(const MemberHost &m, int e) {
    return m.bx > 0 ? (e / m.bx) * m.nx + e % m.bx : e;
}

int host_elems(const MemberHost &m) { return m.bx > 0 ? m.bx * m.by : m.nel; }

int state_to_device(const imexhdg_ctx *c, const MemberHost &m, int vars, const double *a,
                    const double *b, const double *cc, std::vector<double> &h) {
    const int K = c->geom.K, nel = m.nel;
    const double g = c->cfg.g, H = c->cfg.H, phiB = g * H;
    const size_t NN = (size_t)K * K * nel;
    h.assign(3 * NN, 0.0);
    for (int e = 0; e < host_elems(m); ++e)
        for (int n = 0; n < K * K; ++n) {
            const size_t src = (size_t)e * K * K + n,
                         dst = (size_t)n * nel + device_elem(m, e);
            double p, U, V;
            if (vars == IMEXHDG_VARS_DEPTH) {
                // phi_eta = g h - phi_B at the node (one member), the
                // arithmetic of the device path (set_state_device): both
                // products rounded before the difference
                if (c->vdepth) {
                    const double gh = g * a[src];
                    const double pb = g * c->hB[src];
                    p = gh - pb;
                } else {
                    p = g * (a[src] - H);
                }
                U = g * b[src];
                V = g * cc[src];
            } else {
                p = a[src];
                U = b[src];
                V = cc[src];
            }
            const double phi = p + (c->vdepth ? g * c->hB[src] : phiB);
            if (!std::isfinite(p) || !std::isfinite(U) || !std::isfinite(V))
                return fail(IMEXHDG_E_INVAL, "state holds NaN or Inf");
            if (!(phi > 0)) return fail(IMEXHDG_E_INVAL, "total depth must be positive");
            h[dst] = p;
            h[NN + dst] = U;
            h[2 * NN + dst] = V;
        }
    return IMEXHDG_OK;
}

void state_from_device(const imexhdg_ctx *c, const MemberHost &m, int vars,
                       const std::vector<double> &h, double *a, double *b, double *cc) {
    const int K = c->geom.K, nel = m.nel;
    const double g = c->cfg.g, H = c->cfg.H;
    const size_t NN = (size_t)K * K * nel;
    for (int e = 0; e < host_elems(m); ++e)
        for (int n = 0; n < K * K; ++n) {
            const size_t dst = (size_t)e * K * K + n,
                         src = (size_t)n * nel + device_elem(m, e);
            const double p = h[src], U = h[NN + src], V = h[2 * NN + src];
            if (vars == IMEXHDG_VARS_DEPTH) {
                a[dst] = (c->vdepth ? c->hB[dst] : H) + p / g;
                b[dst] = U / g;
                cc[dst] = V / g;
            } else {
                a[dst] = p;
                b[dst] = U;
                cc[dst] = V;
            }
        }
}

void get_nodes_of(const imexhdg_ctx *c, const MemberHost &m, double *x, double *y) {
    const int K = c->geom.K;
    const double hx = m.hx, hy = m.hy;
    const int nx = m.bx > 0 ? m.bx : m.nx, ny = m.by > 0 ? m.by : m.ny;
    size_t o = 0;
    for (int ey = 0; ey < ny; ++ey)
        for (int ex = 0; ex < nx; ++ex)
            for (int j = 0; j < K; ++j)
                for (int i = 0; i < K; ++i, ++o) {
                    x[o] = (ex + (c->ref.x[i] + 1.0) / 2.0) * hx;
                    y[o] = (ey + (c->ref.x[j] + 1.0) / 2.0) * hy;
                }
}

void destroy_ctx(imexhdg_ctx *c) {
    if (!c) return;
    if (c->ws || c->hks) (void)hipStreamSynchronize(c->stream);
    for (size_t i = 0; i < c->ev0.size(); ++i) {
        (void)hipEventDestroy(c->ev0[i]);
        (void)hipEventDestroy(c->ev1[i]);
    }
    drop_graphs(c);
    for (hipEvent_t e : c->gev)
        if (e) (void)hipEventDestroy(e);
    if (c->gstream) (void)hipStreamDestroy(c->gstream);
    if (c->hstat) (void)hipHostFree(c->hstat);
    if (c->own_ws && c->ws) (void)hipFree(c->ws);
    if (c->hks) (void)hipHostFree(c->hks);
    if (c->hpart) (void)hipHostFree(c->hpart);
    if (c->hcpart) (void)hipHostFree(c->hcpart);
    delete c;
}

// Create the engine for a batch of validated configs.
int create_ctx(const imexhdg_config *cfgs, int n, void *stream, void *workspace,
               size_t ws_bytes, imexhdg_ctx **out) {
    *out = nullptr;
    const std::vector<imexhdg_config> cf(cfgs, cfgs + n);
    const Layout L = layout_of(cf);
    if (workspace && ws_bytes < L.total)
        return fail(IMEXHDG_E_INVAL, "workspace smaller than the workspace_bytes() figure");
    if (workspace && ((uintptr_t)workspace & 255))
        return fail(IMEXHDG_E_INVAL, "workspace must be 256-byte aligned");
    imexhdg_ctx *c = new (std::nothrow) imexhdg_ctx();
    if (!c) return fail(IMEXHDG_E_NOMEM, "host allocation failed");
    c->cfg = cf[0];
    c->nm = n;
    c->stream = (hipStream_t)stream;
    c->pstride = L.pstride;
    c->member_set.assign(n, false);
    auto bail = [&](int code) {
        destroy_ctx(c);
        return code;
    };
    const int K = cf[0].degree + 1;
    std::vector<StageOperators> hops;
    try {
        c->ref = make_lgl(cf[0].degree);
        c->tab = make_tableau(cf[0].scheme);
        double aii = 0.0;
        for (int i = 0; i < c->tab.s; ++i)
            if (c->tab.at(i, i) != 0.0) {
                if (aii != 0.0 && std::fabs(aii - c->tab.at(i, i)) > 1e-15)
                    return bail(fail(IMEXHDG_E_INVAL, "tableau is not SDIRK"));
                aii = c->tab.at(i, i);
            }
        c->aii = aii;
        size_t vo = 0, to = 0;
        for (int m = 0; m < n; ++m) {
            MemberHost h;
            device_dims(cf[m], h.nx, h.ny);
            h.nel = h.nx * h.ny;
            if (cf[m].boundary != IMEXHDG_BOUNDARY_PERIODIC) {
                h.bx = cf[m].nx;
                h.by = cf[m].ny;
            }
            h.hx = cf[m].Lx / cf[m].nx;
            h.hy = cf[m].Ly / cf[m].ny;
            h.Lx = cf[m].Lx;
            h.Ly = cf[m].Ly;
            h.dt = cf[m].dt;
            h.N = (size_t)3 * K * K * h.nel;
            h.T = (size_t)6 * K * h.nel;
            h.vo = vo;
            h.to = to;
            vo += h.N;
            to += h.T;
            const double hx = h.hx, hy = h.hy;
            int found = -1;
            for (size_t o = 0; o < c->ops.size(); ++o)
                if (c->ops[o].hx == hx && c->ops[o].hy == hy && c->ops[o].dt == h.dt)
                    found = (int)o;
            if (found < 0) {
                OpSet os;
                os.hx = hx;
                os.hy = hy;
                os.dt = h.dt;
                c->ops.push_back(os);
                hops.push_back(make_stage_operators(c->ref, hx, hy, cf[0].g * cf[0].H,
                                                    h.dt * c->aii));
                found = (int)c->ops.size() - 1;
            }
            h.op = found;
            c->mh.push_back(h);
        }
    } catch (const std::exception &e) {
        return bail(fail(IMEXHDG_E_INVAL, std::string("precompute: ") + e.what()));
    }
    int rc;
    if ((rc = build_plans(c))) return bail(rc);
    c->xcoef = guess_coefficients(c->tab);
    if (cf[0].trace_guess == IMEXHDG_GUESS_LAST) std::fill(c->xcoef.begin(), c->xcoef.end(), 0.0);
    // stage abscissae c_i (row sums of the explicit tableau); boundary
    // data at the stage times need c = c~ (true of the ARS schemes)
    c->cst.assign(c->tab.s, 0.0);
    for (int i = 0; i < c->tab.s; ++i) {
        double ce = 0.0, ci = 0.0;
        for (int j = 0; j < c->tab.s; ++j) {
            ce += c->tab.a(i, j);
            ci += c->tab.at(i, j);
        }
        c->cst[i] = ce;
        if (cf[0].boundary != IMEXHDG_BOUNDARY_PERIODIC && std::fabs(ce - ci) > 1e-14)
            return bail(fail(IMEXHDG_E_INVAL, "boundary data need equal stage abscissae"));
    }
    c->box = cf[0].boundary != IMEXHDG_BOUNDARY_PERIODIC;
    c->wall = cf[0].boundary == IMEXHDG_BOUNDARY_WALL;
    c->vx = Vortex{cf[0].H, cf[0].g, cf[0].vortex[0], cf[0].vortex[1], cf[0].vortex[2],
                   cf[0].vortex[3], cf[0].vortex[4]};
    Geom &g = c->geom;
    g.K = K;
    g.phiB = cf[0].g * cf[0].H;
    g.tau = std::sqrt(g.phiB);
    g.winv0 = 1.0 / c->ref.w[0];
    g.winvk = 1.0 / c->ref.w[K - 1];
    for (int i = 0; i < K; ++i) g.w[i] = c->ref.w[i];
    for (int i = 0; i < K; ++i) g.xi[i] = c->ref.x[i];
    for (int i = 0; i < K * K; ++i) g.D[i] = c->ref.D[i];
    for (int m = 0; m < K; ++m)
        for (int a = 0; a < K; ++a)
            g.Dw[m * K + a] = c->ref.w[m] * c->ref.D[m * K + a] / c->ref.w[a];
    c->N = L.N;
    c->T = L.T;
    c->nnodes = 0;
    for (const imexhdg_config &m : cf) c->nnodes += (size_t)m.nx * m.ny * K * K;

    if (hipGetDevice(&c->device) != hipSuccess)
        return bail(fail(IMEXHDG_E_DEVICE, "no HIP device"));
    // the allocation-free stage solve's scratch on this device (once per
    // device, with the device current)
    if (hipError_t e = scratch_init(c->device); e != hipSuccess)
        return bail(fail(IMEXHDG_E_DEVICE, std::string("scratch address: ") +
                                               hipGetErrorString(e)));
    if (workspace) {
        c->ws = (char *)workspace;
        c->ws_bytes = ws_bytes;
    } else {
        if (hipMalloc((void **)&c->ws, L.total) != hipSuccess) {
            c->ws = nullptr;
            return bail(fail(IMEXHDG_E_NOMEM, "hipMalloc of the workspace failed"));
        }
        c->own_ws = true;
        c->ws_bytes = L.total;
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = c->ws + off;
        off += align256(bytes);
        return p;
    };
    for (double *&qb : c->qbuf) qb = (double *)take(L.N * 8);
    c->q = c->qbuf[0];
    c->Z = (double *)take(L.N * 8);
    c->save = (double *)take(L.N * 8);
    for (int i = 0; i < L.s; ++i) c->NLb.push_back((double *)take(L.N * 8));
    for (int i = 0; i < L.s; ++i) c->Qb.push_back((double *)take(L.N * 8));
    for (int i = 0; i < L.s; ++i) c->Rb.push_back((double *)take(L.N * 8));
    c->mixed = cf[0].precision != IMEXHDG_PREC_FP64;
    c->lp = cf[0].precision == IMEXHDG_PREC_FP32 || cf[0].precision == IMEXHDG_PREC_BF16;
    c->lp_bf16 = cf[0].precision == IMEXHDG_PREC_BF16;
    c->nl32 = c->lp;
    c->lp_ndc = cf[0].local_sweeps > 0 ? cf[0].local_sweeps : (c->lp_bf16 ? 3 : 1);
    double **tv[4] = {&c->x, &c->gv, &c->xsave, &c->xp};
    for (double **p : tv) *p = (double *)take(L.T * 8);
    void **iv[10] = {&c->rin, &c->kr[0], &c->krh, &c->kp[0], &c->kp[1],
                     &c->kv[0], &c->kv[1], &c->kr[1], &c->kt, &c->kd};
    for (void **p : iv) *p = take(L.T * (c->mixed ? 4 : 8));
    const size_t n_loc = 3 * K * K, n_tr = 12 * K;
    for (OpSet &o : c->ops) {
        o.Ainv = (double *)take(local_frag_count((int)n_loc, (int)n_loc) * 8);
        o.W = (double *)take(local_frag_count((int)n_loc, (int)n_tr) * 8);
        o.G = (double *)take(frag_count(K) * 8);
        o.Gh = (double *)take(frag_count(K) * 8);
        o.Ghf = (float *)take(frag_count(K) * 4);
        o.Px = (double *)take(9 * K * K * 8);
        o.Py = (double *)take(9 * K * K * 8);
        if (c->lp) o.Alp = take(lp_frag_bytes((int)n_loc, c->lp_bf16));
        o.dG = (double *)take(side_frag_count(K) * 8);
        o.dGh = (double *)take(side_frag_count(K) * 8);
        o.dGhf = (float *)take(side_frag_count(K) * 4);
    }
    c->tstep = (double *)take(3 * 8);
    c->vdepth = cf[0].variable_depth != 0;
    if (c->vdepth) {
        c->nvb = 0;
        for (const MemberHost &h : c->mh) c->nvb += member_vol_blocks(h.nel);
        c->pB = (double *)take(L.N / 3 * 8);
        c->dres = (double *)take(L.N * 8);
        c->ddel = (double *)take(L.N * 8);
        c->dcpart = (double *)take(2 * (size_t)c->nvb * 8);
    }
    c->kb.P1 = (double *)take(3 * (size_t)c->pstride * 8);
    c->kb.P2 = (double *)take(3 * (size_t)c->pstride * 8);
    c->kb.P3 = (double *)take(2 * (size_t)c->pstride * 8);
    c->kb.stride = c->pstride;
    c->dpart = (double *)take(5 * (size_t)c->pstride * 8);
    c->ks = (KrylovState *)take(n * sizeof(KrylovState));
    c->dmem = (Member *)take(n * sizeof(Member));
    c->dstat = (StageStatus *)take(3 * (size_t)L.s * n * sizeof(StageStatus));
    if (off > c->ws_bytes) return bail(fail(IMEXHDG_E_INVAL, "internal: workspace overflow"));
    // a bounded mesh's faces between ghosts must read zero in every trace
    // vector, and nothing ever writes them: clear the whole workspace once
    if (c->box && (hipMemsetAsync(c->ws, 0, off, c->stream) ||
                   hipStreamSynchronize(c->stream)))
        return bail(fail(IMEXHDG_E_DEVICE, "workspace initialisation failed"));

    if (hipHostMalloc((void **)&c->hks, sizeof(KrylovState)) != hipSuccess ||
        hipHostMalloc((void **)&c->hpart, 5 * (size_t)c->pstride * 8) != hipSuccess ||
        hipHostMalloc((void **)&c->hstat, 3 * (size_t)L.s * n * sizeof(StageStatus)) !=
            hipSuccess)
        return bail(fail(IMEXHDG_E_NOMEM, "hipHostMalloc failed"));
    if (c->vdepth && hipHostMalloc((void **)&c->hcpart, 2 * (size_t)c->nvb * 8) != hipSuccess)
        return bail(fail(IMEXHDG_E_NOMEM, "hipHostMalloc failed"));
    for (hipEvent_t &e : c->gev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
            e = nullptr;
            return bail(fail(IMEXHDG_E_DEVICE, "hipEventCreate failed"));
        }

    for (size_t o = 0; o < c->ops.size(); ++o) {
        const StageOperators &op = hops[o];
        const std::vector<double> G = pack_frags(op.Gx, op.Gy, K);
        const std::vector<double> Gh = pack_frags(op.Gxh, op.Gyh, K);
        const std::vector<float> Ghf(Gh.begin(), Gh.end());
        auto up = [&](double *d, const std::vector<double> &h) {
            return hipMemcpyAsync(d, h.data(), h.size() * 8, hipMemcpyHostToDevice, c->stream);
        };
        const OpSet &os = c->ops[o];
        const int nl = 3 * K * K, nt = 12 * K;
        if (up(os.Ainv, pack_local(op.Ainv, nl, nl)) || up(os.W, pack_local(op.W, nl, nt)) ||
            up(os.G, G) || up(os.Gh, Gh) ||
            hipMemcpyAsync(os.Ghf, Ghf.data(), Ghf.size() * 4, hipMemcpyHostToDevice,
                           c->stream) ||
            up(os.Px, op.Pxinv) || up(os.Py, op.Pyinv) || hipStreamSynchronize(c->stream))
            return bail(fail(IMEXHDG_E_DEVICE, "upload of the element operators failed"));
        if (c->box) {
            std::vector<double> dG[4][kSideEntries], dGh[4][kSideEntries];
            boundary_deltas(op, K, c->wall, dG, dGh);
            const std::vector<double> fG = pack_sides(dG, K), fGh = pack_sides(dGh, K);
            const std::vector<float> fGhf(fGh.begin(), fGh.end());
            if (up(os.dG, fG) || up(os.dGh, fGh) ||
                hipMemcpyAsync(os.dGhf, fGhf.data(), fGhf.size() * 4, hipMemcpyHostToDevice,
                               c->stream) ||
                hipStreamSynchronize(c->stream))
                return bail(fail(IMEXHDG_E_DEVICE, "upload of the element operators failed"));
        }
        if (c->lp) {
            const std::vector<uint8_t> f = pack_lp(op.Ainv, nl, c->lp_bf16);
            if (hipMemcpyAsync(os.Alp, f.data(), f.size(), hipMemcpyHostToDevice, c->stream) ||
                hipStreamSynchronize(c->stream))
                return bail(fail(IMEXHDG_E_DEVICE, "upload of the element operators failed"));
        }
    }
    if (const char *db = std::getenv("IMEXHDG_DEBUG_BREAKDOWN_AT")) c->dbg_brk = std::atoi(db);
    if (hipMemsetAsync(c->x, 0, L.T * 8, c->stream) ||
        hipMemsetAsync(c->ks, 0, n * sizeof(KrylovState), c->stream) ||
        hipMemsetAsync(c->xp, 0, L.T * 8, c->stream) ||
        hipMemsetAsync(c->q, 0, L.N * 8, c->stream) ||
        hipMemsetAsync(c->dstat, 0, 3 * (size_t)L.s * n * sizeof(StageStatus), c->stream) ||
        hipStreamSynchronize(c->stream))
        return bail(fail(IMEXHDG_E_DEVICE, "workspace initialisation failed"));
    if ((rc = build_batch(c))) return bail(rc);
    if (c->vdepth) {
        // flat bottom B = H until imexhdg_set_depth
        c->hB.assign(c->nnodes, cf[0].H);
        const std::vector<double> pb(L.N / 3, cf[0].g * cf[0].H);
        if (hipMemcpyAsync(c->pB, pb.data(), pb.size() * 8, hipMemcpyHostToDevice, c->stream) ||
            hipStreamSynchronize(c->stream))
            return bail(fail(IMEXHDG_E_DEVICE, "upload of the depth failed"));
    }
    *out = c;
    g_last_error.clear();
    return IMEXHDG_OK;
}

int step_ctx_run(imexhdg_ctx *c, int nsteps);

// Steps with their host wall time (every path returns with the stream
// synchronised, so the time covers the device work).
int step_ctx(imexhdg_ctx *c, int nsteps) {
    if (nsteps < 0) return fail(IMEXHDG_E_INVAL, "nsteps must be >= 0");
    if (!c->have_state) return fail(IMEXHDG_E_STATE, "step before set_state");
    const auto t0 = std::chrono::steady_clock::now();
    const int rc = step_ctx_run(c, nsteps);
    c->step_ms +=
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

int step_ctx_run(imexhdg_ctx *c, int nsteps) {
    int status = IMEXHDG_OK;
    if (c->cfg.launch == IMEXHDG_LAUNCH_GRAPH && (c->prof_target == -2 || c->nm > 1) &&
        !c->vdepth) {
        int rc = step_graph(c, nsteps, &status);
        if (rc) return rc;
    } else {
        for (int n = 0; n < nsteps; ++n) {
            const int a = c->cur;
            int rc = step_host(c, c->qbuf[a], c->qbuf[(a + 1) % 3], &status);
            if (rc) return rc;
            advance(c);
            c->cold = false;
        }
        HIP_TRY(stream_sync(c));
    }
    if (status) return fail(status, "a trace solve missed refine_rtol");
    return IMEXHDG_OK;
}

int state_was_set(imexhdg_ctx *c, int m);

int set_member_state(imexhdg_ctx *c, int m, int vars, const double *a, const double *b,
                     const double *cc) {
    if (!a || !b || !cc) return fail(IMEXHDG_E_INVAL, "NULL argument");
    if (m < 0 || m >= c->nm) return fail(IMEXHDG_E_INVAL, "member index out of range");
    if (vars != IMEXHDG_VARS_DEPTH && vars != IMEXHDG_VARS_GEOPOTENTIAL)
        return fail(IMEXHDG_E_INVAL, "unknown vars");
    const MemberHost &mh = c->mh[m];
    std::vector<double> h;
    int rc = state_to_device(c, mh, vars, a, b, cc, h);
    if (rc) return rc;
    // the member's slice of each of the three variables
    const size_t NN = mh.N / 3;
    for (int v = 0; v < 3; ++v)
        HIP_TRY(hipMemcpyAsync(c->q + mh.vo + v * NN, h.data() + v * NN, NN * 8,
                               hipMemcpyHostToDevice, c->stream));
    return state_was_set(c, m);
}

// After member m's state has been written (enqueued): reset its trace guess
// and the step bookkeeping.
int state_was_set(imexhdg_ctx *c, int m) {
    const MemberHost &mh = c->mh[m];
    HIP_TRY(hipMemsetAsync(c->x + mh.to, 0, mh.T * 8, c->stream));
    HIP_TRY(hipMemsetAsync(c->xp + mh.to, 0, mh.T * 8, c->stream));
    if (c->box) HIP_TRY(launch_put(c->tstep + c->cur, 0.0, c->stream));
    HIP_TRY(stream_sync(c));
    c->member_set[m] = true;
    c->have_state = std::all_of(c->member_set.begin(), c->member_set.end(),
                                [](bool v) { return v; });
    c->cold = true;
    c->steps = 0;
    c->step_ms = 0.0;
    return IMEXHDG_OK;
}

// Member m's state from a caller's device array (3 n_nodes values,
// variable-major, host state ordering): converted and checked on the device
// into the member's slice of Z (free between steps), then copied into q only
// if every node passed, so a rejected state leaves q unchanged.
int set_member_state_device(imexhdg_ctx *c, int m, int vars, int dtype, const void *src) {
    if (!src) return fail(IMEXHDG_E_INVAL, "NULL argument");
    if (m < 0 || m >= c->nm) return fail(IMEXHDG_E_INVAL, "member index out of range");
    if (vars != IMEXHDG_VARS_DEPTH && vars != IMEXHDG_VARS_GEOPOTENTIAL)
        return fail(IMEXHDG_E_INVAL, "unknown vars");
    if (dtype != IMEXHDG_DTYPE_F64 && dtype != IMEXHDG_DTYPE_F32)
        return fail(IMEXHDG_E_INVAL, "unknown dtype");
    const MemberHost &mh = c->mh[m];
    const int K = c->geom.K;
    const int blocks = state_in_blocks(host_elems(mh), K, c->pstride);
    HIP_TRY(launch_state_in(src, dtype == IMEXHDG_DTYPE_F32, vars == IMEXHDG_VARS_DEPTH,
                            c->cfg.g, c->cfg.H, host_elems(mh), K, c->Z + mh.vo, c->dpart,
                            blocks, c->stream, mh.bx, mh.nx, c->vdepth ? c->pB : nullptr));
    double bad = 0.0;
    int rc = read_partials(c, 1, 0, blocks, &bad);
    if (rc) return rc;
    if (bad != 0.0)
        return fail(IMEXHDG_E_INVAL, "state rejected at " + std::to_string((int64_t)bad) +
                                         " nodes: NaN or Inf or h <= 0");
    HIP_TRY(hipMemcpyAsync(c->q + mh.vo, c->Z + mh.vo, mh.N * 8, hipMemcpyDeviceToDevice,
                           c->stream));
    return state_was_set(c, m);
}

int get_member_state(imexhdg_ctx *c, int m, int vars, double *a, double *b, double *cc) {
    if (!a || !b || !cc) return fail(IMEXHDG_E_INVAL, "NULL argument");
    if (m < 0 || m >= c->nm) return fail(IMEXHDG_E_INVAL, "member index out of range");
    if (vars != IMEXHDG_VARS_DEPTH && vars != IMEXHDG_VARS_GEOPOTENTIAL)
        return fail(IMEXHDG_E_INVAL, "unknown vars");
    if (!c->have_state) return fail(IMEXHDG_E_STATE, "no state set");
    const MemberHost &mh = c->mh[m];
    std::vector<double> h(mh.N);
    const size_t NN = mh.N / 3;
    for (int v = 0; v < 3; ++v)
        HIP_TRY(hipMemcpyAsync(h.data() + v * NN, c->q + mh.vo + v * NN, NN * 8,
                               hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(stream_sync(c));
    state_from_device(c, mh, vars, h, a, b, cc);
    return IMEXHDG_OK;
}

// Phase of the step a kernel class belongs to (IMEXHDG_PHASE_*).
int phase_of(int k) {
    switch (k) {
        case IMEXHDG_K_NL:
        case IMEXHDG_K_COMBINE: return IMEXHDG_PHASE_EXPLICIT;
        case IMEXHDG_K_LOCAL_APPLY:
        case IMEXHDG_K_TRACE_RHS: return IMEXHDG_PHASE_CONDENSE;
        case IMEXHDG_K_TRACE_RESID:
        case IMEXHDG_K_BICG_INIT:
        case IMEXHDG_K_BICG_K1:
        case IMEXHDG_K_BICG_K2:
        case IMEXHDG_K_BICG_K1F:
        case IMEXHDG_K_AXPY: return IMEXHDG_PHASE_TRACE;
        case IMEXHDG_K_RECOVER: return IMEXHDG_PHASE_RECOVER;
        default: return IMEXHDG_PHASE_OTHER;
    }
}

int member_diag(imexhdg_ctx *c, int m, imexhdg_diag *d) {
    if (!d) return fail(IMEXHDG_E_INVAL, "NULL argument");
    if (m < 0 || m >= c->nm) return fail(IMEXHDG_E_INVAL, "member index out of range");
    if (!c->have_state) return fail(IMEXHDG_E_STATE, "no state set");
    LAUNCH(IMEXHDG_K_DIAG, launch_diag(c->geom, c->bt, c->q, c->dpart, c->pstride, c->stream));
    double t[5];
    int rc = read_partials(c, 5, c->mtab[m].bd, c->mtab[m].nbd, t);
    if (rc) return rc;
    std::memset(d, 0, sizeof(*d));
    for (int i = 0; i < 3; ++i) d->mass[i] = t[i];
    d->energy = t[3];
    d->nonfinite = (t[4] != 0.0 || !std::isfinite(t[3])) ? 1 : 0;
    d->steps = c->steps;
    d->krylov_iters = c->kiters;
    d->stage_solves = c->solves;
    d->refine_sweeps = c->sweeps;
    d->last_relres = c->last_relres;
    d->max_relres = c->max_relres;
    d->graph_steps = c->graph_steps;
    d->redo_steps = c->redos;
    d->step_ms = c->step_ms;
    d->depth_corrections = c->dcorr;
    for (int k = 0; k < IMEXHDG_K_COUNT; ++k) d->phase_ms[phase_of(k)] += c->prof_ms[k];
    return IMEXHDG_OK;
}

// ---- allocation-free stage solve
// The buffers a host-driven stage solve uses beyond its inputs and outputs,
// taken from the device's scratch array instead of the context workspace.
struct SolveBufs {
    double *Z, *gv, *x, *dpart, *P1, *P2, *P3;
    void *rin, *kr[2], *krh, *kp[2], *kv[2], *kt, *kd;
    KrylovState *ks;
};

SolveBufs bufs_of(const imexhdg_ctx *c) {
    SolveBufs b;
    b.Z = c->Z; b.gv = c->gv; b.x = c->x; b.dpart = c->dpart;
    b.P1 = c->kb.P1; b.P2 = c->kb.P2; b.P3 = c->kb.P3;
    b.rin = c->rin; b.krh = c->krh; b.kt = c->kt; b.kd = c->kd;
    for (int i = 0; i < 2; ++i) { b.kr[i] = c->kr[i]; b.kp[i] = c->kp[i]; b.kv[i] = c->kv[i]; }
    b.ks = c->ks;
    return b;
}

void use_bufs(imexhdg_ctx *c, const SolveBufs &b) {
    c->Z = b.Z; c->gv = b.gv; c->x = b.x; c->dpart = b.dpart;
    c->kb.P1 = b.P1; c->kb.P2 = b.P2; c->kb.P3 = b.P3;
    c->rin = b.rin; c->krh = b.krh; c->kt = b.kt; c->kd = b.kd;
    for (int i = 0; i < 2; ++i) { c->kr[i] = b.kr[i]; c->kp[i] = b.kp[i]; c->kv[i] = b.kv[i]; }
    c->ks = b.ks;
}

// Carve the buffers out of `base` (nullptr: only count); returns the bytes.
size_t carve_scratch(const imexhdg_ctx *c, char *base, SolveBufs *b) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += align256(bytes);
        return p;
    };
    const size_t isz = c->mixed ? 4 : 8, ps = (size_t)c->pstride * 8;
    b->Z = (double *)take(c->N * 8);
    b->gv = (double *)take(c->T * 8);
    b->x = (double *)take(c->T * 8);
    void **iv[10] = {&b->rin, &b->kr[0], &b->krh, &b->kp[0], &b->kp[1],
                     &b->kv[0], &b->kv[1], &b->kr[1], &b->kt, &b->kd};
    for (void **p : iv) *p = take(c->T * isz);
    b->P1 = (double *)take(3 * ps);
    b->P2 = (double *)take(3 * ps);
    b->P3 = (double *)take(2 * ps);
    b->dpart = (double *)take(5 * ps);
    b->ks = (KrylovState *)take(c->nm * sizeof(KrylovState));
    return off;
}

std::mutex g_noalloc_mu;   // one allocation-free solve at a time per process
static_assert(sizeof(KrylovState) % 4 == 0, "KrylovState is cleared in 32-bit words");

}  // namespace

extern "C" {

int imexhdg_config_init(imexhdg_config *c) {
    if (!c) return fail(IMEXHDG_E_INVAL, "config is NULL");
    std::memset(c, 0, sizeof(*c));
    c->nx = c->ny = 1;
    c->Lx = c->Ly = 1.0;
    c->degree = 2;
    c->g = c->H = 1.0;
    c->dt = 1e-3;
    c->scheme = IMEXHDG_SCHEME_ARS232;
    c->physics = IMEXHDG_PHYSICS_NONLINEAR;
    c->precision = IMEXHDG_PREC_FP64;
    c->krylov_rtol = 1e-14;
    c->krylov_max_iter = 500;
    c->check_every = 8;
    c->refine_rtol = 1e-13;
    c->refine_max = 4;
    c->launch = IMEXHDG_LAUNCH_GRAPH;
    c->trace_guess = IMEXHDG_GUESS_EXTRAPOLATE;
    c->boundary = IMEXHDG_BOUNDARY_PERIODIC;
    c->vortex[0] = 1.0;   // u_inf, v_inf, beta, xc, yc of Sec. 6.1
    c->vortex[1] = 0.0;
    c->vortex[2] = 5.0;
    return IMEXHDG_OK;
}

int imexhdg_validate(const imexhdg_config *cfg) { return validate(cfg); }

int imexhdg_workspace_bytes(const imexhdg_config *cfg, size_t *bytes) {
    int rc = validate(cfg);
    if (rc) return rc;
    if (!bytes) return fail(IMEXHDG_E_INVAL, "bytes is NULL");
    *bytes = layout_of(std::vector<imexhdg_config>(1, *cfg)).total;
    return IMEXHDG_OK;
}

const char *imexhdg_last_error(void) { return g_last_error.c_str(); }

int imexhdg_create(const imexhdg_config *cfg, void *stream, void *workspace, size_t ws_bytes,
                   imexhdg_ctx **out) {
    int rc = validate(cfg);
    if (rc) return rc;
    if (!out) return fail(IMEXHDG_E_INVAL, "out is NULL");
    return create_ctx(cfg, 1, stream, workspace, ws_bytes, out);
}

void imexhdg_destroy(imexhdg_ctx *c) { destroy_ctx(c); }

int imexhdg_sizes(const imexhdg_ctx *c, int64_t *n_nodes, int64_t *n_trace) {
    if (!c) return fail(IMEXHDG_E_INVAL, "ctx is NULL");
    if (n_nodes) *n_nodes = (int64_t)c->nnodes;
    if (n_trace) *n_trace = (int64_t)c->T;
    return IMEXHDG_OK;
}

int imexhdg_get_nodes(const imexhdg_ctx *c, double *x, double *y) {
    if (!c || !x || !y) return fail(IMEXHDG_E_INVAL, "NULL argument");
    get_nodes_of(c, c->mh[0], x, y);
    return IMEXHDG_OK;
}

int imexhdg_set_state(imexhdg_ctx *c, int vars, const double *a, const double *b,
                      const double *cc) {
    if (!c) return fail(IMEXHDG_E_INVAL, "NULL argument");
    return set_member_state(c, 0, vars, a, b, cc);
}

int imexhdg_set_depth(imexhdg_ctx *c, const double *B) {
    if (!c || !B) return fail(IMEXHDG_E_INVAL, "NULL argument");
    if (!c->vdepth) return fail(IMEXHDG_E_INVAL, "the context has a flat bottom (variable_depth = 0)");
    const MemberHost &m = c->mh[0];
    const int K = c->geom.K;
    for (size_t i = 0; i < (size_t)host_elems(m) * K * K; ++i)
        if (!std::isfinite(B[i]) || !(B[i] > 0.0))
            return fail(IMEXHDG_E_INVAL, "depth must be finite and positive");
    // device element (ex, ey) takes the depth of host element (sx, sy); a
    // walled mesh's ghosts take their real neighbour's depth mirrored across
    // the wall (the face nodes then see one depth on both sides)
    const int hnx = m.bx > 0 ? m.bx : m.nx;
    std::vector<double> h((size_t)K * K * m.nel);
    for (int ey = 0; ey < m.ny; ++ey)
        for (int ex = 0; ex < m.nx; ++ex) {
            int sx = ex, sy = ey;
            bool fx = false, fy = false;
            if (m.bx > 0) {
                if (ex >= m.bx) { sx = ex == m.bx ? m.bx - 1 : 0; fx = true; }
                if (ey >= m.by) { sy = ey == m.by ? m.by - 1 : 0; fy = true; }
            }
            const size_t src = ((size_t)sy * hnx + sx) * K * K;
            const size_t de = (size_t)ey * m.nx + ex;
            for (int j = 0; j < K; ++j)
                for (int i = 0; i < K; ++i) {
                    const int si = fx ? K - 1 - i : i, sj = fy ? K - 1 - j : j;
                    h[(size_t)(j * K + i) * m.nel + de] = c->cfg.g * B[src + sj * K + si];
                }
        }
    HIP_TRY(hipMemcpyAsync(c->pB, h.data(), h.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(stream_sync(c));
    c->hB.assign(B, B + c->nnodes);
    return IMEXHDG_OK;
}

int imexhdg_set_state_device(imexhdg_ctx *c, int vars, int dtype, const void *d_state) {
    if (!c) return fail(IMEXHDG_E_INVAL, "NULL argument");
    return set_member_state_device(c, 0, vars, dtype, d_state);
}

int imexhdg_get_state(imexhdg_ctx *c, int vars, double *a, double *b, double *cc) {
    if (!c) return fail(IMEXHDG_E_INVAL, "NULL argument");
    return get_member_state(c, 0, vars, a, b, cc);
}

int imexhdg_step(imexhdg_ctx *c, int32_t nsteps) {
    if (!c) return fail(IMEXHDG_E_INVAL, "ctx is NULL");
    return step_ctx(c, nsteps);
}

int imexhdg_get_diag(imexhdg_ctx *c, imexhdg_diag *d) {
    if (!c || !d) return fail(IMEXHDG_E_INVAL, "NULL argument");
    return member_diag(c, 0, d);
}

int imexhdg_state_device(imexhdg_ctx *c, double **d_q) {
    if (!c || !d_q) return fail(IMEXHDG_E_INVAL, "NULL argument");
    *d_q = c->q;
    return IMEXHDG_OK;
}

int imexhdg_nl_residual(imexhdg_ctx *c, const double *d_q, double *d_out) {
    if (!c || !d_q || !d_out) return fail(IMEXHDG_E_INVAL, "NULL argument");
    if (c->box || c->vdepth)
        return fail(IMEXHDG_E_INVAL, "operator-level calls take flat-bottom periodic meshes only");
    Comb cb{};
    cb.n = 0;
    cb.self = 1.0;
    cb.out = d_out;
    cb.store = nullptr;
    LAUNCH(IMEXHDG_K_NL, launch_nl(c->geom, c->bt, d_q, cb, false, c->stream, c->nl32));
    return IMEXHDG_OK;
}

int imexhdg_linear_residual(imexhdg_ctx *c, const double *d_Q, const double *d_qhat,
                            double *d_out) {
    if (!c || !d_Q || !d_qhat || !d_out) return fail(IMEXHDG_E_INVAL, "NULL argument");
    if (c->box || c->vdepth)
        return fail(IMEXHDG_E_INVAL, "operator-level calls take flat-bottom periodic meshes only");
    LAUNCH(IMEXHDG_K_LINRES,
           launch_linear_residual(c->geom, c->bt, d_Q, d_qhat, d_out, c->stream));
    return IMEXHDG_OK;
}

int imexhdg_stage_solve_noalloc(imexhdg_ctx *c, const double *d_res0, double *d_Q,
                                double *d_qhat, int32_t *iters, double *relres) {
    if (!c || !d_res0 || !d_Q || !d_qhat) return fail(IMEXHDG_E_INVAL, "NULL argument");
    if (c->box || c->vdepth)
        return fail(IMEXHDG_E_INVAL, "operator-level calls take flat-bottom periodic meshes only");
    if (c->nm != 1) return fail(IMEXHDG_E_INVAL, "a context of one mesh is required");
    SolveBufs sb;
    const size_t need = carve_scratch(c, nullptr, &sb);
    if (need > kScratchBytes)
        return fail(IMEXHDG_E_INVAL,
                    "mesh too large for the allocation-free stage solve: it needs " +
                        std::to_string(need) + " bytes of scratch, the limit is " +
                        std::to_string(kScratchBytes) + " bytes (64 MiB)");
    char *base = (char *)scratch_base(c->device);
    if (!base) return fail(IMEXHDG_E_STATE, "scratch not initialised on this device");
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    carve_scratch(c, base, &sb);
    const SolveBufs keep = bufs_of(c);
    use_bufs(c, sb);
    // the Krylov state starts cleared (the debug breakdown flag must be 0);
    // the other buffers are written before they are read
    hipError_t e = launch_zero(sb.ks, sizeof(KrylovState) / 4, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->x, d_qhat, c->T * 8, hipMemcpyDeviceToDevice, c->stream);
    int rc = e == hipSuccess ? stage_solve(c, d_res0, d_Q, iters, relres, -1)
                             : fail(IMEXHDG_E_DEVICE, hipGetErrorString(e));
    if (!rc || rc == IMEXHDG_E_NOCONV) {
        e = hipMemcpyAsync(d_qhat, c->x, c->T * 8, hipMemcpyDeviceToDevice, c->stream);
        if (e == hipSuccess) e = stream_sync(c);
        if (e != hipSuccess) rc = fail(IMEXHDG_E_DEVICE, hipGetErrorString(e));
    } else {
        (void)hipStreamSynchronize(c->stream);   // the scratch is free again on return
    }
    use_bufs(c, keep);
    return rc;
}

int imexhdg_stage_solve(imexhdg_ctx *c, const double *d_res0, double *d_Q, double *d_qhat,
                        int32_t *iters, double *relres) {
    if (!c || !d_res0 || !d_Q || !d_qhat) return fail(IMEXHDG_E_INVAL, "NULL argument");
    if (c->box || c->vdepth)
        return fail(IMEXHDG_E_INVAL, "operator-level calls take flat-bottom periodic meshes only");
    HIP_TRY(hipMemcpyAsync(c->x, d_qhat, c->T * 8, hipMemcpyDeviceToDevice, c->stream));
    int rc = stage_solve(c, d_res0, d_Q, iters, relres, -1);
    if (rc && rc != IMEXHDG_E_NOCONV) return rc;
    HIP_TRY(hipMemcpyAsync(d_qhat, c->x, c->T * 8, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(stream_sync(c));
    return rc;
}

static const char *kKernelNames[IMEXHDG_K_COUNT] = {
    "nl_residual", "combine", "local_apply", "trace_rhs", "trace_residual", "bicg_init",
    "bicg_k1", "bicg_k2", "bicg_k1f", "axpy", "recover", "diag", "linear_residual"};

const char *imexhdg_kernel_name(int32_t k) {
    return (k >= 0 && k < IMEXHDG_K_COUNT) ? kKernelNames[k] : nullptr;
}

int imexhdg_profile(imexhdg_ctx *c, int32_t kernel) {
    if (!c) return fail(IMEXHDG_E_INVAL, "ctx is NULL");
    if (kernel < -2 || kernel >= IMEXHDG_K_COUNT) return fail(IMEXHDG_E_INVAL, "bad kernel id");
    HIP_TRY(stream_sync(c));
    if (kernel != -2 && c->ev0.empty()) {
        c->ev0.resize(kEventPool);
        c->ev1.resize(kEventPool);
        c->ev_id.resize(kEventPool);
        for (int i = 0; i < kEventPool; ++i) {
            HIP_TRY(hipEventCreate(&c->ev0[i]));
            HIP_TRY(hipEventCreate(&c->ev1[i]));
        }
    }
    c->prof_target = kernel;
    c->ev_used = 0;
    for (int i = 0; i < IMEXHDG_K_COUNT; ++i) {
        c->prof_ms[i] = 0.0;
        c->prof_n[i] = 0;
        c->prof_dur[i].clear();
    }
    return IMEXHDG_OK;
}

int imexhdg_profile_read(imexhdg_ctx *c, int32_t kernel, int64_t *launches, double *total_ms) {
    if (!c) return fail(IMEXHDG_E_INVAL, "ctx is NULL");
    if (kernel < 0 || kernel >= IMEXHDG_K_COUNT) return fail(IMEXHDG_E_INVAL, "bad kernel id");
    HIP_TRY(stream_sync(c));
    if (launches) *launches = c->prof_n[kernel];
    if (total_ms) *total_ms = c->prof_ms[kernel];
    return IMEXHDG_OK;
}

int imexhdg_profile_read_min(imexhdg_ctx *c, int32_t kernel, double min_ms, int64_t *launches,
                             double *total_ms) {
    if (!c) return fail(IMEXHDG_E_INVAL, "ctx is NULL");
    if (kernel < 0 || kernel >= IMEXHDG_K_COUNT) return fail(IMEXHDG_E_INVAL, "bad kernel id");
    HIP_TRY(stream_sync(c));
    prof_harvest(c);
    int64_t n = 0;
    double ms = 0.0;
    for (float d : c->prof_dur[kernel])
        if (d >= min_ms) {
            n += 1;
            ms += d;
        }
    if (launches) *launches = n;
    if (total_ms) *total_ms = ms;
    return IMEXHDG_OK;
}

int imexhdg_get_schedule(const imexhdg_ctx *c, int32_t *sweeps, int32_t *budget) {
    if (!c || !sweeps || !budget) return fail(IMEXHDG_E_INVAL, "NULL argument");
    *sweeps = c->gready ? c->sched_sweeps : 0;
    for (int i = 0; i < kMaxSweeps; ++i) budget[i] = c->gready ? c->sched_budget[i] : 0;
    return IMEXHDG_OK;
}

int imexhdg_set_schedule(imexhdg_ctx *c, int32_t sweeps, const int32_t *budget) {
    if (!c) return fail(IMEXHDG_E_INVAL, "ctx is NULL");
    if (c->cfg.launch != IMEXHDG_LAUNCH_GRAPH)
        return fail(IMEXHDG_E_STATE, "the context does not step on a fixed schedule");
    if (sweeps < 0 || sweeps > max_sweeps(c))
        return fail(IMEXHDG_E_INVAL, "sweeps must be in [0, min(refine_max, 8)]");
    if (sweeps > 0 && !budget) return fail(IMEXHDG_E_INVAL, "budget is NULL");
    for (int i = 0; i < sweeps; ++i)
        if (budget[i] < 1 || budget[i] > c->cfg.krylov_max_iter)
            return fail(IMEXHDG_E_INVAL, "budgets must be in [1, krylov_max_iter]");
    HIP_TRY(stream_sync(c));
    c->sched_sweeps = sweeps;
    for (int i = 0; i < kMaxSweeps; ++i) c->sched_budget[i] = i < sweeps ? budget[i] : 0;
    return capture(c);
}

int imexhdg_set_launch_geometry(imexhdg_ctx *c, int32_t face_grid, int32_t elem_grid) {
    if (!c) return fail(IMEXHDG_E_INVAL, "ctx is NULL");
    if (face_grid < 8 || face_grid > kMaxLaunchGrid || elem_grid < 8 ||
        elem_grid > kMaxLaunchGrid)
        return fail(IMEXHDG_E_INVAL, "grid caps must be in [8, 4096]");
    HIP_TRY(stream_sync(c));
    c->fgrid = face_grid;
    c->egrid = elem_grid;
    int rc = build_batch(c);
    if (rc) return rc;
    if (c->gready) return capture(c);
    return IMEXHDG_OK;
}

// Two host-driven steps from the saved state with every kernel class
// timed; per-class mean launch time (ms) and launch count.
static int tune_trial(imexhdg_ctx *c, int fg, int eg, double *avg, int64_t *cnt) {
    c->fgrid = fg;
    c->egrid = eg;
    int rc = build_batch(c);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(c->q, c->save, c->N * 8, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipMemsetAsync(c->x, 0, c->T * 8, c->stream));
    HIP_TRY(hipMemsetAsync(c->xp, 0, c->T * 8, c->stream));
    if (c->box) HIP_TRY(launch_put(c->tstep + c->cur, (double)c->steps, c->stream));
    rc = imexhdg_profile(c, -1);
    if (rc) return rc;
    int status = IMEXHDG_OK;
    for (int i = 0; i < 2; ++i) {
        const int a = c->cur;
        rc = step_host(c, c->qbuf[a], c->qbuf[(a + 1) % 3], &status);
        if (rc) return rc;
        c->cur = (a + 1) % 3;
        c->q = c->qbuf[c->cur];
    }
    HIP_TRY(stream_sync(c));
    for (int k = 0; k < IMEXHDG_K_COUNT; ++k) {
        cnt[k] = c->prof_n[k];
        avg[k] = c->prof_n[k] ? c->prof_ms[k] / (double)c->prof_n[k] : 0.0;
    }
    return IMEXHDG_OK;
}

int imexhdg_autotune(imexhdg_ctx *c, const char *cache_path, int32_t *face_grid,
                     int32_t *elem_grid) {
    if (!c) return fail(IMEXHDG_E_INVAL, "ctx is NULL");
    if (!c->have_state) return fail(IMEXHDG_E_STATE, "autotune needs a state");
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, c->device));
    std::ostringstream ks;
    ks << prop.gcnArchName << "/" << prop.multiProcessorCount << "cu k=" << c->cfg.degree
       << " mesh=" << c->cfg.nx << "x" << c->cfg.ny << " prec=" << c->cfg.precision;
    const std::string key = ks.str();
    int best_f = -1, best_e = -1;
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (in && std::getline(in, line)) {
            const size_t t1 = line.find('\t');
            if (t1 == std::string::npos || line.compare(0, t1, key) != 0 || t1 != key.size())
                continue;
            std::istringstream rest(line.substr(t1 + 1));
            int f = 0, e = 0;
            if (!(rest >> f >> e) || f < 8 || f > kMaxLaunchGrid || e < 8 || e > kMaxLaunchGrid)
                return fail(IMEXHDG_E_INVAL, "malformed autotune cache line: " + line);
            best_f = f;
            best_e = e;
        }
    }
    if (best_f < 0) {
        // time the candidates from a copy of the current state
        HIP_TRY(stream_sync(c));
        HIP_TRY(hipMemcpyAsync(c->save, c->q, c->N * 8, hipMemcpyDeviceToDevice, c->stream));
        const int64_t keep[4] = {c->steps, c->kiters, c->solves, c->sweeps};
        const double keep_r[2] = {c->last_relres, c->max_relres};
        double avg[IMEXHDG_K_COUNT], base_avg[IMEXHDG_K_COUNT];
        int64_t cnt[IMEXHDG_K_COUNT], w[IMEXHDG_K_COUNT];
        const int face_k[4] = {IMEXHDG_K_TRACE_RESID, IMEXHDG_K_BICG_K1, IMEXHDG_K_BICG_K2,
                               IMEXHDG_K_BICG_K1F};
        const int elem_k[1] = {IMEXHDG_K_BICG_INIT};
        const int cand[5] = {256, 512, 1024, 2048, 4096};
        const int f0 = c->fgrid, e0 = c->egrid;
        const MemberHost &mh = c->mh[0];
        const int K = c->geom.K;
        // a discarded warm-up trial, then the incumbent; a candidate must beat
        // the incumbent by 2% to replace it (two steps per trial are noisy)
        int rc = tune_trial(c, f0, e0, base_avg, w);
        if (!rc) rc = tune_trial(c, f0, e0, base_avg, w);
        auto score = [&](const double *a, const int *ks_, int nk) {
            double s = 0.0;
            for (int i = 0; i < nk; ++i) s += a[ks_[i]] * (double)w[ks_[i]];
            return s;
        };
        best_f = f0;
        best_e = e0;
        double best = rc ? 0.0 : score(base_avg, face_k, 4);
        for (int i = 0; i < 5 && !rc; ++i) {
            if (member_face_blocks(mh.nx, mh.ny, cand[i]) ==
                member_face_blocks(mh.nx, mh.ny, best_f))
                continue;
            if ((rc = tune_trial(c, cand[i], e0, avg, cnt))) break;
            const double sc = score(avg, face_k, 4);
            if (sc < 0.98 * best) {
                best = sc;
                best_f = cand[i];
            }
        }
        if (!rc) best = score(base_avg, elem_k, 1);
        for (int i = 0; i < 5 && !rc; ++i) {
            if (member_elem_blocks(mh.nel, K, cand[i]) == member_elem_blocks(mh.nel, K, best_e))
                continue;
            if ((rc = tune_trial(c, best_f, cand[i], avg, cnt))) break;
            const double sc = score(avg, elem_k, 1);
            if (sc < 0.98 * best) {
                best = sc;
                best_e = cand[i];
            }
        }
        // restore the state, the counters and the profiler
        c->prof_target = -2;
        c->ev_used = 0;
        for (int k = 0; k < IMEXHDG_K_COUNT; ++k) {
            c->prof_ms[k] = 0.0;
            c->prof_n[k] = 0;
        }
        HIP_TRY(hipMemcpyAsync(c->q, c->save, c->N * 8, hipMemcpyDeviceToDevice, c->stream));
        HIP_TRY(hipMemsetAsync(c->x, 0, c->T * 8, c->stream));
        HIP_TRY(hipMemsetAsync(c->xp, 0, c->T * 8, c->stream));
        if (c->box) HIP_TRY(launch_put(c->tstep + c->cur, (double)keep[0], c->stream));
        HIP_TRY(stream_sync(c));
        c->steps = keep[0];
        c->kiters = keep[1];
        c->solves = keep[2];
        c->sweeps = keep[3];
        c->last_relres = keep_r[0];
        c->max_relres = keep_r[1];
        c->cold = true;
        if (rc) {
            c->fgrid = f0;
            c->egrid = e0;
            (void)build_batch(c);
            return rc;
        }
        if (cache_path) {
            std::ofstream out(cache_path, std::ios::app);
            if (out) out << key << '\t' << best_f << '\t' << best_e << '\n';
        }
    }
    if (face_grid) *face_grid = best_f;
    if (elem_grid) *elem_grid = best_e;
    return imexhdg_set_launch_geometry(c, best_f, best_e);
}

// ------------------------------------------------------------- ensembles
// Ensemble autotuner: the face blocks of each member are either capped
// (fg) or sized to a number of tiles per block (tpb > 0, the same work per
// block whatever the member's size, so that no large member's blocks form
// the tail of a launch); members that have converged still launch their
// blocks (as no-ops), so fewer blocks per member can win.  Times graph
// steps (one warm step, then two) from a saved state for each candidate.
static int ens_trial(imexhdg_ctx *c, int fg, int tpb, double *ms) {
    c->ftpb = tpb;
    int rc = imexhdg_set_launch_geometry(c, fg, c->egrid);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(c->q, c->save, c->N * 8, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->x, c->xsave, c->T * 8, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->xp, c->xsave, c->T * 8, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(stream_sync(c));
    if ((rc = step_ctx(c, 1))) return rc;
    const auto t0 = std::chrono::steady_clock::now();
    if ((rc = step_ctx(c, 2))) return rc;
    HIP_TRY(stream_sync(c));
    *ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return IMEXHDG_OK;
}

int imexhdg_ens_autotune(imexhdg_ens *e, const char *cache_path, int32_t *face_grid,
                         int32_t *tiles_per_block) {
    if (!e) return fail(IMEXHDG_E_INVAL, "ens is NULL");
    imexhdg_ctx *c = e->c;
    if (!c->have_state) return fail(IMEXHDG_E_STATE, "autotune needs a state");
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, c->device));
    int64_t nel = 0;
    for (const MemberHost &h : c->mh) nel += h.nel;
    std::ostringstream ks;
    ks << prop.gcnArchName << "/" << prop.multiProcessorCount << "cu ensemble k="
       << c->cfg.degree << " members=" << c->nm << " elements=" << nel
       << " prec=" << c->cfg.precision;
    const std::string key = ks.str();
    int best_f = -1, best_t = 0;
    if (cache_path) {
        std::ifstream in(cache_path);
        std::string line;
        while (in && std::getline(in, line)) {
            const size_t t1 = line.find('\t');
            if (t1 == std::string::npos || t1 != key.size() || line.compare(0, t1, key) != 0)
                continue;
            std::istringstream rest(line.substr(t1 + 1));
            int f = 0, t = 0;
            if (!(rest >> f) || f < 8 || f > kMaxLaunchGrid)
                return fail(IMEXHDG_E_INVAL, "malformed autotune cache line: " + line);
            if (!(rest >> t)) t = 0;   // tiles per block: optional
            if (t < 0 || t > 64)
                return fail(IMEXHDG_E_INVAL, "malformed autotune cache line: " + line);
            best_f = f;
            best_t = t;
        }
    }
    if (best_f < 0) {
        if (c->cold || !c->gready) {
            int rc = step_ctx(c, 2);   // learn the schedule first
            if (rc) return rc;
        }
        HIP_TRY(stream_sync(c));
        HIP_TRY(hipMemcpyAsync(c->save, c->q, c->N * 8, hipMemcpyDeviceToDevice, c->stream));
        HIP_TRY(hipMemcpyAsync(c->xsave, c->x, c->T * 8, hipMemcpyDeviceToDevice, c->stream));
        const int64_t keep[6] = {c->steps, c->kiters, c->solves, c->sweeps, c->graph_steps,
                                 c->redos};
        const double keep_r[3] = {c->last_relres, c->max_relres, c->step_ms};
        // (cap, tiles per block): caps alone, then uniform tiles per block
        const int cand[12][2] = {{16, 0},   {32, 0},   {48, 0},   {64, 0},
                                 {96, 0},   {128, 0},  {1024, 0}, {kMaxLaunchGrid, 2},
                                 {kMaxLaunchGrid, 3}, {kMaxLaunchGrid, 4},
                                 {kMaxLaunchGrid, 6}, {kMaxLaunchGrid, 8}};
        const int f0 = c->fgrid, t0 = c->ftpb;
        double best = 0.0, ms = 0.0;
        int rc = ens_trial(c, f0, t0, &ms);          // warm-up
        if (!rc) rc = ens_trial(c, f0, t0, &best);
        best_f = f0;
        best_t = t0;
        for (int i = 0; i < 12 && !rc; ++i) {
            if (cand[i][0] == best_f && cand[i][1] == best_t) continue;
            if ((rc = ens_trial(c, cand[i][0], cand[i][1], &ms))) break;
            if (ms < 0.98 * best) {
                best = ms;
                best_f = cand[i][0];
                best_t = cand[i][1];
            }
        }
        HIP_TRY(hipMemcpyAsync(c->q, c->save, c->N * 8, hipMemcpyDeviceToDevice, c->stream));
        HIP_TRY(hipMemcpyAsync(c->x, c->xsave, c->T * 8, hipMemcpyDeviceToDevice, c->stream));
    HIP_TRY(hipMemcpyAsync(c->xp, c->xsave, c->T * 8, hipMemcpyDeviceToDevice, c->stream));
        HIP_TRY(stream_sync(c));
        c->steps = keep[0];
        c->kiters = keep[1];
        c->solves = keep[2];
        c->sweeps = keep[3];
        c->graph_steps = keep[4];
        c->redos = keep[5];
        c->last_relres = keep_r[0];
        c->max_relres = keep_r[1];
        c->step_ms = keep_r[2];
        if (rc) {
            c->ftpb = t0;
            (void)imexhdg_set_launch_geometry(c, f0, c->egrid);
            return rc;
        }
        if (cache_path) {
            std::ofstream out(cache_path, std::ios::app);
            if (out) out << key << '\t' << best_f << '\t' << best_t << '\n';
        }
    }
    if (face_grid) *face_grid = best_f;
    if (tiles_per_block) *tiles_per_block = best_t;
    c->ftpb = best_t;
    return imexhdg_set_launch_geometry(c, best_f, c->egrid);
}

int imexhdg_ens_workspace_bytes(const imexhdg_config *cfgs, int32_t n, size_t *bytes) {
    int rc = validate_batch(cfgs, n);
    if (rc) return rc;
    if (!bytes) return fail(IMEXHDG_E_INVAL, "bytes is NULL");
    *bytes = layout_of(std::vector<imexhdg_config>(cfgs, cfgs + n)).total;
    return IMEXHDG_OK;
}

int imexhdg_ens_create(const imexhdg_config *cfgs, int32_t n, void *stream, void *workspace,
                       size_t ws_bytes, imexhdg_ens **out) {
    int rc = validate_batch(cfgs, n);
    if (rc) return rc;
    if (!out) return fail(IMEXHDG_E_INVAL, "out is NULL");
    *out = nullptr;
    imexhdg_ens *e = new (std::nothrow) imexhdg_ens();
    if (!e) return fail(IMEXHDG_E_NOMEM, "host allocation failed");
    rc = create_ctx(cfgs, n, stream, workspace, ws_bytes, &e->c);
    if (rc) {
        delete e;
        return rc;
    }
    *out = e;
    return IMEXHDG_OK;
}

void imexhdg_ens_destroy(imexhdg_ens *e) {
    if (!e) return;
    destroy_ctx(e->c);
    delete e;
}

int imexhdg_ens_members(const imexhdg_ens *e, int32_t *n) {
    if (!e || !n) return fail(IMEXHDG_E_INVAL, "NULL argument");
    *n = e->c->nm;
    return IMEXHDG_OK;
}

int imexhdg_ens_sizes(const imexhdg_ens *e, int32_t m, int64_t *n_nodes, int64_t *n_trace) {
    if (!e) return fail(IMEXHDG_E_INVAL, "ens is NULL");
    if (m < 0 || m >= e->c->nm) return fail(IMEXHDG_E_INVAL, "member index out of range");
    if (n_nodes) *n_nodes = (int64_t)e->c->mh[m].N / 3;
    if (n_trace) *n_trace = (int64_t)e->c->mh[m].T;
    return IMEXHDG_OK;
}

int imexhdg_ens_get_nodes(const imexhdg_ens *e, int32_t m, double *x, double *y) {
    if (!e || !x || !y) return fail(IMEXHDG_E_INVAL, "NULL argument");
    if (m < 0 || m >= e->c->nm) return fail(IMEXHDG_E_INVAL, "member index out of range");
    get_nodes_of(e->c, e->c->mh[m], x, y);
    return IMEXHDG_OK;
}

int imexhdg_ens_set_state(imexhdg_ens *e, int32_t m, int vars, const double *a,
                          const double *b, const double *c) {
    if (!e) return fail(IMEXHDG_E_INVAL, "ens is NULL");
    return set_member_state(e->c, m, vars, a, b, c);
}

int imexhdg_ens_set_state_device(imexhdg_ens *e, int32_t m, int vars, int dtype,
                                 const void *d_state) {
    if (!e) return fail(IMEXHDG_E_INVAL, "ens is NULL");
    return set_member_state_device(e->c, m, vars, dtype, d_state);
}

int imexhdg_ens_get_state(imexhdg_ens *e, int32_t m, int vars, double *a, double *b,
                          double *c) {
    if (!e) return fail(IMEXHDG_E_INVAL, "ens is NULL");
    return get_member_state(e->c, m, vars, a, b, c);
}

int imexhdg_ens_step(imexhdg_ens *e, int32_t nsteps) {
    if (!e) return fail(IMEXHDG_E_INVAL, "ens is NULL");
    return step_ctx(e->c, nsteps);
}

int imexhdg_ens_get_diag(imexhdg_ens *e, int32_t m, imexhdg_diag *d) {
    if (!e) return fail(IMEXHDG_E_INVAL, "ens is NULL");
    return member_diag(e->c, m, d);
}

int imexhdg_ens_get_schedule(const imexhdg_ens *e, int32_t *sweeps, int32_t *budget) {
    if (!e) return fail(IMEXHDG_E_INVAL, "ens is NULL");
    return imexhdg_get_schedule(e->c, sweeps, budget);
}

int imexhdg_ens_set_launch_geometry(imexhdg_ens *e, int32_t face_grid, int32_t elem_grid) {
    if (!e) return fail(IMEXHDG_E_INVAL, "ens is NULL");
    e->c->ftpb = 0;
    return imexhdg_set_launch_geometry(e->c, face_grid, elem_grid);
}

}  // extern "C"
