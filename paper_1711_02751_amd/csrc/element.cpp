// Host FP64 precomputation: LGL element, local solver and trace-system blocks.
#include "element.hpp"

#include <cmath>
#include <stdexcept>

namespace imexhdg {

namespace {

// P_k and P_k' at x by the three-term recurrence; P_k' from
// (1 - x^2) P_k' = k (P_{k-1} - x P_k) away from the endpoints.
void legendre(int k, double x, double &p, double &dp) {
    double p0 = 1.0, p1 = x;
    if (k == 0) { p = 1.0; dp = 0.0; return; }
    for (int m = 1; m < k; ++m) {
        double p2 = ((2.0 * m + 1.0) * x * p1 - m * p0) / (m + 1.0);
        p0 = p1;
        p1 = p2;
    }
    p = p1;
    dp = k * (p0 - x * p1) / (1.0 - x * x);
}

}  // namespace

LGL make_lgl(int k) {
    if (k < 1) throw std::invalid_argument("degree must be >= 1");
    LGL r;
    r.k = k;
    r.K = k + 1;
    r.x.assign(r.K, 0.0);
    r.w.assign(r.K, 0.0);
    r.x[0] = -1.0;
    r.x[k] = 1.0;
    // interior nodes: roots of P_k', Newton with P_k'' from Legendre's ODE
    // (1 - x^2) P'' = 2 x P' - k (k+1) P.
    for (int i = 1; i < k; ++i) {
        double x = -std::cos(M_PI * i / k);
        for (int it = 0; it < 100; ++it) {
            double p, dp;
            legendre(k, x, p, dp);
            double d2p = (2.0 * x * dp - k * (k + 1.0) * p) / (1.0 - x * x);
            double step = dp / d2p;
            x -= step;
            if (std::fabs(step) < 1e-16) break;
        }
        r.x[i] = x;
    }
    for (int i = 0; i < r.K; ++i) {
        double p, dp;
        if (i == 0 || i == k) p = (i == 0 && (k % 2)) ? -1.0 : 1.0;
        else legendre(k, r.x[i], p, dp);
        r.w[i] = 2.0 / (k * (k + 1.0) * p * p);
    }
    // differentiation matrix from barycentric weights
    std::vector<double> lam(r.K, 1.0);
    for (int j = 0; j < r.K; ++j)
        for (int m = 0; m < r.K; ++m)
            if (m != j) lam[j] /= (r.x[j] - r.x[m]);
    r.D.assign(r.K * r.K, 0.0);
    for (int i = 0; i < r.K; ++i) {
        double diag = 0.0;
        for (int j = 0; j < r.K; ++j) {
            if (i == j) continue;
            double v = (lam[j] / lam[i]) / (r.x[i] - r.x[j]);
            r.D[i * r.K + j] = v;
            diag -= v;
        }
        r.D[i * r.K + i] = diag;
    }
    return r;
}

bool invert(std::vector<double> &a, int n) {
    std::vector<int> piv(n);
    std::vector<double> lu = a;
    for (int col = 0; col < n; ++col) {
        int best = col;
        double bv = std::fabs(lu[col * n + col]);
        for (int r = col + 1; r < n; ++r) {
            double v = std::fabs(lu[r * n + col]);
            if (v > bv) { bv = v; best = r; }
        }
        if (bv == 0.0) return false;
        piv[col] = best;
        if (best != col)
            for (int c = 0; c < n; ++c) std::swap(lu[col * n + c], lu[best * n + c]);
        double inv = 1.0 / lu[col * n + col];
        for (int r = col + 1; r < n; ++r) {
            double f = lu[r * n + col] * inv;
            lu[r * n + col] = f;
            for (int c = col + 1; c < n; ++c) lu[r * n + c] -= f * lu[col * n + c];
        }
    }
    // solve for each column of the identity (with the row swaps applied)
    std::vector<double> out(n * n, 0.0), b(n);
    for (int e = 0; e < n; ++e) {
        for (int i = 0; i < n; ++i) b[i] = (i == e) ? 1.0 : 0.0;
        for (int col = 0; col < n; ++col) std::swap(b[col], b[piv[col]]);
        for (int i = 0; i < n; ++i) {
            double s = b[i];
            for (int j = 0; j < i; ++j) s -= lu[i * n + j] * b[j];
            b[i] = s;
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = b[i];
            for (int j = i + 1; j < n; ++j) s -= lu[i * n + j] * b[j];
            b[i] = s / lu[i * n + i];
        }
        for (int i = 0; i < n; ++i) out[i * n + e] = b[i];
    }
    a.swap(out);
    return true;
}

namespace {

void matmul(const std::vector<double> &A, const std::vector<double> &B,
            std::vector<double> &C, int m, int kk, int n) {
    C.assign((size_t)m * n, 0.0);
    for (int i = 0; i < m; ++i)
        for (int p = 0; p < kk; ++p) {
            double a = A[(size_t)i * kk + p];
            if (a == 0.0) continue;
            for (int j = 0; j < n; ++j) C[(size_t)i * n + j] += a * B[(size_t)p * n + j];
        }
}

}  // namespace

StageOperators make_stage_operators(const LGL &r, double hx, double hy,
                                    double phiB, double c) {
    StageOperators op;
    const int K = r.K, k = r.k;
    op.K = K;
    op.n_loc = 3 * K * K;
    op.n_tr = 12 * K;
    op.c = c;
    op.phiB = phiB;
    op.tau = std::sqrt(phiB);
    const int NL = op.n_loc, NT = op.n_tr;
    auto v = [K](int comp, int i, int j) { return comp * K * K + j * K + i; };
    auto t = [K](int f, int comp, int j) { return (f * 3 + comp) * K + j; };

    op.Lq.assign((size_t)NL * NL, 0.0);
    op.Lh.assign((size_t)NL * NT, 0.0);
    const double sx = 2.0 / hx, sy = 2.0 / hy;
    // volume (F_L(Q), grad v)_K / M: d/dx carried by U and phi_B phi_eta,
    // d/dy by V and phi_B phi_eta (eq. psweLinearFluxTensor); weak form
    // (2/h) sum_m (w_m / w_a) D[m][a] F(m).
    for (int j = 0; j < K; ++j)
        for (int a = 0; a < K; ++a)
            for (int m = 0; m < K; ++m) {
                double cx = sx * r.w[m] / r.w[a] * r.D[m * K + a];
                op.Lq[(size_t)v(0, a, j) * NL + v(1, m, j)] += cx;
                op.Lq[(size_t)v(1, a, j) * NL + v(0, m, j)] += cx * phiB;
                double cy = sy * r.w[m] / r.w[a] * r.D[m * K + a];
                op.Lq[(size_t)v(0, j, a) * NL + v(2, j, m)] += cy;
                op.Lq[(size_t)v(2, j, a) * NL + v(0, j, m)] += cy * phiB;
            }
    // surface: - <Fhat_L . n, v>_dK / M with the hybridized Lax-Friedrichs
    // flux n.Fhat_L = F_L(Q).n + tau (Q - Qhat) (eq. linear_hdgflux3).
    struct Face { int f; double nx, ny; };
    const Face faces[4] = {{0, -1, 0}, {1, 1, 0}, {2, 0, -1}, {3, 0, 1}};
    auto face_node = [k](int f, int j, int &a, int &b) {
        if (f == 0) { a = 0; b = j; }
        else if (f == 1) { a = k; b = j; }
        else if (f == 2) { a = j; b = 0; }
        else { a = j; b = k; }
    };
    for (const Face &F : faces) {
        const double s = (F.f < 2 ? sx : sy) / (F.f % 2 == 0 ? r.w[0] : r.w[k]);
        for (int j = 0; j < K; ++j) {
            int a, b;
            face_node(F.f, j, a, b);
            const int p = v(0, a, b), U = v(1, a, b), V = v(2, a, b);
            op.Lq[(size_t)p * NL + U] -= s * F.nx;
            op.Lq[(size_t)p * NL + V] -= s * F.ny;
            op.Lq[(size_t)U * NL + p] -= s * F.nx * phiB;
            op.Lq[(size_t)V * NL + p] -= s * F.ny * phiB;
            for (int comp = 0; comp < 3; ++comp) {
                const int row = v(comp, a, b);
                op.Lq[(size_t)row * NL + row] -= s * op.tau;
                op.Lh[(size_t)row * NT + t(F.f, comp, j)] += s * op.tau;
            }
        }
    }
    // A = I - c Lq, B = -c Lh; W = A^-1 B.
    op.Ainv.assign((size_t)NL * NL, 0.0);
    for (size_t i = 0; i < (size_t)NL * NL; ++i) op.Ainv[i] = -c * op.Lq[i];
    for (int i = 0; i < NL; ++i) op.Ainv[(size_t)i * NL + i] += 1.0;
    if (!invert(op.Ainv, NL)) throw std::runtime_error("local solver matrix is singular");
    std::vector<double> B((size_t)NL * NT);
    for (size_t i = 0; i < B.size(); ++i) B[i] = -c * op.Lh[i];
    matmul(op.Ainv, B, op.W, NL, NL, NT);
    // C: this element's part of the conservation condition at its face nodes
    std::vector<double> C((size_t)NT * NL, 0.0);
    for (const Face &F : faces)
        for (int j = 0; j < K; ++j) {
            int a, b;
            face_node(F.f, j, a, b);
            const int p = v(0, a, b), U = v(1, a, b), V = v(2, a, b);
            C[(size_t)t(F.f, 0, j) * NL + U] += F.nx;
            C[(size_t)t(F.f, 0, j) * NL + V] += F.ny;
            C[(size_t)t(F.f, 1, j) * NL + p] += F.nx * phiB;
            C[(size_t)t(F.f, 2, j) * NL + p] += F.ny * phiB;
            for (int comp = 0; comp < 3; ++comp)
                C[(size_t)t(F.f, comp, j) * NL + v(comp, a, b)] += op.tau;
        }
    matmul(C, op.W, op.S, NT, NL, NT);

    // Row blocks of G = 2 tau I + sum_K C_K W_K for one x-face and one
    // y-face.  The face is local face `fp` of element K+ and `fm` of K-;
    // slot_of_plus[f] / slot_of_minus[f] give the neighbour slot of each
    // local face of K+ / K-.
    const int B3 = 3 * K;
    auto build = [&](int fp, const int *slot_plus, int fm, const int *slot_minus,
                     std::vector<double> &G) {
        G.assign((size_t)7 * B3 * B3, 0.0);
        for (int i = 0; i < B3; ++i) G[(size_t)i * B3 + i] += 2.0 * op.tau;
        auto add = [&](int fself, const int *slots) {
            for (int rc = 0; rc < B3; ++rc)         // row (c, j) of the face
                for (int f = 0; f < 4; ++f)
                    for (int cc = 0; cc < B3; ++cc) {
                        double val = op.S[(size_t)(fself * B3 + rc) * NT + f * B3 + cc];
                        G[(size_t)slots[f] * B3 * B3 + (size_t)rc * B3 + cc] += val;
                    }
        };
        add(fp, slot_plus);
        add(fm, slot_minus);
    };
    // x-face e: K+ = e (face = its west), K- = west(e) (face = its east)
    const int xs_plus[4] = {0, 1, 2, 3};
    const int xs_minus[4] = {4, 0, 5, 6};
    build(0, xs_plus, 1, xs_minus, op.Gx);
    // y-face e: K+ = e (face = its south), K- = south(e) (face = its north)
    const int ys_plus[4] = {1, 2, 0, 3};
    const int ys_minus[4] = {5, 6, 4, 0};
    build(2, ys_plus, 3, ys_minus, op.Gy);

    auto precondition = [&](const std::vector<double> &G, std::vector<double> &Pinv,
                            std::vector<double> &Gh) {
        Pinv.assign(G.begin(), G.begin() + (size_t)B3 * B3);
        if (!invert(Pinv, B3)) throw std::runtime_error("trace block is singular");
        Gh.assign(G.size(), 0.0);
        for (int s = 0; s < 7; ++s) {
            std::vector<double> blk(G.begin() + (size_t)s * B3 * B3,
                                    G.begin() + (size_t)(s + 1) * B3 * B3), out;
            matmul(Pinv, blk, out, B3, B3, B3);
            std::copy(out.begin(), out.end(), Gh.begin() + (size_t)s * B3 * B3);
        }
    };
    precondition(op.Gx, op.Pxinv, op.Gxh);
    precondition(op.Gy, op.Pyinv, op.Gyh);
    return op;
}

}  // namespace imexhdg
