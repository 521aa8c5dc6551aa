// Host-side FP64 precomputation of the reference-element operators.
//
// Everything here runs once per context on the CPU in double precision and
// is uploaded afterwards; nothing is timed inside a step.
#pragma once
#include <vector>

namespace imexhdg {

// Legendre-Gauss-Lobatto line element of degree k (nodal DG on tensor
// quadrilaterals, Sec. 4.1; LGL nodes and collocated quadrature are the
// reading taken for the unspecified basis).
struct LGL {
    int k = 0, K = 0;
    std::vector<double> x, w;   // nodes, weights
    std::vector<double> D;      // D[i*K + j] = l_j'(x_i)
};
LGL make_lgl(int k);

// Operators of one implicit stage on the (shared) reference element of an
// hx-by-hy rectangle, with c = dt * a_ii and tau = sqrt(phi_B).
//
// Local orderings (K = k + 1):
//   volume  v(c, i, j) = c*K*K + j*K + i        (n_loc = 3 K^2)
//   trace   t(f, c, j) = (f*3 + c)*K + j        (n_tr = 12 K)
//           faces f: 0 = west, 1 = east, 2 = south, 3 = north;
//           j runs along the face (y for west/east, x for south/north).
//
// Stage system (Sec. 5, eq. linearizedHDGsystem) per element:
//   A Q + B Qhat = R1,  A = I - c M^-1 dL/dQ,  B = -c M^-1 dL/dQhat
// and, per face node, the conservation condition (eq. HDGcont with LGL edge
// quadrature) sum_sides [F_L(Q).n + tau Q] - 2 tau Qhat = 0.  Eliminating Q
// (eq. recover_volume_unknowns, Q = A^-1 R1 - A^-1 B Qhat) gives the trace
// system (eq. linearizedHDGsystem_schur) in the scaled form
//   G Qhat = g,   G = 2 tau I + sum_K C_K W_K,   g = sum_K C_K Z_K,
// with W = A^-1 B, Z = A^-1 R1 and C_K Q = [F_L(Q).n_K + tau Q] at the
// element's face nodes.
struct StageOperators {
    int K = 0, n_loc = 0, n_tr = 0;
    double c = 0, tau = 0, phiB = 0;
    std::vector<double> Lq, Lh;      // M^-1 L = Lq Q + Lh Qhat (n_loc x n_loc, n_loc x n_tr)
    std::vector<double> Ainv;        // n_loc x n_loc
    std::vector<double> W;           // A^-1 B, n_loc x n_tr
    std::vector<double> S;           // C W, n_tr x n_tr
    // Row blocks of G for one x-face and one y-face: 7 neighbour slots of
    // (3K x 3K), face-local order (c, j).  Slot layouts:
    //   x-face e: 0 self, 1 x(east e), 2 y(e), 3 y(north e), 4 x(west e),
    //             5 y(west e), 6 y(north west e)
    //   y-face e: 0 self, 1 x(e), 2 x(east e), 3 y(north e), 4 y(south e),
    //             5 x(south e), 6 x(east south e)
    std::vector<double> Gx, Gy;      // 7*(3K)^2 each
    std::vector<double> Pxinv, Pyinv;// inverses of the self blocks (block Jacobi)
    std::vector<double> Gxh, Gyh;    // P^-1 G row blocks (left preconditioned)
};
StageOperators make_stage_operators(const LGL &r, double hx, double hy,
                                    double phiB, double c);

// Dense LU with partial pivoting; returns false if singular.  a is n x n
// row-major and is replaced by its inverse.
bool invert(std::vector<double> &a, int n);

}  // namespace imexhdg
