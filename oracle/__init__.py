"""Plain FP64 CPU oracle for one IMEX HDG-DG step of the planar shallow-water
equations (Kang, Giraldo & Bui-Thanh, arXiv:1711.02751).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code, tables or constants with the
HIP library; the only thing both sides consume is the seeded input
generator module, which holds none of the method's arithmetic.

Modules
  lgl        Legendre-Gauss-Lobatto reference element (nodes, weights, D).
  swe        Mesh, flux split F = F_L + F_NL (Sec. 3.1), the nonlinear DG
             residual with the Rusanov flux (Sec. 4.3, eq. Full_russanov) and
             the linear operator (Sec. 4.3) assembled as a sparse matrix.
  imex       IMEX Runge-Kutta tableaux (ARS2(2,3,2), ARS3(4,4,3)) and the
             step of Algorithm 1 (Sec. 5), stage solve by an LU factored once.
  hdg_dense  Brute-force dense HDG block system (Sec. 5, eq.
             linearizedHDGsystem) for tiny meshes, used to pin the stage solve.
  box        Bounded rectangle: the exact moving vortex (Sec. 6.1) or
             reflecting walls (Sec. 4.3, eq. reflection) as the boundary
             faces' imaginary neighbour.
  bathy      Variable depth on the periodic grid: nodal phi_B and the source
             term of the linear part (Sec. 3.1, eq. psweGov).
  basin      Reflecting walls over a variable depth (box's walls with
             bathy's depth).

Where the paper is silent the oracle takes these readings (each is listed in
the design notes of the repository):
  * nodal DG with LGL nodes and collocated LGL quadrature (diagonal mass),
    trace nodes = LGL edge nodes;
  * the jump of a normal-carrying quantity is v- n- + v+ n+;
  * tau* uses the total geopotential phi = phi_eta + phi_B and u = U / phi;
  * ARS(2,3,2) explicit coefficient delta = -2 sqrt(2) / 3 (Ascher, Ruuth &
    Spiteri 1997); this constant is "parity unpinned" beyond order checks;
  * the NL dissipation (tau* - tau_L*) is used as printed, without clipping.
"""
