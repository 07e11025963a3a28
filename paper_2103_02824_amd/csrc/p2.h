// The P2 (quadratic Lagrange) fine space: reference tables and the launch
// interface of its element kernels (p2.hip). Not part of the ABI.
//
// Local nodes of a tet: its 4 vertices, then the midpoints of the edges
// (0,1) (0,2) (0,3) (1,2) (1,3) (2,3). Basis in barycentric coordinates:
// lambda_a (2 lambda_a - 1) at vertex a, 4 lambda_a lambda_b at edge (a, b).
//
// Quadrature: Stroud's conical product rule with 3 points per direction
// (degree 5, 27 points, positive weights). The tet is the image of the unit
// cube under xi = u, eta = (1-u) v, zeta = (1-u)(1-v) w; the Jacobian
// (1-u)^2 (1-v) goes into Gauss-Jacobi weights in u and v, w is
// Gauss-Legendre. Points in the order u (slowest), v, w (fastest). The rule
// is exact for the P2 mass matrix (degree 4) and stiffness (degree 2).
#pragma once

#include <cstdint>
#include <vector>

#include <hip/hip_runtime.h>

namespace mlc {

constexpr int P2_NE = 10;   // nodes per tet
constexpr int P2_NQ = 27;   // quadrature points per tet
constexpr int P2_NP = 55;   // symmetric local pairs (a <= b)

// Table layout (doubles), built on the host by p2_tables and copied to the
// device once per context:
//   L  [q][c]        barycentric coordinates of point q          (27 x 4)
//   W  [q]           weight of point q relative to |T| (sum 1)   (27)
//   B  [q][a]        phi_a at point q                            (27 x 10)
//   D  [q][a][c]     d phi_a / d lambda_c at point q             (27 x 10 x 4)
//   SK [p][k]        stiffness pieces: K_ab = |T| sum_k SK[p][k] G_k with
//                    G_k = grad lambda_c . grad lambda_d over the 10 pairs
//                    k = (c <= d) in order (0,0)(0,1)(0,2)(0,3)(1,1)...(3,3)
//                                                                (55 x 10)
//   MM [p]           mass: M_ab = |T| MM[p]                      (55)
// with p the pair (a <= b) in order (0,0)(0,1)..(0,9)(1,1)..(9,9).
constexpr int P2_T_L = 0;
constexpr int P2_T_W = P2_T_L + P2_NQ * 4;
constexpr int P2_T_B = P2_T_W + P2_NQ;
constexpr int P2_T_D = P2_T_B + P2_NQ * P2_NE;
constexpr int P2_T_SK = P2_T_D + P2_NQ * P2_NE * 4;
constexpr int P2_T_MM = P2_T_SK + P2_NP * 10;
constexpr int P2_TAB = P2_T_MM + P2_NP;

// Builds the table above (the Gauss-Jacobi rules from the moments of their
// weights: the monic orthogonal cubic, its roots by bisection, the weights
// by the moment equations).
void p2_tables(std::vector<double>& tab);

// P2 counterparts of the P1 element kernels (same operands; fields at the
// quadrature points are nt x 27, element node lists nt x 10, slot lists
// nt x 100, coarse hats (4 x 27 + 1) x nt).
void launch_qp_density_p2(hipStream_t s, int64_t nt, const int32_t* el, const int32_t* v2d, const double* X, int N,
                          const double* occ, const double* tab, double* rho_out);
void launch_qp_fields_p2(hipStream_t s, int64_t nt, const int32_t* el, const int32_t* v2d, const double* Phi, int N,
                         const double* occ, const double* wnod, const double* vext, const double* geo,
                         const double* qpx, int xck, double xalpha, const double* tab, double* vxc, double* exc,
                         double* veff, double* rho, double* partials);
void launch_field_p2(hipStream_t s, int64_t nt, const int32_t* el, const double* nod, const int32_t* v2d,
                     const double* dofv, const double* add1, const double* add2, const double* tab, double* out);
void launch_assemble2_p2(hipStream_t s, int64_t nt, int64_t n, int64_t nnz, const double* geo,
                         const int32_t* slot_ptr, const int32_t* slot_of, const int32_t* diag_slot, double* esl,
                         double cK1, const double* f1, double cM1, double* val1, double* dinv1, double cK2,
                         const double* f2, double* val2, const double* tab);
void launch_load_p2(hipStream_t s, int64_t n, int64_t nt, const int32_t* adj_ptr, const int32_t* adj_tet,
                    const int8_t* adj_loc, const int32_t* el, const double* geo, const double* f_qp, double scale,
                    const double* gnod, const int32_t* v2d, const double* tab, double* scratch, double* b,
                    double* lvec);
void launch_coarse_hats_p2(hipStream_t s, int64_t cnt, int64_t ng, const int32_t* grp_ptr, const int32_t* grp_tet,
                           const int32_t* el, const double* geo, const double* xyz, const double* cgeo,
                           const double* tab, double* chat);
void launch_coarse_ops_p2(hipStream_t s, int64_t cnt, int64_t ng, const int32_t* grp_ptr, const int32_t* grp_tet,
                          const double* chat, const double* cgeo, const double* fA, const double* fW,
                          const double* tab, double* out);
void launch_coarse_orb_p2(hipStream_t s, int64_t cnt, int64_t ng, const int32_t* grp_ptr, const int32_t* grp_dof,
                          const double* chat, const double* U, int N, const double* tab, double* out);
void launch_coarse_tri_p2(hipStream_t s, int64_t cnt, const int32_t* grp_ptr, const int32_t* grp_tet,
                          const int32_t* el, const double* geo, const double* xyz, const double* cgeo,
                          const double* tab, double* out);
void launch_energy_p2(hipStream_t s, int64_t nt, const int32_t* el, const int32_t* v2d, const double* Phi, int N,
                      const double* occ, const double* wnod, const double* vxc_old, const double* geo, int xck,
                      double xalpha, const double* tab, double* partials);

}  // namespace mlc
