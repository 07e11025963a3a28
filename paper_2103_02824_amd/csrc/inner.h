// Host-side pieces shared by step.cpp and inner.cpp.
#pragma once

#include <utility>
#include <vector>

#include "mlc_internal.h"

namespace mlc {

// Small blocks produced by the fine stage (Algorithm 3 step 1), host copies.
// Orbital-indexed arrays are row-major [k * N + i].
struct FineBlocks {
  std::vector<double> ptF, ptW, ptM, ptK;  // nH x N: P^T O u_i for A_fix, M_{w0}, M, K
  std::vector<double> utF, utW, utM, utK;  // N x N:  U^T O U
  std::vector<double> d, liftH;            // nH: P^T K w0, P^T l
  double zeta = 0.0, liftT = 0.0;          // w0^T K w0, w0^T l
  std::vector<double> cel_ops;             // cnt x 40
  std::vector<double> cel_orb;             // cnt x N x 14
  std::vector<double> cel_pairs;           // joint variant: cnt x npair x 4, (u_j u_l, psi_m)
};

struct InnerOut {
  std::vector<double> lam, phiH, theta2, wH;
  std::vector<double> D;                   // joint variant: N x N coefficients of the u_j (row j, orbital i)
  double theta1 = 0.0, last_diff = 0.0, ms = 0.0;
  int iters = 0;
};

mlc_status inner_loop(mlc_ctx* c, const FineBlocks& fb, InnerOut& out);
mlc_status inner_loop_joint(mlc_ctx* c, const FineBlocks& fb, InnerOut& out);
// orbital pairs (j <= l) in the order of the pair integrals: p(j, l)
inline int pair_index(int N, int j, int l) {
  if (j > l) std::swap(j, l);
  return j * N - (j * (j - 1)) / 2 + (l - j);
}
void add_trilinear_matrix(const mlc_ctx* c, const std::vector<double>& tri, const double* w, double s,
                          std::vector<double>& A);

}  // namespace mlc
