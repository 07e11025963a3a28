// Test driver for the library's host eigen-solver of the augmented problems
// (the bordered tridiagonal [[T, u], [u^T, alpha]] of Algorithm 3 step 2):
// builds T from a dense symmetric C, then reports the k lowest eigenvalues,
// the border weight of each and the inverse-iteration eigenvector, all in the
// basis of C.
#include <cstddef>
#include <vector>

#include "dense.h"

using namespace mlc::dense;

extern "C" void probe_bordered(const double* C0, const double* uc, double alpha, int n, int k, double* ev_out,
                               double* w_out, double* Y, double* s_out) {
  std::vector<double> C(C0, C0 + (std::size_t)n * n);
  Tridiag Tr;
  tridiagonalize(C, n, Tr);
  std::vector<double> u(uc, uc + n), y(n);
  apply_QT(Tr, u.data());
  std::vector<double> ev = lowest_eigenvalues(Tr, u.data(), alpha, k);
  for (int j = 0; j < k; ++j) {
    ev_out[j] = ev[j];
    w_out[j] = border_weight(Tr, u.data(), alpha, ev[j]);
    double s;
    eigenvector(Tr, u.data(), alpha, ev[j], y.data(), &s);
    apply_Q(Tr, y.data());
    for (int r = 0; r < n; ++r) Y[(std::size_t)r * k + j] = y[r];
    s_out[j] = s;
  }
}

// The selection of Algorithm 2 (a) as the library runs it: the k lowest
// eigenvalues of [[T, u], [u^T, alpha]] and, among them, the eigenvector with
// the largest component along v = [vy; vs] (vy in the basis of C). Output:
// the eigenvalues, the index kept, its eigenvector (y in the basis of C, s)
// with x . v > 0, and x . v.
extern "C" int probe_select(const double* C0, const double* uc, double alpha, int n, int k, const double* vyc,
                            double vs, double* ev_out, double* y_out, double* s_out, double* proj_out) {
  std::vector<double> C(C0, C0 + (std::size_t)n * n);
  Tridiag Tr;
  tridiagonalize(C, n, Tr);
  std::vector<double> u(uc, uc + n), vy(vyc, vyc + n), y(n);
  apply_QT(Tr, u.data());
  apply_QT(Tr, vy.data());
  std::vector<double> ev = lowest_eigenvalues(Tr, u.data(), alpha, k);
  for (int j = 0; j < k; ++j) ev_out[j] = ev[j];
  int j = select_projection(Tr, u.data(), alpha, ev, vy.data(), vs, y.data(), s_out, proj_out);
  apply_Q(Tr, y.data());
  for (int r = 0; r < n; ++r) y_out[r] = y[r];
  return j;
}

// C = L^{-1} A L^{-T} with L the Cholesky factor of M (the pencil reduction
// of every inner iteration); returns 0 when M is not positive definite.
extern "C" int probe_congruence(const double* M0, const double* A0, int n, double* C_out) {
  std::vector<double> L(M0, M0 + (std::size_t)n * n), A(A0, A0 + (std::size_t)n * n), C;
  if (!cholesky(L, n)) return 0;
  congruence(L, A, n, C);
  for (std::size_t i = 0; i < (std::size_t)n * n; ++i) C_out[i] = C[i];
  return 1;
}

// lowest_eigenvalues_group on P problems sharing T (from C) against P
// separate lowest_eigenvalues calls: ev_group and ev_single, P x k each.
extern "C" void probe_group(const double* C0, int n, int P, const double* U, const double* alpha, int k,
                            double* ev_group, double* ev_single) {
  std::vector<double> C(C0, C0 + (std::size_t)n * n);
  Tridiag Tr;
  tridiagonalize(C, n, Tr);
  std::vector<std::vector<double>> Ut(P, std::vector<double>(n));
  std::vector<const double*> up(P);
  for (int q = 0; q < P; ++q) {
    for (int i = 0; i < n; ++i) Ut[q][i] = U[(std::size_t)q * n + i];
    apply_QT(Tr, Ut[q].data());
    up[q] = Ut[q].data();
  }
  std::vector<std::vector<double>> evg(P);
  lowest_eigenvalues_group(Tr, P, up.data(), alpha, k, evg.data());
  for (int q = 0; q < P; ++q) {
    std::vector<double> evs = lowest_eigenvalues(Tr, up[q], alpha[q], k);
    for (int j = 0; j < k; ++j) {
      ev_group[(std::size_t)q * k + j] = evg[q][j];
      ev_single[(std::size_t)q * k + j] = evs[j];
    }
  }
}
