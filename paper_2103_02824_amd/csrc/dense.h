// Host FP64 dense linear algebra for the small augmented problems
// (Algorithm 3 step 2) and the coarse self-consistent solve (Algorithm 1
// step 1). Row-major square matrices of order n.
#pragma once

#include <cstdint>
#include <vector>

namespace mlc {
namespace dense {

// In-place Cholesky A = L L^T (lower triangle of A overwritten by L; the
// strict upper triangle is zeroed). Returns false if A is not SPD.
bool cholesky(std::vector<double>& A, int64_t n);
// Solve L x = b (forward) and L^T x = b (backward) in place.
void forward(const std::vector<double>& L, int64_t n, double* x);
void backward(const std::vector<double>& L, int64_t n, double* x);
// C = L^{-1} A L^{-T} for symmetric A.
void congruence(const std::vector<double>& L, const std::vector<double>& A, int64_t n, std::vector<double>& C);

// Householder tridiagonalisation of symmetric C = Q T Q^T. C is overwritten
// with the reflectors; d (n) and e (n-1) hold T.
struct Tridiag {
  int64_t n = 0;
  std::vector<double> V;    // reflectors (row k: v_k in entries k+1..n-1)
  std::vector<double> tau;  // n
  std::vector<double> d, e;
};
void tridiagonalize(std::vector<double>& C, int64_t n, Tridiag& T);
void apply_QT(const Tridiag& T, double* x);  // x <- Q^T x
void apply_Q(const Tridiag& T, double* x);   // x <- Q x

// Eigenvalues of the bordered tridiagonal K = [[T, u], [u^T, alpha]] (order
// n+1; u may be null for plain T of order n) by bisection on inertia counts.
// Returns the k lowest eigenvalues in ascending order.
std::vector<double> lowest_eigenvalues(const Tridiag& T, const double* u, double alpha, int k);
// The same for P <= 4 bordered problems that share T (borders u[q], corners
// alpha[q], all non-null), their bisections advanced together so that their
// inertia counts, each a chain of dependent divisions, overlap: ev[q] is
// exactly what lowest_eigenvalues(T, u[q], alpha[q], k) returns.
void lowest_eigenvalues_group(const Tridiag& T, int P, const double* const* u, const double* alpha, int k,
                              std::vector<double>* ev);
// Eigenvector of K for eigenvalue mu by inverse iteration (normalised).
// Output: y (n) and s (border coordinate; unused when u is null).
void eigenvector(const Tridiag& T, const double* u, double alpha, double mu, double* y, double* s);
// Eigenvector of K for eigenvalue mu by inverse iteration from the start
// vector [y0; s0] (normalised). Within a repeated eigenvalue the iteration
// keeps the direction of the start vector's projection onto the eigenspace.
void eigenvector_from(const Tridiag& T, const double* u, double alpha, double mu, const double* y0, double s0,
                      double* y, double* s);
// Algorithm 2 (a) in the coordinates of K: v = [vy; vs] are the coordinates
// of u_i. Among the eigenvalues ev (ascending) the eigenvector x with the
// largest |x . v| (the largest component of u_i; within a repeated eigenvalue
// the normalised projection of v onto its eigenspace), the first of equal
// values (to 1e-10 relative) winning. Returns its index; y, s: x with
// x . v > 0; *proj = x . v.
int select_projection(const Tridiag& T, const double* u, double alpha, const std::vector<double>& ev,
                      const double* vy, double vs, double* y, double* s, double* proj);
// |s| of the normalised eigenvector of K for eigenvalue mu (border weight),
// O(n): 1/sqrt(1 + |(T - mu)^{-1} u|^2) when [(T - mu)^{-1} u; -1] is an
// eigenvector of K to 1e-9 |K| relative residual, and 0 otherwise (mu is then
// an eigenvalue of T whose eigenvectors are orthogonal to u, as in degenerate
// or symmetric spectra, and K's eigenvector is [q; 0]).
double border_weight(const Tridiag& T, const double* u, double alpha, double mu);

}  // namespace dense
}  // namespace mlc
