// Host FP64 dense linear algebra, written for the small problems of the
// method (order N_H + 1 of a few thousand at most). Parallel loops use
// OpenMP over independent rows.
#include "dense.h"

#include <algorithm>
#include <cmath>
#include <limits>

namespace mlc {
namespace dense {

bool cholesky(std::vector<double>& A, int64_t n) {
  // row-oriented: L_ij = (A_ij - sum_{k<j} L_ik L_jk) / L_jj, rows contiguous
  for (int64_t i = 0; i < n; ++i) {
    double* Li = &A[i * n];
    for (int64_t j = 0; j <= i; ++j) {
      const double* Lj = &A[j * n];
      double s = Li[j];
      for (int64_t k = 0; k < j; ++k) s -= Li[k] * Lj[k];
      if (j == i) {
        if (!(s > 0.0)) return false;
        Li[i] = std::sqrt(s);
      } else {
        Li[j] = s / Lj[j];
      }
    }
    for (int64_t j = i + 1; j < n; ++j) Li[j] = 0.0;
  }
  return true;
}

void forward(const std::vector<double>& L, int64_t n, double* x) {
  for (int64_t i = 0; i < n; ++i) {
    const double* Li = &L[i * n];
    double s = x[i];
    for (int64_t k = 0; k < i; ++k) s -= Li[k] * x[k];
    x[i] = s / Li[i];
  }
}

void backward(const std::vector<double>& L, int64_t n, double* x) {
  for (int64_t i = n - 1; i >= 0; --i) {
    double s = x[i];
    for (int64_t k = i + 1; k < n; ++k) s -= L[k * n + i] * x[k];
    x[i] = s / L[i * n + i];
  }
}

namespace {

// forward() on nb <= B right-hand sides at once, stored interleaved
// (X[k B + b] is entry k of right-hand side b): each row of L is read once
// for all of them instead of once per right-hand side. Every right-hand side
// takes the same operations in the same order as forward(), so the results
// are the same.
template <int B>
void forward_block(const std::vector<double>& L, int64_t n, double* X, int nb) {
  for (int64_t i = 0; i < n; ++i) {
    const double* Li = &L[i * n];
    double s[B];
    for (int b = 0; b < B; ++b) s[b] = X[i * B + b];
    for (int64_t k = 0; k < i; ++k) {
      const double lk = Li[k];
      const double* xk = &X[k * B];
      for (int b = 0; b < B; ++b) s[b] -= lk * xk[b];
    }
    for (int b = 0; b < B; ++b) X[i * B + b] = s[b] / Li[i];
  }
  (void)nb;
}

constexpr int CONG_B = 16;  // right-hand sides per pass over L

}  // namespace

void congruence(const std::vector<double>& L, const std::vector<double>& A, int64_t n, std::vector<double>& C) {
  const int64_t nblk = (n + CONG_B - 1) / CONG_B;
  // X = L^{-1} A: column j of A (= row j, A symmetric) solved into row j of Xt,
  // CONG_B columns per pass (the unused slots of the last pass hold zeros)
  std::vector<double> Xt(n * n);
#pragma omp parallel
  {
    std::vector<double> X(n * CONG_B);
#pragma omp for schedule(dynamic, 1)
    for (int64_t blk = 0; blk < nblk; ++blk) {
      const int64_t j0 = blk * CONG_B;
      const int nb = (int)std::min<int64_t>(CONG_B, n - j0);
      for (int64_t i = 0; i < n; ++i)
        for (int b = 0; b < CONG_B; ++b) X[i * CONG_B + b] = b < nb ? A[(j0 + b) * n + i] : 0.0;
      forward_block<CONG_B>(L, n, X.data(), nb);
      for (int b = 0; b < nb; ++b)
        for (int64_t i = 0; i < n; ++i) Xt[(j0 + b) * n + i] = X[i * CONG_B + b];
    }
  }
  // C = L^{-1} X^T: column j of X^T = row j of X = column j of Xt
  C.assign(n * n, 0.0);
#pragma omp parallel
  {
    std::vector<double> X(n * CONG_B);
#pragma omp for schedule(dynamic, 1)
    for (int64_t blk = 0; blk < nblk; ++blk) {
      const int64_t j0 = blk * CONG_B;
      const int nb = (int)std::min<int64_t>(CONG_B, n - j0);
      for (int64_t i = 0; i < n; ++i)
        for (int b = 0; b < CONG_B; ++b) X[i * CONG_B + b] = b < nb ? Xt[i * n + j0 + b] : 0.0;
      forward_block<CONG_B>(L, n, X.data(), nb);
      for (int b = 0; b < nb; ++b)
        for (int64_t i = 0; i < n; ++i) C[(j0 + b) * n + i] = X[i * CONG_B + b];
    }
  }
  // symmetrise against rounding
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < i; ++j) {
      double v = 0.5 * (C[i * n + j] + C[j * n + i]);
      C[i * n + j] = v;
      C[j * n + i] = v;
    }
}

// Householder reduction, one column k at a time: v from column k below the
// diagonal, p = tau C22 v, w = p - (tau/2)(p.v) v, C22 -= v w^T + w v^T.
// The rank-2 update of column k is applied row by row in the same pass that
// forms the next column's product C22 v: first the next column itself is
// brought up to date (it defines the next reflector), then each row of the
// trailing matrix is updated and, while it is in cache, multiplied by the
// next v. Every element receives the same operations in the same order as
// with separate passes (update, then product), so the result is the same;
// the trailing matrix is streamed twice per column instead of three times.
void tridiagonalize(std::vector<double>& C, int64_t n, Tridiag& T) {
  T.n = n;
  T.V.assign(n * n, 0.0);
  T.tau.assign(n, 0.0);
  T.d.assign(n, 0.0);
  T.e.assign(n > 1 ? n - 1 : 0, 0.0);
  std::vector<double> v(n), p(n);
  // pending rank-2 update of rows and columns q0..n-1: C[r][c] -= xu[r-q0] wu[c-q0] + wu[r-q0] xu[c-q0]
  std::vector<double> xu(n), wu(n);
  bool pending = false;
  int64_t q0 = 0;
  // apply the pending update to row r, columns c0..n-1
  auto update_row = [&](int64_t r, int64_t c0) {
    double* Cr = &C[r * n];
    const double xi = xu[r - q0], wi = wu[r - q0];
    for (int64_t c = c0; c < n; ++c) Cr[c] -= xi * wu[c - q0] + wi * xu[c - q0];
  };
  for (int64_t k = 0; k + 2 < n; ++k) {
    int64_t m = n - k - 1;  // trailing size
    // column k (rows k..n-1) brought up to date
    if (pending)
      for (int64_t r = k; r < n; ++r) {
        const int64_t i = r - q0;
        C[r * n + k] -= xu[i] * wu[0] + wu[i] * xu[0];
      }
    double* x = &v[k + 1];
    double nrm2 = 0.0;
    for (int64_t i = 0; i < m; ++i) {
      x[i] = C[(k + 1 + i) * n + k];
      nrm2 += x[i] * x[i];
    }
    double nrm = std::sqrt(nrm2);
    T.d[k] = C[k * n + k];
    if (nrm == 0.0) {
      T.e[k] = 0.0;
      T.tau[k] = 0.0;
      // no reflector: finish the pending update of rows k..n-1
      if (pending) {
#pragma omp parallel for schedule(static) if (m > 128)
        for (int64_t r = k; r < n; ++r) update_row(r, k + 1);
        pending = false;
      }
      continue;
    }
    double alpha = x[0] >= 0 ? -nrm : nrm;  // e_k
    x[0] -= alpha;                          // v = x - alpha e1
    // vv = |x - alpha e1|^2 computed directly for safety
    double vv = 0.0;
    for (int64_t i = 0; i < m; ++i) vv += x[i] * x[i];
    double tau = 2.0 / vv;
    T.e[k] = alpha;
    T.tau[k] = tau;
    for (int64_t i = 0; i < m; ++i) T.V[k * n + k + 1 + i] = x[i];
    // the pending update of row k (columns k+1..), then of each trailing row
    // together with p = tau * C22 v
    // (four rows at a time: their sums are independent chains, each in its
    // own order, so they overlap in the floating-point pipeline)
    if (pending) update_row(k, k + 1);
    const int64_t m4 = (m + 3) / 4;
#pragma omp parallel for schedule(static) if (m > 128)
    for (int64_t i4 = 0; i4 < m4; ++i4) {
      const int64_t i0 = 4 * i4;
      if (i0 + 4 <= m) {
        if (pending)
          for (int64_t i = i0; i < i0 + 4; ++i) update_row(k + 1 + i, k + 1);
        const double* C0 = &C[(k + 1 + i0) * n + k + 1];
        const double* C1 = C0 + n;
        const double* C2 = C1 + n;
        const double* C3 = C2 + n;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        for (int64_t j = 0; j < m; ++j) {
          const double xj = x[j];
          s0 += C0[j] * xj;
          s1 += C1[j] * xj;
          s2 += C2[j] * xj;
          s3 += C3[j] * xj;
        }
        p[k + 1 + i0] = tau * s0;
        p[k + 2 + i0] = tau * s1;
        p[k + 3 + i0] = tau * s2;
        p[k + 4 + i0] = tau * s3;
      } else {
        for (int64_t i = i0; i < m; ++i) {
          if (pending) update_row(k + 1 + i, k + 1);
          const double* Ci = &C[(k + 1 + i) * n + k + 1];
          double s = 0.0;
          for (int64_t j = 0; j < m; ++j) s += Ci[j] * x[j];
          p[k + 1 + i] = tau * s;
        }
      }
    }
    double pv = 0.0;
    for (int64_t i = 0; i < m; ++i) pv += p[k + 1 + i] * x[i];
    double h = 0.5 * tau * pv;
    for (int64_t i = 0; i < m; ++i) p[k + 1 + i] -= h * x[i];  // w
    // this column's update (rows and columns k+1..n-1) becomes the pending one
    q0 = k + 1;
    for (int64_t i = 0; i < m; ++i) {
      xu[i] = x[i];
      wu[i] = p[k + 1 + i];
    }
    pending = true;
  }
  if (pending) {
    const int64_t k0 = q0;
#pragma omp parallel for schedule(static) if (n - k0 > 128)
    for (int64_t r = k0; r < n; ++r) update_row(r, k0);
  }
  if (n >= 2) {
    T.d[n - 2] = C[(n - 2) * n + n - 2];
    T.e[n - 2] = C[(n - 1) * n + n - 2];
  }
  T.d[n - 1] = C[(n - 1) * n + n - 1];
}

// Q = H_0 H_1 ... H_{n-3}, H_k = I - tau_k v_k v_k^T
void apply_QT(const Tridiag& T, double* x) {
  int64_t n = T.n;
  for (int64_t k = 0; k + 2 < n; ++k) {
    if (T.tau[k] == 0.0) continue;
    const double* v = &T.V[k * n];
    double s = 0.0;
    for (int64_t i = k + 1; i < n; ++i) s += v[i] * x[i];
    s *= T.tau[k];
    for (int64_t i = k + 1; i < n; ++i) x[i] -= s * v[i];
  }
}

void apply_Q(const Tridiag& T, double* x) {
  int64_t n = T.n;
  for (int64_t k = n - 3; k >= 0; --k) {
    if (T.tau[k] == 0.0) continue;
    const double* v = &T.V[k * n];
    double s = 0.0;
    for (int64_t i = k + 1; i < n; ++i) s += v[i] * x[i];
    s *= T.tau[k];
    for (int64_t i = k + 1; i < n; ++i) x[i] -= s * v[i];
  }
}

namespace {

// Number of eigenvalues of [[T, u],[u^T, alpha]] (or of T if u is null) that
// are smaller than mu: negative pivots of the LDL^T factorisation of
// T - mu I plus the sign of the Schur complement of the border.
int64_t count_below(const Tridiag& T, const double* u, double alpha, double mu, double pivmin) {
  int64_t n = T.n;
  int64_t cnt = 0;
  double dprev = 1.0, wprev = 0.0, schur = alpha - mu;
  for (int64_t j = 0; j < n; ++j) {
    double dj = T.d[j] - mu;
    double wj = u ? u[j] : 0.0;
    if (j > 0) {
      double ej = T.e[j - 1];
      dj -= ej * ej / dprev;
      wj -= ej / dprev * wprev;
    }
    if (std::fabs(dj) < pivmin) dj = -pivmin;
    if (dj < 0) ++cnt;
    if (u) schur -= wj * wj / dj;
    dprev = dj;
    wprev = wj;
  }
  if (u && schur < 0) ++cnt;
  return cnt;
}

double gersh(const Tridiag& T, const double* u, double alpha, double* lo) {
  int64_t n = T.n;
  double mn = 1e300, mx = -1e300, su = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    double r = (j > 0 ? std::fabs(T.e[j - 1]) : 0.0) + (j + 1 < n ? std::fabs(T.e[j]) : 0.0) +
               (u ? std::fabs(u[j]) : 0.0);
    mn = std::min(mn, T.d[j] - r);
    mx = std::max(mx, T.d[j] + r);
    if (u) su += std::fabs(u[j]);
  }
  if (u) {
    mn = std::min(mn, alpha - su);
    mx = std::max(mx, alpha + su);
  }
  *lo = mn;
  return mx;
}

// Solve (K - mu I) [x; t] = [r; q] for the bordered tridiagonal (u may be null).
void bordered_solve(const Tridiag& T, const double* u, double alpha, double mu, const double* r, double q,
                    double* x, double* t) {
  int64_t n = T.n;
  double eps = std::numeric_limits<double>::epsilon();
  double scale = 0.0;
  for (int64_t j = 0; j < n; ++j) scale = std::max(scale, std::fabs(T.d[j]) + (j < n - 1 ? std::fabs(T.e[j]) : 0));
  double pivmin = eps * std::max(scale, 1e-300);
  std::vector<double> dd(n), yr(n), yu(n);
  // L D L^T of T - mu I, forward solves for r and u
  for (int64_t j = 0; j < n; ++j) {
    double dj = T.d[j] - mu;
    double a = r[j], b = u ? u[j] : 0.0;
    if (j > 0) {
      double l = T.e[j - 1] / dd[j - 1];
      dj -= l * T.e[j - 1];
      a -= l * yr[j - 1];
      b -= l * yu[j - 1];
    }
    if (std::fabs(dj) < pivmin) dj = dj < 0 ? -pivmin : pivmin;
    dd[j] = dj;
    yr[j] = a;
    yu[j] = b;
  }
  // backward: z = (T - mu)^{-1} * [r, u]
  std::vector<double> zr(n), zu(n);
  for (int64_t j = n - 1; j >= 0; --j) {
    double a = yr[j] / dd[j], b = yu[j] / dd[j];
    if (j + 1 < n) {
      double l = T.e[j] / dd[j];
      a -= l * zr[j + 1];
      b -= l * zu[j + 1];
    }
    zr[j] = a;
    zu[j] = b;
  }
  if (!u) {
    for (int64_t j = 0; j < n; ++j) x[j] = zr[j];
    *t = 0.0;
    return;
  }
  double ur = 0.0, uu = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    ur += u[j] * zr[j];
    uu += u[j] * zu[j];
  }
  double s = alpha - mu - uu;
  if (std::fabs(s) < pivmin) s = s < 0 ? -pivmin : pivmin;
  double tt = (q - ur) / s;
  for (int64_t j = 0; j < n; ++j) x[j] = zr[j] - zu[j] * tt;
  *t = tt;
}

}  // namespace

std::vector<double> lowest_eigenvalues(const Tridiag& T, const double* u, double alpha, int k) {
  double lo, hi = gersh(T, u, alpha, &lo);
  double eps = std::numeric_limits<double>::epsilon();
  double scale = std::max(std::fabs(lo), std::fabs(hi));
  double pivmin = eps * std::max(scale, 1e-300) * 1e-3;
  std::vector<double> ev(k);
  double a0 = lo - 1e-12 * scale - 1e-300, b0 = hi + 1e-12 * scale;
  for (int j = 0; j < k; ++j) {
    // find mu with count_below(mu) <= j < count_below(next)
    double a = j > 0 ? std::max(a0, ev[j - 1] - 4 * eps * scale) : a0, b = b0;
    for (int it = 0; it < 200; ++it) {
      double m = 0.5 * (a + b);
      if (b - a <= 2.0 * eps * std::max(std::fabs(a), std::fabs(b)) + 1e-300 || m == a || m == b) break;
      if (count_below(T, u, alpha, m, pivmin) > j)
        b = m;
      else
        a = m;
    }
    ev[j] = 0.5 * (a + b);
  }
  return ev;
}

namespace {

constexpr int GROUP_P = 4;

// count_below for GROUP_P problems at once (the same operations per problem)
void count_below_group(const Tridiag& T, const double* const* u, const double* alpha, const double* mu,
                       const double* pivmin, int64_t* cnt) {
  const int64_t n = T.n;
  int64_t c[GROUP_P];
  double dprev[GROUP_P], wprev[GROUP_P], schur[GROUP_P];
  for (int q = 0; q < GROUP_P; ++q) {
    c[q] = 0;
    dprev[q] = 1.0;
    wprev[q] = 0.0;
    schur[q] = alpha[q] - mu[q];
  }
  for (int64_t j = 0; j < n; ++j) {
    for (int q = 0; q < GROUP_P; ++q) {
      double dj = T.d[j] - mu[q];
      double wj = u[q][j];
      if (j > 0) {
        double ej = T.e[j - 1];
        dj -= ej * ej / dprev[q];
        wj -= ej / dprev[q] * wprev[q];
      }
      if (std::fabs(dj) < pivmin[q]) dj = -pivmin[q];
      if (dj < 0) ++c[q];
      schur[q] -= wj * wj / dj;
      dprev[q] = dj;
      wprev[q] = wj;
    }
  }
  for (int q = 0; q < GROUP_P; ++q) cnt[q] = c[q] + (schur[q] < 0 ? 1 : 0);
}

// the bisection of lowest_eigenvalues as a state machine: next() gives the
// next point to count at (false once all k eigenvalues are found), feed()
// takes its count
struct Bisection {
  double a0, b0, eps, scale, pivmin, a, b;
  int k, j, it;
  std::vector<double>* ev;
  void start() {
    a = j > 0 ? std::max(a0, (*ev)[j - 1] - 4 * eps * scale) : a0;
    b = b0;
    it = 0;
  }
  bool next(double* m) {
    while (j < k) {
      const double mm = 0.5 * (a + b);
      if (it >= 200 || b - a <= 2.0 * eps * std::max(std::fabs(a), std::fabs(b)) + 1e-300 || mm == a || mm == b) {
        (*ev)[j] = 0.5 * (a + b);
        if (++j < k) start();
        continue;
      }
      *m = mm;
      return true;
    }
    return false;
  }
  void feed(double m, int64_t cnt) {
    if (cnt > j)
      b = m;
    else
      a = m;
    ++it;
  }
};

}  // namespace

void lowest_eigenvalues_group(const Tridiag& T, int P, const double* const* u, const double* alpha, int k,
                              std::vector<double>* ev) {
  Bisection B[GROUP_P];
  for (int q = 0; q < P; ++q) {
    double lo, hi = gersh(T, u[q], alpha[q], &lo);
    Bisection& s = B[q];
    s.eps = std::numeric_limits<double>::epsilon();
    s.scale = std::max(std::fabs(lo), std::fabs(hi));
    s.pivmin = s.eps * std::max(s.scale, 1e-300) * 1e-3;
    s.a0 = lo - 1e-12 * s.scale - 1e-300;
    s.b0 = hi + 1e-12 * s.scale;
    s.k = k;
    s.j = 0;
    s.ev = &ev[q];
    ev[q].assign(k, 0.0);
    if (k > 0) s.start();
  }
  for (;;) {
    double m[GROUP_P], mu[GROUP_P], pv[GROUP_P], al[GROUP_P];
    const double* uu[GROUP_P];
    bool need[GROUP_P];
    int live = -1;
    for (int q = 0; q < GROUP_P; ++q) {
      need[q] = q < P && B[q].next(&m[q]);
      if (need[q]) live = q;
    }
    if (live < 0) break;
    // slots without a pending count repeat a live one (their counts are not used)
    for (int q = 0; q < GROUP_P; ++q) {
      const int r = need[q] ? q : live;
      uu[q] = u[r];
      al[q] = alpha[r];
      mu[q] = m[r];
      pv[q] = B[r].pivmin;
    }
    int64_t cnt[GROUP_P];
    count_below_group(T, uu, al, mu, pv, cnt);
    for (int q = 0; q < GROUP_P; ++q)
      if (need[q]) B[q].feed(m[q], cnt[q]);
  }
}

double border_weight(const Tridiag& T, const double* u, double alpha, double mu) {
  // The closed form takes the eigenvector to be x = [z; -1] with
  // z = (T - mu)^{-1} u, which holds when mu solves the secular equation
  // alpha - mu - u^T (T - mu)^{-1} u = 0. An eigenvalue of K that is also an
  // eigenvalue of T with an eigenvector q orthogonal to u (degenerate or
  // symmetric spectra) has the eigenvector [q; 0] instead, border weight
  // zero; there the secular equation does not hold and x is not an
  // eigenvector. So x is accepted only if its residual |(K - mu) x| / |x| is
  // below 1e-9 |K| (a coupled eigenpair of weight above ~1e-6 meets it with
  // orders to spare: its residual is |f'(mu)| |dmu| / |x| ~ |x| eps |K|).
  const int64_t n = T.n;
  std::vector<double> z(n);
  double tt;
  bordered_solve(T, nullptr, 0.0, mu, u, 0.0, z.data(), &tt);
  double z2 = 0.0, uz = 0.0, r2 = 0.0;
  for (int64_t j = 0; j < n; ++j) {
    z2 += z[j] * z[j];
    uz += u[j] * z[j];
    double r = (T.d[j] - mu) * z[j] - u[j];
    if (j > 0) r += T.e[j - 1] * z[j - 1];
    if (j + 1 < n) r += T.e[j] * z[j + 1];
    r2 += r * r;
  }
  const double f = alpha - mu - uz;
  double lo, hi = gersh(T, u, alpha, &lo);
  const double knorm = std::max(std::fabs(lo), std::fabs(hi));
  if (!(std::sqrt((r2 + f * f) / (1.0 + z2)) <= 1e-9 * knorm)) return 0.0;
  return 1.0 / std::sqrt(1.0 + z2);
}

void eigenvector_from(const Tridiag& T, const double* u, double alpha, double mu, const double* y0, double s0,
                      double* y, double* s) {
  const int64_t n = T.n;
  std::vector<double> x(y0, y0 + n), xn(n);
  double t = u ? s0 : 0.0, tn;
  const double eps = std::numeric_limits<double>::epsilon();
  const double mus = mu + eps * std::max(1.0, std::fabs(mu)) * 16.0;
  for (int it = 0; it < 3; ++it) {
    double nr = t * t;
    for (int64_t j = 0; j < n; ++j) nr += x[j] * x[j];
    nr = std::sqrt(nr);
    if (!(nr > 0.0)) break;
    for (int64_t j = 0; j < n; ++j) x[j] /= nr;
    t /= nr;
    bordered_solve(T, u, alpha, mus, x.data(), t, xn.data(), &tn);
    x.swap(xn);
    t = u ? tn : 0.0;
  }
  double nr = t * t;
  for (int64_t j = 0; j < n; ++j) nr += x[j] * x[j];
  nr = std::sqrt(nr);
  for (int64_t j = 0; j < n; ++j) y[j] = nr > 0.0 ? x[j] / nr : 0.0;
  if (s) *s = nr > 0.0 ? t / nr : 0.0;
}

int select_projection(const Tridiag& T, const double* u, double alpha, const std::vector<double>& ev,
                      const double* vy, double vs, double* y, double* s, double* proj) {
  const int64_t n = T.n;
  std::vector<double> xy(n);
  double xs = 0.0, best = -1.0;
  int jbest = 0;
  for (int j = 0; j < (int)ev.size(); ++j) {
    eigenvector_from(T, u, alpha, ev[j], vy, vs, xy.data(), &xs);
    double p = xs * vs;
    for (int64_t k = 0; k < n; ++k) p += xy[k] * vy[k];
    const double ap = std::fabs(p);
    if (ap > best * (1.0 + 1e-10)) {
      best = ap;
      jbest = j;
      const double sg = p < 0.0 ? -1.0 : 1.0;
      for (int64_t k = 0; k < n; ++k) y[k] = sg * xy[k];
      *s = sg * xs;
    }
  }
  *proj = best;
  return jbest;
}

void eigenvector(const Tridiag& T, const double* u, double alpha, double mu, double* y, double* s) {
  int64_t n = T.n;
  std::vector<double> x(n), xn(n);
  double t = 1.0, tn;
  // start: for a bordered matrix, [-(T-mu)^{-1} u; 1]; otherwise all ones
  if (u) {
    double tt;
    bordered_solve(T, nullptr, 0.0, mu, u, 0.0, x.data(), &tt);
    for (int64_t j = 0; j < n; ++j) x[j] = -x[j];
  } else {
    for (int64_t j = 0; j < n; ++j) x[j] = 1.0 / std::sqrt((double)n) * (1.0 + 1e-3 * std::sin((double)j));
    t = 0.0;
  }
  double eps = std::numeric_limits<double>::epsilon();
  double mus = mu + eps * std::max(1.0, std::fabs(mu)) * 16.0;
  for (int it = 0; it < 3; ++it) {
    double nr = t * t;
    for (int64_t j = 0; j < n; ++j) nr += x[j] * x[j];
    nr = std::sqrt(nr);
    for (int64_t j = 0; j < n; ++j) x[j] /= nr;
    t /= nr;
    bordered_solve(T, u, alpha, mus, x.data(), t, xn.data(), &tn);
    x.swap(xn);
    t = tn;
  }
  double nr = u ? t * t : 0.0;
  for (int64_t j = 0; j < n; ++j) nr += x[j] * x[j];
  nr = std::sqrt(nr);
  for (int64_t j = 0; j < n; ++j) y[j] = x[j] / nr;
  if (s) *s = u ? t / nr : 0.0;
}

}  // namespace dense
}  // namespace mlc
