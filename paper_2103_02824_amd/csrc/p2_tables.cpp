// Reference tables of the P2 space (layout in p2.h): the 27-point conical
// product rule and the basis values, derivatives and element-matrix pieces
// at its points.
#include <cmath>

#include "p2.h"

namespace mlc {

namespace {

// 3-point Gauss rule on [0, 1] for the weight (1 - u)^alpha. Moments
// m_k = int_0^1 u^k (1-u)^alpha du = k! alpha! / (k + alpha + 1)!; the monic
// cubic orthogonal to 1, u, u^2 solves the Hankel system
// sum_j c_j m_{k+j} = -m_{k+3}; its three roots lie in (0, 1) and are found
// by bisection between its sign changes; the weights solve
// sum_i w_i x_i^k = m_k, k = 0, 1, 2.
void gauss_jacobi3(int alpha, double x[3], double w[3]) {
  long double m[6];
  for (int k = 0; k < 6; ++k) {
    long double num = 1.0L, den = 1.0L;
    for (int i = 2; i <= k; ++i) num *= i;
    for (int i = 2; i <= alpha; ++i) num *= i;
    for (int i = 2; i <= k + alpha + 1; ++i) den *= i;
    m[k] = num / den;
  }
  // Hankel system H c = r, H[k][j] = m[k + j], r[k] = -m[k + 3] (Gaussian elimination, partial pivoting)
  long double H[3][4];
  for (int k = 0; k < 3; ++k) {
    for (int j = 0; j < 3; ++j) H[k][j] = m[k + j];
    H[k][3] = -m[k + 3];
  }
  for (int p = 0; p < 3; ++p) {
    int piv = p;
    for (int r = p + 1; r < 3; ++r)
      if (std::fabs((double)H[r][p]) > std::fabs((double)H[piv][p])) piv = r;
    for (int j = 0; j < 4; ++j) std::swap(H[p][j], H[piv][j]);
    for (int r = p + 1; r < 3; ++r) {
      long double f = H[r][p] / H[p][p];
      for (int j = p; j < 4; ++j) H[r][j] -= f * H[p][j];
    }
  }
  long double cc[3];
  for (int p = 2; p >= 0; --p) {
    long double v = H[p][3];
    for (int j = p + 1; j < 3; ++j) v -= H[p][j] * cc[j];
    cc[p] = v / H[p][p];
  }
  auto poly = [&](long double u) { return ((u + cc[2]) * u + cc[1]) * u + cc[0]; };
  int found = 0;
  const int G = 4096;
  long double a = 0.0L, fa = poly(a);
  for (int g = 1; g <= G && found < 3; ++g) {
    long double b = (long double)g / G, fb = poly(b);
    if (fa == 0.0L) {
      x[found++] = (double)a;
    } else if ((fa < 0) != (fb < 0)) {
      long double lo = a, hi = b, flo = fa;
      for (int it = 0; it < 200; ++it) {
        long double mid = 0.5L * (lo + hi), fm = poly(mid);
        if ((fm < 0) == (flo < 0)) {
          lo = mid;
          flo = fm;
        } else {
          hi = mid;
        }
      }
      x[found++] = (double)(0.5L * (lo + hi));
    }
    a = b;
    fa = fb;
  }
  // weights: Vandermonde V[k][i] = x_i^k
  long double V[3][4];
  for (int k = 0; k < 3; ++k) {
    for (int i = 0; i < 3; ++i) V[k][i] = std::pow((long double)x[i], (long double)k);
    V[k][3] = m[k];
  }
  for (int p = 0; p < 3; ++p) {
    int piv = p;
    for (int r = p + 1; r < 3; ++r)
      if (std::fabs((double)V[r][p]) > std::fabs((double)V[piv][p])) piv = r;
    for (int j = 0; j < 4; ++j) std::swap(V[p][j], V[piv][j]);
    for (int r = p + 1; r < 3; ++r) {
      long double f = V[r][p] / V[p][p];
      for (int j = p; j < 4; ++j) V[r][j] -= f * V[p][j];
    }
  }
  for (int p = 2; p >= 0; --p) {
    long double v = V[p][3];
    for (int j = p + 1; j < 3; ++j) v -= V[p][j] * (long double)w[j];
    w[p] = (double)(v / V[p][p]);
  }
}

const int EDGE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};

}  // namespace

void p2_tables(std::vector<double>& tab) {
  tab.assign(P2_TAB, 0.0);
  double xu[3], wu[3], xv[3], wv[3], xw[3], ww[3];
  gauss_jacobi3(2, xu, wu);
  gauss_jacobi3(1, xv, wv);
  gauss_jacobi3(0, xw, ww);
  int q = 0;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k, ++q) {
        const double xi = xu[i], eta = (1.0 - xu[i]) * xv[j], zeta = (1.0 - xu[i]) * (1.0 - xv[j]) * xw[k];
        double* L = &tab[P2_T_L + 4 * q];
        L[0] = 1.0 - xi - eta - zeta;
        L[1] = xi;
        L[2] = eta;
        L[3] = zeta;
        tab[P2_T_W + q] = 6.0 * wu[i] * wv[j] * ww[k];
        double* B = &tab[P2_T_B + P2_NE * q];
        double* D = &tab[P2_T_D + 4 * P2_NE * q];
        for (int a = 0; a < 4; ++a) {
          B[a] = L[a] * (2.0 * L[a] - 1.0);
          D[4 * a + a] = 4.0 * L[a] - 1.0;
        }
        for (int e = 0; e < 6; ++e) {
          const int a = EDGE[e][0], b = EDGE[e][1];
          B[4 + e] = 4.0 * L[a] * L[b];
          D[4 * (4 + e) + a] = 4.0 * L[b];
          D[4 * (4 + e) + b] = 4.0 * L[a];
        }
      }
  int p = 0;
  for (int a = 0; a < P2_NE; ++a)
    for (int b = a; b < P2_NE; ++b, ++p) {
      double mm = 0.0;
      for (int r = 0; r < P2_NQ; ++r)
        mm += tab[P2_T_W + r] * tab[P2_T_B + P2_NE * r + a] * tab[P2_T_B + P2_NE * r + b];
      tab[P2_T_MM + p] = mm;
      int k = 0;
      for (int c = 0; c < 4; ++c)
        for (int d = c; d < 4; ++d, ++k) {
          double s = 0.0;
          for (int r = 0; r < P2_NQ; ++r) {
            const double* D = &tab[P2_T_D + 4 * P2_NE * r];
            double v = D[4 * a + c] * D[4 * b + d];
            if (d != c) v += D[4 * a + d] * D[4 * b + c];
            s += tab[P2_T_W + r] * v;
          }
          tab[P2_T_SK + 10 * p + k] = s;
        }
    }
}

}  // namespace mlc
