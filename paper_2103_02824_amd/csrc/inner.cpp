// Host FP64 parts of the method:
//  * Algorithm 2 (inner Hartree iteration) implemented as in Algorithm 3
//    step 2: every fine-mesh integral was precomputed on the GPU, so one inner
//    iteration only touches coarse-size data;
//  * Algorithm 1 step 1: the self-consistent Kohn-Sham solve on the coarse
//    mesh that provides the initial state, and step 4's transfer to the fine
//    mesh.
//
// The augmented eigenproblem of each orbital (eq. Eigenvalue_H_h) shares its
// coarse block A_H with every other orbital. Per inner iteration the pencil
// (A_H, M_H) is reduced once to tridiagonal form, C = L^{-1} A_H L^{-T} =
// Q T Q^T (M_H = L L^T). For orbital i the border (b, beta; c, gamma) is first
// made M-orthogonal to V_H (a = M_H^{-1} c), which turns the pencil into the
// standard symmetric problem [[T, u], [u^T, alpha]] of order N_H + 1; its
// lowest eigenvalues come from bisection on inertia counts, and the kept
// eigenvector (the largest component in span{u_i}) from inverse iteration
// started at u_i's coordinates, both O(N_H) per evaluation.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include "dense.h"
#include "inner.h"
#include "mlc_internal.h"

namespace mlc {

namespace {

// slot of the symmetric pair (j<=k) in the 10-entry element layout
inline int sym10(int j, int k) {
  if (j > k) std::swap(j, k);
  static const int base[4] = {0, 4, 7, 9};
  return base[j] + (k - j);
}
// slot of the sorted triple in the 20-entry trilinear layout
int tri20(int a, int b, int c) {
  int v[3] = {a, b, c};
  std::sort(v, v + 3);
  int k = 0;
  for (int j = 0; j < 4; ++j)
    for (int m = j; m < 4; ++m)
      for (int l = m; l < 4; ++l, ++k)
        if (j == v[0] && m == v[1] && l == v[2]) return k;
  return -1;
}

struct TriIndex {
  int idx[4][4][4];
  TriIndex() {
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b)
        for (int c = 0; c < 4; ++c) idx[a][b][c] = tri20(a, b, c);
  }
};
const TriIndex& tri_index() {
  static TriIndex t;
  return t;
}

void assemble_dense(const mlc_ctx* c, const double* cel, int stride, int off, std::vector<double>& A) {
  int64_t nH = c->nH;
  A.assign(nH * nH, 0.0);
  for (int64_t C = 0; C < c->cnt; ++C) {
    int k[4];
    for (int a = 0; a < 4; ++a) k[a] = c->cv2d[c->ctets[4 * C + a]];
    const double* e = cel + (int64_t)stride * C + off;
    for (int a = 0; a < 4; ++a) {
      if (k[a] < 0) continue;
      for (int b = 0; b < 4; ++b) {
        if (k[b] < 0) continue;
        A[(int64_t)k[a] * nH + k[b]] += e[sym10(a, b)];
      }
    }
  }
}

inline double dot(const double* a, const double* b, int64_t n) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

void symv(const std::vector<double>& A, int64_t n, const double* x, double* y) {
#pragma omp parallel for schedule(static) if (n > 512)
  for (int64_t i = 0; i < n; ++i) y[i] = dot(&A[i * n], x, n);
}

// Minimum-norm least-squares solution of the symmetric positive semidefinite
// system A x = r (order m <= 16) by cyclic Jacobi eigen-decomposition:
// eigenvalues below 1e-12 of the largest are treated as zero.
void sym_lstsq(std::vector<double> A, int m, const std::vector<double>& r, std::vector<double>& x) {
  std::vector<double> V(m * m, 0.0);
  for (int i = 0; i < m; ++i) V[i * m + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) (i == j ? tot : off) += A[i * m + j] * A[i * m + j];
    if (off <= 1e-30 * (tot + off) || off == 0.0) break;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) {
        double apq = A[p * m + q];
        if (apq == 0.0) continue;
        double th = 0.5 * (A[q * m + q] - A[p * m + p]) / apq;
        double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        double cs = 1.0 / std::sqrt(t * t + 1.0), sn = t * cs;
        for (int k = 0; k < m; ++k) {  // A <- A J
          double akp = A[k * m + p], akq = A[k * m + q];
          A[k * m + p] = cs * akp - sn * akq;
          A[k * m + q] = sn * akp + cs * akq;
        }
        for (int k = 0; k < m; ++k) {  // A <- J^T A
          double apk = A[p * m + k], aqk = A[q * m + k];
          A[p * m + k] = cs * apk - sn * aqk;
          A[q * m + k] = sn * apk + cs * aqk;
        }
        for (int k = 0; k < m; ++k) {
          double vkp = V[k * m + p], vkq = V[k * m + q];
          V[k * m + p] = cs * vkp - sn * vkq;
          V[k * m + q] = sn * vkp + cs * vkq;
        }
      }
  }
  double emax = 0.0;
  for (int i = 0; i < m; ++i) emax = std::max(emax, std::fabs(A[i * m + i]));
  x.assign(m, 0.0);
  for (int k = 0; k < m; ++k) {
    double ev = A[k * m + k];
    if (!(std::fabs(ev) > 1e-12 * emax)) continue;
    double c = 0.0;
    for (int i = 0; i < m; ++i) c += V[i * m + k] * r[i];
    c /= ev;
    for (int i = 0; i < m; ++i) x[i] += c * V[i * m + k];
  }
}

// Anderson (Pulay) mixing of a fixed-point iteration x -> x + F(x): with the
// differences dX, dF of the last m + 1 inputs and residuals, gamma minimises
// |F - dF gamma|_G, and the next input is (x - dX gamma) + beta (F - dF gamma);
// the first call takes the damped step x + beta F. G is applied by the caller
// (GF = G F) so that the normal equations need no further products with G.
struct Anderson {
  int m = 0;
  double beta = 1.0;
  std::vector<std::vector<double>> X, F, GF;
  void next(std::vector<double>& x, const std::vector<double>& f, const std::vector<double>& gf) {
    X.push_back(x);
    F.push_back(f);
    GF.push_back(gf);
    if ((int)X.size() > m + 1) {
      X.erase(X.begin());
      F.erase(F.begin());
      GF.erase(GF.begin());
    }
    const size_t len = x.size();
    const int k = (int)X.size() - 1;
    if (k == 0) {
      for (size_t a = 0; a < len; ++a) x[a] += beta * f[a];
      return;
    }
    std::vector<double> A(k * k), r(k), gam;
    for (int i = 0; i < k; ++i) {
      double ri = 0.0;
      for (size_t a = 0; a < len; ++a) ri += (GF[i + 1][a] - GF[i][a]) * f[a];
      r[i] = ri;
      for (int j = 0; j < k; ++j) {
        double aij = 0.0;
        for (size_t a = 0; a < len; ++a) aij += (F[i + 1][a] - F[i][a]) * (GF[j + 1][a] - GF[j][a]);
        A[i * k + j] = aij;
      }
    }
    for (int i = 0; i < k; ++i)  // symmetrise the rounding
      for (int j = i + 1; j < k; ++j) A[i * k + j] = A[j * k + i] = 0.5 * (A[i * k + j] + A[j * k + i]);
    sym_lstsq(A, k, r, gam);
    for (size_t a = 0; a < len; ++a) {
      double dxg = 0.0, dfg = 0.0;
      for (int i = 0; i < k; ++i) {
        dxg += (X[i + 1][a] - X[i][a]) * gam[i];
        dfg += (F[i + 1][a] - F[i][a]) * gam[i];
      }
      x[a] = (x[a] - dxg) + beta * (f[a] - dfg);
    }
  }
};

}  // namespace

// A_{H,2}(w) = sum_m T_{jkm} w_m added into dense A (scale s)
void add_trilinear_matrix(const mlc_ctx* c, const std::vector<double>& tri, const double* w, double s,
                          std::vector<double>& A) {
  const TriIndex& ti = tri_index();
  int64_t nH = c->nH;
  for (int64_t C = 0; C < c->cnt; ++C) {
    int k[4];
    double wl[4];
    for (int a = 0; a < 4; ++a) {
      k[a] = c->cv2d[c->ctets[4 * C + a]];
      wl[a] = k[a] >= 0 ? w[k[a]] : 0.0;
    }
    const double* T = &tri[20 * C];
    for (int a = 0; a < 4; ++a) {
      if (k[a] < 0) continue;
      for (int b = 0; b < 4; ++b) {
        if (k[b] < 0) continue;
        double v = 0.0;
        for (int m = 0; m < 4; ++m) v += T[ti.idx[a][b][m]] * wl[m];
        A[(int64_t)k[a] * nH + k[b]] += s * v;
      }
    }
  }
}

mlc_status inner_loop(mlc_ctx* c, const FineBlocks& fb, InnerOut& out) {
  using namespace dense;
  const int64_t nH = c->nH;
  const int N = c->N;
  const int hart = c->hartree;
  const TriIndex& ti = tri_index();
  auto t0 = std::chrono::steady_clock::now();

  std::vector<double> AfixH, G, MH, KH;
  assemble_dense(c, fb.cel_ops.data(), 40, 0, AfixH);
  assemble_dense(c, fb.cel_ops.data(), 40, 10, G);
  if (c->h_Mh_chol.empty()) {
    assemble_dense(c, fb.cel_ops.data(), 40, 20, MH);
    assemble_dense(c, fb.cel_ops.data(), 40, 30, KH);
    c->h_MH = MH;
    c->h_KH = KH;
    c->h_Mh_chol = MH;
    if (!cholesky(c->h_Mh_chol, nH)) return fail(c, MLC_ERR_NONFINITE, "coarse mass matrix not SPD");
    c->h_Kh_chol = KH;
    if (!cholesky(c->h_Kh_chol, nH)) return fail(c, MLC_ERR_NONFINITE, "coarse stiffness not SPD");
  }
  const std::vector<double>& L = c->h_Mh_chol;
  const std::vector<double>& MHd = c->h_MH;
  const std::vector<double>& KHd = c->h_KH;

  // per-orbital sparse pieces: A_h4 as element arrays, rhs assembled
  std::vector<double> rhsv(nH * N, 0.0);  // [k*N + i]
  for (int64_t C = 0; C < c->cnt; ++C)
    for (int a = 0; a < 4; ++a) {
      int k = c->cv2d[c->ctets[4 * C + a]];
      if (k < 0) continue;
      for (int i = 0; i < N; ++i) rhsv[(int64_t)k * N + i] += fb.cel_orb[(C * N + i) * 14 + 10 + a];
    }
  auto ah4_apply = [&](int i, const double* x, double* y) {  // y = A_h4,i x (coarse dof vectors)
    std::fill(y, y + nH, 0.0);
    for (int64_t C = 0; C < c->cnt; ++C) {
      int k[4];
      for (int a = 0; a < 4; ++a) k[a] = c->cv2d[c->ctets[4 * C + a]];
      const double* e = &fb.cel_orb[(C * N + i) * 14];
      for (int a = 0; a < 4; ++a) {
        if (k[a] < 0) continue;
        double s = 0.0;
        for (int b = 0; b < 4; ++b)
          if (k[b] >= 0) s += e[sym10(a, b)] * x[k[b]];
        y[k[a]] += s;
      }
    }
  };

  // Hartree system pieces (fixed in the inner loop): Schur complement of the border
  std::vector<double> yd(nH, 0.0);
  double schur = 1.0;
  if (hart) {
    for (int64_t k = 0; k < nH; ++k) yd[k] = fb.d[k];
    forward(c->h_Kh_chol, nH, yd.data());
    backward(c->h_Kh_chol, nH, yd.data());
    schur = fb.zeta - dot(fb.d.data(), yd.data(), nH);
    if (!(schur > 0.0)) return fail(c, MLC_ERR_NONFINITE, "Hartree augmented matrix not SPD");
  }

  std::vector<double> wH(nH, 0.0), phiH(nH * N, 0.0), phiH_old(nH * N, 0.0);
  std::vector<double> theta2(N, 0.0), theta2_old(N, 1.0), lam(N, 0.0);
  double th1 = hart ? 1.0 : 0.0;
  std::vector<double> AH, Cm, KpM(nH * nH);
  for (int64_t k = 0; k < nH * nH; ++k) KpM[k] = KHd[k] + MHd[k];
  std::vector<double> tmp(nH), fH(nH);
  Tridiag Tr;
  // per orbital, fixed in the inner loop: a_i = M_H^{-1} P^T M u_i and the
  // M-norm^2 of the part of u_i M-orthogonal to V_H, gamma_i - c_i . a_i
  std::vector<double> aM(nH * N), gpv(N);
  for (int i = 0; i < N; ++i) {
    double* ai = &aM[(int64_t)i * nH];
    for (int64_t k = 0; k < nH; ++k) ai[k] = fb.ptM[k * N + i];
    forward(L, nH, ai);
    backward(L, nH, ai);
    double ca = 0.0;
    for (int64_t k = 0; k < nH; ++k) ca += fb.ptM[k * N + i] * ai[k];
    const double gam = fb.utM[i * N + i];
    gpv[i] = gam - ca;
    if (!(gpv[i] > 1e-14 * std::fabs(gam))) return fail(c, MLC_ERR_NONFINITE, "auxiliary solution lies in the coarse space");
  }
  // L^T a_i: the coarse part of u_i in the M-orthonormal coordinates of V_H
  std::vector<double> LTa(nH * N, 0.0);
#pragma omp parallel for schedule(static) if (N > 1)
  for (int i = 0; i < N; ++i) {
    const double* ai = &aM[(int64_t)i * nH];
    double* o = &LTa[(int64_t)i * nH];
    for (int64_t r = 0; r < nH; ++r) {
      const double* Lr = &L[r * nH];
      for (int64_t k = 0; k <= r; ++k) o[k] += Lr[k] * ai[r];
    }
  }
  int n_keep = (int)std::min<int64_t>(nH + 1, (int64_t)N + c->opt.n_extra);
  int its = 0;
  double diff = 0.0;
  mlc_status st = MLC_OK;
  int maxit = std::max(1, c->opt.inner_maxit);
  std::vector<double> xin(nH + 1), xout(nH + 1, 0.0), fres(nH + 1), gres(nH + 1);
  // per orbital, within one inner iteration: border in the tridiagonal basis,
  // corner entry, lowest eigenvalues
  std::vector<double> Ub(nH * N), alphab(N);
  std::vector<std::vector<double>> evb(N);
  // Hartree right-hand side: coarse DoF of each tet vertex (-1 on the
  // boundary), and each orbital's addends
  std::vector<int> hs_dof(hart ? 4 * c->cnt : 0);
  for (int64_t C = 0; C < (hart ? c->cnt : 0); ++C)
    for (int q = 0; q < 4; ++q) hs_dof[4 * C + q] = c->cv2d[c->ctets[4 * C + q]];
  std::vector<double> hs_tet(hart ? (int64_t)N * c->cnt * 4 : 0), hs_dofv(hart ? nH * N : 0), hs_g(N);
  Anderson mix;
  mix.m = c->opt.inner_mix_history;
  mix.beta = c->opt.inner_mix_beta;
  for (int s = 0; s < maxit; ++s) {
    its = s + 1;
    // (a) A_H = A_{H,1} + A_{H,4} + A_{H,2}(w_H) + theta1 A_{H,3}
    AH = AfixH;
    if (hart) {
      add_trilinear_matrix(c, c->h_tri, wH.data(), 1.0, AH);
      for (int64_t k = 0; k < nH * nH; ++k) AH[k] += th1 * G[k];
    }
    congruence(L, AH, nH, Cm);
    tridiagonalize(Cm, nH, Tr);
    // the N augmented problems are independent given A_H. Three passes over
    // the orbitals: their borders (one orbital per thread), the bisections
    // for their lowest eigenvalues (GROUP orbitals per thread, their inertia
    // counts advanced together), then the selection and reconstruction (one
    // orbital per thread); each orbital's arithmetic is that of one pass.
    constexpr int GROUP = 4;
    const int ngroup = (N + GROUP - 1) / GROUP;
    int bad = 0;
#pragma omp parallel if (N > 1)
    {
      std::vector<double> b(nH), Aa(nH), y(nH), tmp(nH), vy(nH);
#pragma omp for schedule(dynamic, 1)
      for (int i = 0; i < N; ++i) {
        const double* ai = &aM[(int64_t)i * nH];
        double* u = &Ub[(int64_t)i * nH];
        // border of orbital i (eqs. bdef, betadef)
        if (hart) ah4_apply(i, wH.data(), tmp.data());
        double beta = fb.utF[i * N + i] + th1 * fb.utW[i * N + i];
        for (int64_t k = 0; k < nH; ++k) {
          b[k] = fb.ptF[k * N + i] + (hart ? tmp[k] + th1 * fb.ptW[k * N + i] : 0.0);
          beta += hart ? rhsv[k * N + i] * wH[k] : 0.0;
        }
        for (int64_t k = 0; k < nH; ++k) Aa[k] = dot(&AH[k * nH], ai, nH);
        double ba = dot(b.data(), ai, nH), aAa = dot(ai, Aa.data(), nH);
        const double gp = gpv[i], sg = std::sqrt(gp);
        double bp = beta - 2.0 * ba + aAa;
        for (int64_t k = 0; k < nH; ++k) u[k] = b[k] - Aa[k];
        forward(L, nH, u);
        for (int64_t k = 0; k < nH; ++k) u[k] /= sg;
        apply_QT(Tr, u);
        alphab[i] = bp / gp;
      }
#pragma omp for schedule(dynamic, 1)
      for (int g = 0; g < ngroup; ++g) {
        const int i0 = g * GROUP, P = std::min(GROUP, N - i0);
        const double* up[GROUP];
        for (int q = 0; q < P; ++q) up[q] = &Ub[(int64_t)(i0 + q) * nH];
        lowest_eigenvalues_group(Tr, P, up, &alphab[i0], n_keep, &evb[i0]);
      }
#pragma omp for schedule(dynamic, 1) reduction(+ : bad)
      for (int i = 0; i < N; ++i) {
        const double* ai = &aM[(int64_t)i * nH];
        const double* u = &Ub[(int64_t)i * nH];
        const double sg = std::sqrt(gpv[i]);
        const double alpha = alphab[i];
        const std::vector<double>& ev = evb[i];
        // (a): the eigenfunction with the largest component in span{u_i}; u_i
        // has the coordinates [Q^T L^T a_i; sqrt(gamma')] (its coarse part P a_i
        // and its part M-orthogonal to V_H)
        std::copy(&LTa[(int64_t)i * nH], &LTa[(int64_t)i * nH] + nH, vy.begin());
        apply_QT(Tr, vy.data());
        double sv, pj;
        const int jsel = select_projection(Tr, u, alpha, ev, vy.data(), sg, y.data(), &sv, &pj);
        (void)pj;
        apply_Q(Tr, y.data());
        backward(L, nH, y.data());
        double t2 = sv / sg;
        for (int64_t k = 0; k < nH; ++k) phiH[k * N + i] = y[k] - t2 * ai[k];
        theta2[i] = t2;
        lam[i] = ev[jsel];
        bad += !std::isfinite(t2) || !std::isfinite(lam[i]);
      }
    }
    if (bad) return fail(c, MLC_ERR_NONFINITE, "non-finite solution of an augmented problem");
    // (b) Hartree problem in W_{H,h} (eqs. Hartree_H_h, fH, gdef with the
    //     factor 2, the theta2^2 term and the occupations)
    if (hart) {
      // each orbital's addends in parallel (its trilinear terms per coarse tet
      // and vertex, its A_h4 and rhs terms per coarse DoF, its scalar), then
      // added into fH and gsum in orbital order, as one pass would
#pragma omp parallel if (N > 1)
      {
        std::vector<double> ph(nH), tq(nH);
#pragma omp for schedule(dynamic, 1)
        for (int i = 0; i < N; ++i) {
          double f = c->occ[i];
          if (f == 0.0) continue;
          for (int64_t k = 0; k < nH; ++k) ph[k] = phiH[k * N + i];
          double t2 = theta2[i];
          double* sa = &hs_tet[(int64_t)i * c->cnt * 4];
          // (phi_H^2, psi_j) through the trilinear tensor
          for (int64_t C = 0; C < c->cnt; ++C) {
            const int* k = &hs_dof[4 * C];
            double pl[4];
            for (int q = 0; q < 4; ++q) pl[q] = k[q] >= 0 ? ph[k[q]] : 0.0;
            const double* T = &c->h_tri[20 * C];
            for (int j = 0; j < 4; ++j) {
              if (k[j] < 0) continue;
              double sacc = 0.0;
              for (int m = 0; m < 4; ++m)
                for (int l = 0; l < 4; ++l) sacc += T[ti.idx[j][m][l]] * pl[m] * pl[l];
              sa[4 * C + j] = f * sacc;
            }
          }
          ah4_apply(i, ph.data(), tq.data());
          double* so = &hs_dofv[(int64_t)i * nH];
          for (int64_t k = 0; k < nH; ++k) so[k] = f * (2.0 * t2 * tq[k] + t2 * t2 * rhsv[k * N + i]);
          symv(G, nH, ph.data(), tq.data());
          double g1 = dot(ph.data(), tq.data(), nH);
          double g2 = 0.0;
          for (int64_t k = 0; k < nH; ++k) g2 += fb.ptW[k * N + i] * ph[k];
          hs_g[i] = f * (g1 + 2.0 * t2 * g2 + t2 * t2 * fb.utW[i * N + i]);
        }
      }
      std::fill(fH.begin(), fH.end(), 0.0);
      double gsum = 0.0;
      for (int i = 0; i < N; ++i) {
        if (c->occ[i] == 0.0) continue;
        const double* sa = &hs_tet[(int64_t)i * c->cnt * 4];
        for (int64_t C = 0; C < c->cnt; ++C)
          for (int j = 0; j < 4; ++j) {
            const int k = hs_dof[4 * C + j];
            if (k >= 0) fH[k] += sa[4 * C + j];
          }
        const double* so = &hs_dofv[(int64_t)i * nH];
        for (int64_t k = 0; k < nH; ++k) fH[k] += so[k];
        gsum += hs_g[i];
      }
      const double fourpi = 4.0 * 3.14159265358979323846;
      std::vector<double> r1(nH);
      for (int64_t k = 0; k < nH; ++k) r1[k] = fourpi * fH[k] - fb.liftH[k];
      double r2 = fourpi * gsum - fb.liftT;
      forward(c->h_Kh_chol, nH, r1.data());
      backward(c->h_Kh_chol, nH, r1.data());
      double t1 = (r2 - dot(fb.d.data(), r1.data(), nH)) / schur;
      for (int64_t k = 0; k < nH; ++k) xout[k] = r1[k] - yd[k] * t1;
      xout[nH] = t1;
    }
    // (c) ||Phi^{s+1} - Phi^s||_{H^1} in the basis [P, u_i]
    double d2 = 0.0;
    std::vector<double> dp(nH), kd(nH);
    for (int i = 0; i < N; ++i) {
      for (int64_t k = 0; k < nH; ++k) dp[k] = phiH[k * N + i] - phiH_old[k * N + i];
      double dt = theta2[i] - theta2_old[i];
      symv(KpM, nH, dp.data(), kd.data());
      double cross = 0.0;
      for (int64_t k = 0; k < nH; ++k) cross += dp[k] * (fb.ptK[k * N + i] + fb.ptM[k * N + i]);
      d2 += dot(dp.data(), kd.data(), nH) + 2.0 * dt * cross + dt * dt * (fb.utK[i * N + i] + fb.utM[i * N + i]);
    }
    diff = std::sqrt(std::max(d2, 0.0));
    phiH_old = phiH;
    theta2_old = theta2;
    if (!hart) break;
    const bool done = diff < c->opt.inner_tol;
    if (!done && s == maxit - 1) st = MLC_WARN_INNER_MAXIT;
    if (done || s == maxit - 1 || c->opt.inner_mix_history <= 0) {
      // output (and, unmixed, the next input): the Hartree potential of the new orbitals
      std::copy(xout.begin(), xout.begin() + nH, wH.begin());
      th1 = xout[nH];
      if (done || s == maxit - 1) break;
      continue;
    }
    // next input by Anderson mixing in the energy inner product of W_{H,h}:
    // G [x_h; x_t] = [K_H x_h + d x_t; d.x_h + zeta x_t]
    std::copy(wH.begin(), wH.end(), xin.begin());
    xin[nH] = th1;
    for (int64_t k = 0; k <= nH; ++k) fres[k] = xout[k] - xin[k];
    symv(KHd, nH, fres.data(), gres.data());
    for (int64_t k = 0; k < nH; ++k) gres[k] += fb.d[k] * fres[nH];
    gres[nH] = dot(fb.d.data(), fres.data(), nH) + fb.zeta * fres[nH];
    mix.next(xin, fres, gres);
    std::copy(xin.begin(), xin.begin() + nH, wH.begin());
    th1 = xin[nH];
  }
  out.lam = lam;
  out.phiH = phiH;
  out.theta2 = theta2;
  out.wH = wH;
  out.theta1 = th1;
  out.iters = its;
  out.last_diff = diff;
  out.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return st;
}

// ---------------------------------------------------------------------------
// The joint-space variant (the earlier multilevel correction method the paper
// compares against): Algorithm 2 with step (a) replaced by one eigenproblem in
// V_H + span{u_1, ..., u_N}, whose lowest N eigenpairs are the new orbitals
// (M-orthonormal by construction). Every fine-mesh integral comes from the
// fine stage: the per-orbital pieces of the eigenpairwise form, the full
// U^T O U blocks, and the pair integrals (u_j u_l, psi_m) that the Hartree
// term of the u-u block and the density need (the N^2 cross terms).
mlc_status inner_loop_joint(mlc_ctx* c, const FineBlocks& fb, InnerOut& out) {
  using namespace dense;
  const int64_t nH = c->nH;
  const int N = c->N;
  const int64_t m = nH + N;
  const int hart = c->hartree;
  const int npair = N * (N + 1) / 2;
  const TriIndex& ti = tri_index();
  auto t0 = std::chrono::steady_clock::now();

  std::vector<double> AfixH, G, MH, KH;
  assemble_dense(c, fb.cel_ops.data(), 40, 0, AfixH);
  assemble_dense(c, fb.cel_ops.data(), 40, 10, G);
  if (c->h_Mh_chol.empty()) {
    assemble_dense(c, fb.cel_ops.data(), 40, 20, MH);
    assemble_dense(c, fb.cel_ops.data(), 40, 30, KH);
    c->h_MH = MH;
    c->h_KH = KH;
    c->h_Mh_chol = MH;
    if (!cholesky(c->h_Mh_chol, nH)) return fail(c, MLC_ERR_NONFINITE, "coarse mass matrix not SPD");
    c->h_Kh_chol = KH;
    if (!cholesky(c->h_Kh_chol, nH)) return fail(c, MLC_ERR_NONFINITE, "coarse stiffness not SPD");
  }
  const std::vector<double>& MHd = c->h_MH;
  const std::vector<double>& KHd = c->h_KH;

  // coarse-dof vectors of the per-orbital and pair integrals: rhsv[k N + i] =
  // (u_i^2, psi_k), R[k npair + p] = (u_j u_l, psi_k)
  std::vector<double> R((size_t)nH * npair, 0.0);
  for (int64_t C = 0; C < c->cnt; ++C)
    for (int a = 0; a < 4; ++a) {
      const int k = c->cv2d[c->ctets[4 * C + a]];
      if (k < 0) continue;
      for (int p = 0; p < npair; ++p) R[(int64_t)k * npair + p] += fb.cel_pairs[((int64_t)C * npair + p) * 4 + a];
    }
  auto ah4_apply = [&](int i, const double* x, double* y) {  // y = A_h4,i x
    std::fill(y, y + nH, 0.0);
    for (int64_t C = 0; C < c->cnt; ++C) {
      int k[4];
      for (int a = 0; a < 4; ++a) k[a] = c->cv2d[c->ctets[4 * C + a]];
      const double* e = &fb.cel_orb[(C * N + i) * 14];
      for (int a = 0; a < 4; ++a) {
        if (k[a] < 0) continue;
        double sacc = 0.0;
        for (int b = 0; b < 4; ++b)
          if (k[b] >= 0) sacc += e[sym10(a, b)] * x[k[b]];
        y[k[a]] += sacc;
      }
    }
  };
  // Hartree system pieces, as in the eigenpairwise loop
  std::vector<double> yd(nH, 0.0);
  double schur = 1.0;
  if (hart) {
    for (int64_t k = 0; k < nH; ++k) yd[k] = fb.d[k];
    forward(c->h_Kh_chol, nH, yd.data());
    backward(c->h_Kh_chol, nH, yd.data());
    schur = fb.zeta - dot(fb.d.data(), yd.data(), nH);
    if (!(schur > 0.0)) return fail(c, MLC_ERR_NONFINITE, "Hartree augmented matrix not SPD");
  }
  // the mass and H^1 matrices of the joint basis [P, u_1..u_N] (fixed in the loop)
  std::vector<double> Mj(m * m, 0.0), KMj(m * m, 0.0);
  for (int64_t a = 0; a < nH; ++a)
    for (int64_t b = 0; b < nH; ++b) {
      Mj[a * m + b] = MHd[a * nH + b];
      KMj[a * m + b] = KHd[a * nH + b] + MHd[a * nH + b];
    }
  for (int64_t k = 0; k < nH; ++k)
    for (int j = 0; j < N; ++j) {
      Mj[k * m + nH + j] = Mj[(nH + j) * m + k] = fb.ptM[k * N + j];
      KMj[k * m + nH + j] = KMj[(nH + j) * m + k] = fb.ptK[k * N + j] + fb.ptM[k * N + j];
    }
  for (int j = 0; j < N; ++j)
    for (int l = 0; l < N; ++l) {
      Mj[(nH + j) * m + nH + l] = 0.5 * (fb.utM[j * N + l] + fb.utM[l * N + j]);
      KMj[(nH + j) * m + nH + l] =
          0.5 * (fb.utK[j * N + l] + fb.utK[l * N + j] + fb.utM[j * N + l] + fb.utM[l * N + j]);
    }
  std::vector<double> Lj = Mj;
  if (!cholesky(Lj, m)) return fail(c, MLC_ERR_NONFINITE, "mass matrix of the joint space not SPD");

  std::vector<double> wH(nH, 0.0), X((size_t)m * N, 0.0), Xold((size_t)m * N, 0.0), lam(N, 0.0);
  for (int i = 0; i < N; ++i) Xold[(size_t)i * m + nH + i] = 1.0;  // the first iterate: u_i
  double th1 = hart ? 1.0 : 0.0;
  std::vector<double> Kj, Cm, tmp(nH), fH(nH), xin(nH + 1), xout(nH + 1, 0.0), fres(nH + 1), gres(nH + 1);
  std::vector<std::vector<double>> Ah4w(N, std::vector<double>(nH));
  Tridiag Tr;
  Anderson mix;
  mix.m = c->opt.inner_mix_history;
  mix.beta = c->opt.inner_mix_beta;
  const int maxit = std::max(1, c->opt.inner_maxit);
  int its = 0;
  double diff = 0.0;
  mlc_status st = MLC_OK;
  for (int s = 0; s < maxit; ++s) {
    its = s + 1;
    // (a) the joint matrix: [[A_H, B], [B^T, E]] with the Hartree input (w_H, theta1)
    std::vector<double> AH = AfixH;
    if (hart) {
      add_trilinear_matrix(c, c->h_tri, wH.data(), 1.0, AH);
      for (int64_t k = 0; k < nH * nH; ++k) AH[k] += th1 * G[k];
    }
    Kj.assign(m * m, 0.0);
    for (int64_t a = 0; a < nH; ++a)
      for (int64_t b = 0; b < nH; ++b) Kj[a * m + b] = AH[a * nH + b];
    for (int j = 0; j < N; ++j) {
      if (hart) ah4_apply(j, wH.data(), Ah4w[j].data());
      for (int64_t k = 0; k < nH; ++k) {
        const double v = fb.ptF[k * N + j] + (hart ? Ah4w[j][k] + th1 * fb.ptW[k * N + j] : 0.0);
        Kj[k * m + nH + j] = Kj[(nH + j) * m + k] = v;
      }
    }
    for (int j = 0; j < N; ++j)
      for (int l = j; l < N; ++l) {
        double v = 0.5 * (fb.utF[j * N + l] + fb.utF[l * N + j]);
        if (hart) {
          v += th1 * 0.5 * (fb.utW[j * N + l] + fb.utW[l * N + j]);
          const int p = pair_index(N, j, l);
          for (int64_t k = 0; k < nH; ++k) v += wH[k] * R[(int64_t)k * npair + p];
        }
        Kj[(nH + j) * m + nH + l] = Kj[(nH + l) * m + nH + j] = v;
      }
    // the lowest N eigenpairs: C = L^-1 K L^-T = Q T Q^T, bisection, inverse
    // iteration (orthogonalised within clusters of equal eigenvalues)
    congruence(Lj, Kj, m, Cm);
    tridiagonalize(Cm, m, Tr);
    std::vector<double> ev = lowest_eigenvalues(Tr, nullptr, 0.0, N);
    double scale = 0.0;
    for (int64_t k = 0; k < m; ++k) scale = std::max(scale, std::fabs(Tr.d[k]) + (k + 1 < m ? std::fabs(Tr.e[k]) : 0));
    std::vector<double> Y((size_t)m * N), y(m);
    for (int i = 0; i < N; ++i) {
      std::vector<double> x0(m);
      for (int64_t k = 0; k < m; ++k) x0[k] = 1.0 + 1e-3 * std::sin(0.7 * (double)k + 1.3 * (double)i);
      double sv;
      eigenvector_from(Tr, nullptr, 0.0, ev[i], x0.data(), 0.0, y.data(), &sv);
      for (int pass = 0; pass < 2; ++pass)
        for (int k = 0; k < i; ++k) {
          if (std::fabs(ev[k] - ev[i]) > 1e-8 * std::max(1.0, scale)) continue;
          const double* yk = &Y[(size_t)k * m];
          double pr = dot(y.data(), yk, m);
          for (int64_t q = 0; q < m; ++q) y[q] -= pr * yk[q];
          double nr = std::sqrt(dot(y.data(), y.data(), m));
          for (int64_t q = 0; q < m; ++q) y[q] /= nr;
        }
      std::copy(y.begin(), y.end(), &Y[(size_t)i * m]);
    }
    bool finite = true;
    for (int i = 0; i < N; ++i) {
      double* xi = &X[(size_t)i * m];
      std::copy(&Y[(size_t)i * m], &Y[(size_t)i * m] + m, xi);
      apply_Q(Tr, xi);
      backward(Lj, m, xi);
      // sign of the previous iterate: (phi^{s+1}, phi^s)_M > 0
      const double* xo = &Xold[(size_t)i * m];
      double pr = 0.0;
      for (int64_t a = 0; a < m; ++a) pr += xi[a] * dot(&Mj[a * m], xo, m);
      if (pr < 0.0)
        for (int64_t a = 0; a < m; ++a) xi[a] = -xi[a];
      lam[i] = ev[i];
      finite = finite && std::isfinite(lam[i]);
    }
    if (!finite) return fail(c, MLC_ERR_NONFINITE, "non-finite solution of the joint problem");
    // (b) Hartree problem for phi_i = P c_i + sum_j d_ji u_j
    if (hart) {
      std::fill(fH.begin(), fH.end(), 0.0);
      double gsum = 0.0;
      std::vector<double> ph(nH);
      for (int i = 0; i < N; ++i) {
        const double f = c->occ[i];
        if (f == 0.0) continue;
        const double* xi = &X[(size_t)i * m];
        const double* di = xi + nH;
        for (int64_t k = 0; k < nH; ++k) ph[k] = xi[k];
        for (int64_t C = 0; C < c->cnt; ++C) {  // ((P c_i)^2, psi_k) through the trilinear tensor
          int k[4];
          double pl[4];
          for (int q = 0; q < 4; ++q) {
            k[q] = c->cv2d[c->ctets[4 * C + q]];
            pl[q] = k[q] >= 0 ? ph[k[q]] : 0.0;
          }
          const double* T = &c->h_tri[20 * C];
          for (int jj = 0; jj < 4; ++jj) {
            if (k[jj] < 0) continue;
            double sacc = 0.0;
            for (int mm = 0; mm < 4; ++mm)
              for (int ll = 0; ll < 4; ++ll) sacc += T[ti.idx[jj][mm][ll]] * pl[mm] * pl[ll];
            fH[k[jj]] += f * sacc;
          }
        }
        symv(G, nH, ph.data(), tmp.data());
        double g1 = dot(ph.data(), tmp.data(), nH), g2 = 0.0, g3 = 0.0;
        for (int j = 0; j < N; ++j) {
          if (di[j] == 0.0) continue;
          ah4_apply(j, ph.data(), tmp.data());  // (u_j P c_i, psi_k)
          for (int64_t k = 0; k < nH; ++k) fH[k] += f * 2.0 * di[j] * tmp[k];
          double pw = 0.0;
          for (int64_t k = 0; k < nH; ++k) pw += fb.ptW[k * N + j] * ph[k];
          g2 += di[j] * pw;
          for (int l = 0; l < N; ++l) {
            const double dd = di[j] * di[l];
            const int p = pair_index(N, j, l);
            for (int64_t k = 0; k < nH; ++k) fH[k] += f * dd * R[(int64_t)k * npair + p];
            g3 += dd * 0.5 * (fb.utW[j * N + l] + fb.utW[l * N + j]);
          }
        }
        gsum += f * (g1 + 2.0 * g2 + g3);
      }
      const double fourpi = 4.0 * 3.14159265358979323846;
      std::vector<double> r1(nH);
      for (int64_t k = 0; k < nH; ++k) r1[k] = fourpi * fH[k] - fb.liftH[k];
      const double r2 = fourpi * gsum - fb.liftT;
      forward(c->h_Kh_chol, nH, r1.data());
      backward(c->h_Kh_chol, nH, r1.data());
      const double t1 = (r2 - dot(fb.d.data(), r1.data(), nH)) / schur;
      for (int64_t k = 0; k < nH; ++k) xout[k] = r1[k] - yd[k] * t1;
      xout[nH] = t1;
    }
    // (c) ||Phi^{s+1} - Phi^s||_{H^1} in the joint basis
    double d2 = 0.0;
    std::vector<double> dx(m);
    for (int i = 0; i < N; ++i) {
      for (int64_t a = 0; a < m; ++a) dx[a] = X[(size_t)i * m + a] - Xold[(size_t)i * m + a];
      for (int64_t a = 0; a < m; ++a) d2 += dx[a] * dot(&KMj[a * m], dx.data(), m);
    }
    diff = std::sqrt(std::max(d2, 0.0));
    Xold = X;
    if (!hart) break;
    const bool done = diff < c->opt.inner_tol;
    if (!done && s == maxit - 1) st = MLC_WARN_INNER_MAXIT;
    if (done || s == maxit - 1 || c->opt.inner_mix_history <= 0) {
      std::copy(xout.begin(), xout.begin() + nH, wH.begin());
      th1 = xout[nH];
      if (done || s == maxit - 1) break;
      continue;
    }
    std::copy(wH.begin(), wH.end(), xin.begin());
    xin[nH] = th1;
    for (int64_t k = 0; k <= nH; ++k) fres[k] = xout[k] - xin[k];
    symv(KHd, nH, fres.data(), gres.data());
    for (int64_t k = 0; k < nH; ++k) gres[k] += fb.d[k] * fres[nH];
    gres[nH] = dot(fb.d.data(), fres.data(), nH) + fb.zeta * fres[nH];
    mix.next(xin, fres, gres);
    std::copy(xin.begin(), xin.begin() + nH, wH.begin());
    th1 = xin[nH];
  }
  out.lam = lam;
  out.phiH.assign((size_t)nH * N, 0.0);
  out.D.assign((size_t)N * N, 0.0);
  out.theta2.assign(N, 0.0);
  for (int i = 0; i < N; ++i) {
    const double* xi = &Xold[(size_t)i * m];
    for (int64_t k = 0; k < nH; ++k) out.phiH[k * N + i] = xi[k];
    for (int j = 0; j < N; ++j) out.D[(size_t)j * N + i] = xi[nH + j];
    out.theta2[i] = xi[nH + i];
  }
  out.wH = wH;
  out.theta1 = th1;
  out.iters = its;
  out.last_diff = diff;
  out.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return st;
}

}  // namespace mlc
