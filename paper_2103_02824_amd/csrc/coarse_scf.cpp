// Algorithm 1 step 1: the discrete Kohn-Sham problem on the coarse mesh,
// solved self-consistently (host FP64), and step 4: its transfer to the fine
// mesh (Phi = P Phi_H exactly, the spaces being nested; w interpolated; the
// eigenvalues carried over).
//
// One SCF step: rho at the coarse quadrature points -> V_xc, multipole
// Dirichlet data, coarse Poisson solve -> H = 1/2 K + M_{V_ext + w + V_xc}
// -> lowest N eigenpairs of (H, M) -> output density. The input density is
// updated by Anderson mixing (history 6, damping 0.5, L^2 inner product at the
// quadrature points); the fixed point does not depend on the mixing.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "dense.h"
#include "mlc_internal.h"

namespace mlc {

namespace {

const double kPi = 3.14159265358979323846;

void xc_host(int kind, double xalpha, double rho, double* eps, double* v) {
  if (kind == 0 || !(rho > 1e-30)) {
    *eps = 0.0;
    *v = 0.0;
    return;
  }
  double c13 = std::cbrt(rho);
  if (kind == 2) {
    double vv = -1.5 * xalpha * std::cbrt(3.0 / kPi) * c13;
    *v = vv;
    *eps = 0.75 * vv;
    return;
  }
  double ex = -0.75 * std::cbrt(3.0 / kPi) * c13;
  double rs = std::cbrt(3.0 / (4.0 * kPi * rho));
  double ec, vc;
  if (rs >= 1.0) {
    const double g = -0.1423, b1 = 1.0529, b2 = 0.3334;
    double sq = std::sqrt(rs), den = 1.0 + b1 * sq + b2 * rs;
    ec = g / den;
    vc = ec * (1.0 + (7.0 / 6.0) * b1 * sq + (4.0 / 3.0) * b2 * rs) / den;
  } else {
    const double A = 0.0311, B = -0.048, C = 0.0020, D = -0.0116;
    double lr = std::log(rs);
    ec = A * lr + B + C * rs * lr + D * rs;
    vc = A * lr + (B - A / 3.0) + (2.0 / 3.0) * C * rs * lr + ((2.0 * D - C) / 3.0) * rs;
  }
  *eps = ex + ec;
  *v = ex * (4.0 / 3.0) + vc;
}

double vext_host(const mlc_ctx* c, const double* x) {
  if (c->potential == MLC_POT_HARMONIC) return 0.5 * c->omega * c->omega * (x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
  double v = 0.0;
  for (int k = 0; k < c->n_nuclei; ++k) {
    double dx = x[0] - c->R[3 * k], dy = x[1] - c->R[3 * k + 1], dz = x[2] - c->R[3 * k + 2];
    double r = std::sqrt(dx * dx + dy * dy + dz * dz);
    if (c->potential == MLC_POT_BARE)
      v -= c->Z[k] / r;
    else
      v -= r < 1e-12 ? c->Z[k] * 2.0 / (std::sqrt(kPi) * c->rc) : c->Z[k] * std::erf(r / c->rc) / r;
  }
  return v;
}

inline double Lq(int q, int j) { return q == j ? QA : QB; }

struct Coarse {
  int64_t nt, nv, nH;
  std::vector<double> vol, grad, qp, qw;  // grad: nt x 4 x 3
  std::vector<int32_t> tets, v2d;
  std::vector<int32_t> bverts;
};

}  // namespace

mlc_status coarse_scf(mlc_ctx* c, double tol, int maxit, int* iters_out) {
  using namespace dense;
  Coarse m;
  m.nt = c->cnt;
  m.nv = c->cnv;
  m.nH = c->nH;
  m.tets = c->ctets;
  m.v2d = c->cv2d;
  for (int64_t v = 0; v < m.nv; ++v)
    if (m.v2d[v] < 0) m.bverts.push_back((int32_t)v);
  m.vol = c->cvol;
  m.grad.assign(12 * m.nt, 0.0);
  m.qp.assign(12 * m.nt, 0.0);
  m.qw.assign(4 * m.nt, 0.0);
  for (int64_t t = 0; t < m.nt; ++t) {
    const double* Ji = &c->cgeo[12 * t + 3];
    for (int k = 0; k < 3; ++k) {
      m.grad[12 * t + 3 + k] = Ji[k];
      m.grad[12 * t + 6 + k] = Ji[3 + k];
      m.grad[12 * t + 9 + k] = Ji[6 + k];
      m.grad[12 * t + k] = -(Ji[k] + Ji[3 + k] + Ji[6 + k]);
    }
    for (int q = 0; q < 4; ++q) {
      m.qw[4 * t + q] = 0.25 * m.vol[t];
      for (int k = 0; k < 3; ++k) {
        double s = 0.0;
        for (int j = 0; j < 4; ++j) s += Lq(q, j) * c->cxyz[3 * (int64_t)m.tets[4 * t + j] + k];
        m.qp[12 * t + 3 * q + k] = s;
      }
    }
  }
  const int64_t nH = m.nH, nq = 4 * m.nt;
  const int N = c->N;
  // fixed matrices: K, M (interior dense), V_ext at qp
  std::vector<double> K(nH * nH, 0.0), M(nH * nH, 0.0), vext(nq);
  for (int64_t t = 0; t < m.nt; ++t) {
    for (int q = 0; q < 4; ++q) vext[4 * t + q] = vext_host(c, &m.qp[12 * t + 3 * q]);
    for (int a = 0; a < 4; ++a) {
      int ia = m.v2d[m.tets[4 * t + a]];
      if (ia < 0) continue;
      for (int b = 0; b < 4; ++b) {
        int ib = m.v2d[m.tets[4 * t + b]];
        if (ib < 0) continue;
        const double* ga = &m.grad[12 * t + 3 * a];
        const double* gb = &m.grad[12 * t + 3 * b];
        K[(int64_t)ia * nH + ib] += m.vol[t] * (ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2]);
        double mm = 0.0;
        for (int q = 0; q < 4; ++q) mm += 0.25 * m.vol[t] * Lq(q, a) * Lq(q, b);
        M[(int64_t)ia * nH + ib] += mm;
      }
    }
  }
  std::vector<double> LM = M, LK = K;
  if (!cholesky(LM, nH) || !cholesky(LK, nH)) return fail(c, MLC_ERR_NONFINITE, "coarse matrices not SPD");

  auto hartree = [&](const std::vector<double>& rho, std::vector<double>& wnod) {
    wnod.assign(m.nv, 0.0);
    if (!c->hartree) return;
    double mom[10] = {0};
    for (int64_t i = 0; i < nq; ++i) {
      double w = m.qw[i] * rho[i];
      const double* x = &m.qp[3 * i];
      mom[0] += w;
      mom[1] += w * x[0];
      mom[2] += w * x[1];
      mom[3] += w * x[2];
      mom[4] += w * x[0] * x[0];
      mom[5] += w * x[1] * x[1];
      mom[6] += w * x[2] * x[2];
      mom[7] += w * x[0] * x[1];
      mom[8] += w * x[0] * x[2];
      mom[9] += w * x[1] * x[2];
    }
    double Q = mom[0];
    if (!(Q > 0)) return;
    double cc[3] = {mom[1] / Q, mom[2] / Q, mom[3] / Q};
    double p[3] = {mom[1] - Q * cc[0], mom[2] - Q * cc[1], mom[3] - Q * cc[2]};
    double S[3][3] = {{mom[4], mom[7], mom[8]}, {mom[7], mom[5], mom[9]}, {mom[8], mom[9], mom[6]}};
    double Sc[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) Sc[a][b] = S[a][b] - cc[a] * mom[1 + b] - cc[b] * mom[1 + a] + Q * cc[a] * cc[b];
    double tr = Sc[0][0] + Sc[1][1] + Sc[2][2];
    for (int32_t v : m.bverts) {
      double r[3] = {c->cxyz[3 * (int64_t)v] - cc[0], c->cxyz[3 * (int64_t)v + 1] - cc[1], c->cxyz[3 * (int64_t)v + 2] - cc[2]};
      double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2], rn = std::sqrt(r2);
      double quad = 0.0;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) quad += r[a] * (3.0 * Sc[a][b] - (a == b ? tr : 0.0)) * r[b];
      wnod[v] = Q / rn + (p[0] * r[0] + p[1] * r[1] + p[2] * r[2]) / (r2 * rn) + 0.5 * quad / (r2 * r2 * rn);
    }
    std::vector<double> b(nH, 0.0);
    for (int64_t t = 0; t < m.nt; ++t)
      for (int a = 0; a < 4; ++a) {
        int ia = m.v2d[m.tets[4 * t + a]];
        if (ia < 0) continue;
        for (int q = 0; q < 4; ++q) b[ia] += 4.0 * kPi * m.qw[4 * t + q] * rho[4 * t + q] * Lq(q, a);
        for (int bb = 0; bb < 4; ++bb) {
          int v = m.tets[4 * t + bb];
          if (m.v2d[v] >= 0) continue;
          const double* ga = &m.grad[12 * t + 3 * a];
          const double* gb = &m.grad[12 * t + 3 * bb];
          b[ia] -= m.vol[t] * (ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2]) * wnod[v];
        }
      }
    forward(LK, nH, b.data());
    backward(LK, nH, b.data());
    for (int64_t v = 0; v < m.nv; ++v)
      if (m.v2d[v] >= 0) wnod[v] = b[m.v2d[v]];
  };

  std::vector<double> rho_in(nq, 0.0), rho_out(nq, 0.0), wnod, lam(N), Phi(nH * N);
  std::vector<std::vector<double>> Xh, Fh;
  bool nonlinear = c->hartree || c->xc != MLC_XC_NONE;
  int it = 0;
  double res = 0.0;
  std::vector<double> H, C;
  Tridiag Tr;
  for (it = 0; it < std::max(1, maxit); ++it) {
    hartree(rho_in, wnod);
    H.assign(nH * nH, 0.0);
    for (int64_t t = 0; t < m.nt; ++t) {
      double f[4];
      double wl[4];
      for (int j = 0; j < 4; ++j) wl[j] = wnod[m.tets[4 * t + j]];
      for (int q = 0; q < 4; ++q) {
        double e, vx;
        xc_host(c->xc, c->xalpha, rho_in[4 * t + q], &e, &vx);
        double wq = 0.0;
        for (int j = 0; j < 4; ++j) wq += Lq(q, j) * wl[j];
        f[q] = vext[4 * t + q] + wq + vx;
      }
      for (int a = 0; a < 4; ++a) {
        int ia = m.v2d[m.tets[4 * t + a]];
        if (ia < 0) continue;
        for (int b = 0; b < 4; ++b) {
          int ib = m.v2d[m.tets[4 * t + b]];
          if (ib < 0) continue;
          const double* ga = &m.grad[12 * t + 3 * a];
          const double* gb = &m.grad[12 * t + 3 * b];
          double v = 0.5 * m.vol[t] * (ga[0] * gb[0] + ga[1] * gb[1] + ga[2] * gb[2]);
          for (int q = 0; q < 4; ++q) v += 0.25 * m.vol[t] * f[q] * Lq(q, a) * Lq(q, b);
          H[(int64_t)ia * nH + ib] += v;
        }
      }
    }
    congruence(LM, H, nH, C);
    tridiagonalize(C, nH, Tr);
    std::vector<double> ev = lowest_eigenvalues(Tr, nullptr, 0.0, N);
    double scale = 0.0;
    for (double d : Tr.d) scale = std::max(scale, std::fabs(d));
    std::vector<std::vector<double>> Ys;
    for (int j = 0; j < N; ++j) {
      std::vector<double> y(nH);
      eigenvector(Tr, nullptr, 0.0, ev[j], y.data(), nullptr);
      // orthogonalise within clusters of (nearly) equal eigenvalues
      for (int pass = 0; pass < 2; ++pass) {
        for (int k = 0; k < j; ++k) {
          if (std::fabs(ev[k] - ev[j]) > 1e-8 * std::max(1.0, scale)) continue;
          double s = 0.0;
          for (int64_t r = 0; r < nH; ++r) s += Ys[k][r] * y[r];
          for (int64_t r = 0; r < nH; ++r) y[r] -= s * Ys[k][r];
        }
        double nr = 0.0;
        for (double v : y) nr += v * v;
        nr = std::sqrt(nr);
        for (double& v : y) v /= nr;
      }
      Ys.push_back(y);
      apply_Q(Tr, y.data());
      backward(LM, nH, y.data());
      for (int64_t r = 0; r < nH; ++r) Phi[r * N + j] = y[r];
      lam[j] = ev[j];
    }
    // output density at qp
    std::fill(rho_out.begin(), rho_out.end(), 0.0);
    for (int64_t t = 0; t < m.nt; ++t) {
      int k[4];
      for (int j = 0; j < 4; ++j) k[j] = m.v2d[m.tets[4 * t + j]];
      for (int i = 0; i < N; ++i) {
        double u[4];
        for (int j = 0; j < 4; ++j) u[j] = k[j] >= 0 ? Phi[(int64_t)k[j] * N + i] : 0.0;
        for (int q = 0; q < 4; ++q) {
          double uq = 0.0;
          for (int j = 0; j < 4; ++j) uq += Lq(q, j) * u[j];
          rho_out[4 * t + q] += c->occ[i] * uq * uq;
        }
      }
    }
    res = 0.0;
    for (int64_t i = 0; i < nq; ++i) res += m.qw[i] * std::fabs(rho_out[i] - rho_in[i]);
    if (!nonlinear || res < tol) break;
    // Anderson mixing of the input density
    std::vector<double> F(nq);
    for (int64_t i = 0; i < nq; ++i) F[i] = rho_out[i] - rho_in[i];
    Xh.push_back(rho_in);
    Fh.push_back(F);
    if (Xh.size() > 7) {
      Xh.erase(Xh.begin());
      Fh.erase(Fh.begin());
    }
    int mh = (int)Xh.size() - 1;
    std::vector<double> next(nq);
    if (mh == 0) {
      for (int64_t i = 0; i < nq; ++i) next[i] = rho_in[i] + 0.5 * F[i];
    } else {
      // least squares min |F - sum g_k dF_k| by normal equations (small)
      std::vector<double> A(mh * mh), r(mh);
      std::vector<std::vector<double>> dF(mh, std::vector<double>(nq)), dX(mh, std::vector<double>(nq));
      for (int k = 0; k < mh; ++k)
        for (int64_t i = 0; i < nq; ++i) {
          dF[k][i] = Fh[k + 1][i] - Fh[k][i];
          dX[k][i] = Xh[k + 1][i] - Xh[k][i];
        }
      for (int a = 0; a < mh; ++a) {
        r[a] = 0.0;
        for (int64_t i = 0; i < nq; ++i) r[a] += m.qw[i] * dF[a][i] * F[i];
        for (int b = 0; b < mh; ++b) {
          double s = 0.0;
          for (int64_t i = 0; i < nq; ++i) s += m.qw[i] * dF[a][i] * dF[b][i];
          A[a * mh + b] = s;
        }
      }
      // regularised Cholesky solve
      double tr = 0.0;
      for (int a = 0; a < mh; ++a) tr += A[a * mh + a];
      for (int a = 0; a < mh; ++a) A[a * mh + a] += 1e-12 * tr / mh;
      std::vector<double> LA = A;
      std::vector<double> gmm = r;
      if (cholesky(LA, mh)) {
        forward(LA, mh, gmm.data());
        backward(LA, mh, gmm.data());
      } else {
        std::fill(gmm.begin(), gmm.end(), 0.0);
      }
      for (int64_t i = 0; i < nq; ++i) {
        double xb = rho_in[i], fb = F[i];
        for (int k = 0; k < mh; ++k) {
          xb -= gmm[k] * dX[k][i];
          fb -= gmm[k] * dF[k][i];
        }
        next[i] = xb + 0.5 * fb;
      }
    }
    for (int64_t i = 0; i < nq; ++i) rho_in[i] = std::max(0.0, next[i]);
  }
  if (iters_out) *iters_out = it + 1;
  // Hartree potential of the final output density
  hartree(rho_out, wnod);
  // step 4: transfer to the fine mesh
  std::vector<double> phi_f(c->n * N, 0.0), w_f(c->nv, 0.0);
  for (int64_t a = 0; a < c->n; ++a)
    for (int s = 0; s < 4; ++s) {
      int k = c->Pk[4 * a + s];
      if (k < 0) continue;
      for (int i = 0; i < N; ++i) phi_f[a * N + i] += c->Pw[4 * a + s] * Phi[(int64_t)k * N + i];
    }
  for (int64_t v = 0; v < c->nv; ++v)
    for (int s = 0; s < 4; ++s) {
      int cv = c->Pfull_k[4 * v + s];
      if (cv >= 0) w_f[v] += c->Pfull_w[4 * v + s] * wnod[cv];
    }
  hipError_t e = hipMemcpyAsync(c->d.Phi, phi_f.data(), sizeof(double) * phi_f.size(), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->d.w, w_f.data(), sizeof(double) * w_f.size(), hipMemcpyHostToDevice, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(c, e, "initial state upload");
  c->lam = lam;
  c->has_state = true;
  c->has_step = false;
  return MLC_OK;
}

}  // namespace mlc
