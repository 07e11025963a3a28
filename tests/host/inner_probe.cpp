// Test driver for the host inner loop (Algorithm 2 as in Algorithm 3 step 2)
// on synthetic coarse-space data: a structured Kuhn coarse mesh with P1
// element matrices, small random fine-stage blocks. Writes the loop's
// outputs (status, eigenvalues, coarse coefficients, theta2, w_H, theta1, the
// last difference and the iteration count) to a binary file.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include "inner.h"
namespace mlc {
mlc_status fail(mlc_ctx* c, mlc_status s, const std::string& msg) { if (c) c->err = msg; return s; }
}
using namespace mlc;
static int sym10(int j, int k) { if (j > k) std::swap(j, k); static const int base[4] = {0, 4, 7, 9}; return base[j] + (k - j); }
int main(int argc, char** argv) {
  const int n = argc > 1 ? atoi(argv[1]) : 8;       // cubes per side
  const int N = argc > 2 ? atoi(argv[2]) : 13;      // orbitals
  const char* out_path = argc > 3 ? argv[3] : "inner.bin";
  mlc_ctx c;
  c.N = N;
  c.hartree = argc > 4 ? atoi(argv[4]) : 1;                 // 0: no Hartree term
  const bool zero_occ = argc > 5 && atoi(argv[5]) != 0;    // every third orbital unoccupied
  const int nv1 = n + 1;
  auto vid = [&](int i, int j, int k) { return (i * nv1 + j) * nv1 + k; };
  std::vector<double> X(3 * nv1 * nv1 * nv1);
  for (int i = 0; i <= n; ++i) for (int j = 0; j <= n; ++j) for (int k = 0; k <= n; ++k) {
    int v = vid(i, j, k); X[3 * v] = i; X[3 * v + 1] = j; X[3 * v + 2] = k; }
  c.cv2d.assign(nv1 * nv1 * nv1, -1);
  int64_t nH = 0;
  for (int i = 1; i < n; ++i) for (int j = 1; j < n; ++j) for (int k = 1; k < n; ++k) c.cv2d[vid(i, j, k)] = (int32_t)nH++;
  c.nH = nH;
  // Kuhn: 6 tets per cube along the paths of the permutations of the axes
  const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  for (int i = 0; i < n; ++i) for (int j = 0; j < n; ++j) for (int k = 0; k < n; ++k)
    for (int p = 0; p < 6; ++p) {
      int q[3] = {i, j, k};
      c.ctets.push_back(vid(q[0], q[1], q[2]));
      for (int s = 0; s < 3; ++s) { q[perm[p][s]]++; c.ctets.push_back(vid(q[0], q[1], q[2])); }
    }
  c.cnt = (int64_t)c.ctets.size() / 4;
  std::mt19937_64 rng(17);
  std::uniform_real_distribution<double> U(-1.0, 1.0);
  FineBlocks fb;
  fb.cel_ops.assign(c.cnt * 40, 0.0);
  fb.cel_orb.assign(c.cnt * N * 14, 0.0);
  c.h_tri.assign(c.cnt * 20, 0.0);
  for (int64_t t = 0; t < c.cnt; ++t) {
    const int* v = &c.ctets[4 * t];
    double P[4][3];
    for (int a = 0; a < 4; ++a) for (int d = 0; d < 3; ++d) P[a][d] = X[3 * v[a] + d];
    double J[3][3];
    for (int r = 0; r < 3; ++r) for (int d = 0; d < 3; ++d) J[d][r] = P[r + 1][d] - P[0][d];
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    double vol = std::fabs(det) / 6.0;
    // barycentric gradients: rows of J^{-1}
    double inv[3][3];
    inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det; inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det; inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det; inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det; inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    double g[4][3];
    for (int d = 0; d < 3; ++d) { g[1][d] = inv[0][d]; g[2][d] = inv[1][d]; g[3][d] = inv[2][d]; g[0][d] = -(g[1][d] + g[2][d] + g[3][d]); }
    for (int a = 0; a < 4; ++a) for (int b = a; b < 4; ++b) {
      double K = vol * (g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2]);
      double M = vol / 20.0 * (a == b ? 2.0 : 1.0);
      double* e = &fb.cel_ops[t * 40];
      e[sym10(a, b)] = 0.5 * K - 0.4 * M;       // A_fix
      e[10 + sym10(a, b)] = 0.3 * M;            // M_{w0}
      e[20 + sym10(a, b)] = M;                  // M
      e[30 + sym10(a, b)] = K;                  // K
      for (int i = 0; i < N; ++i) fb.cel_orb[(t * N + i) * 14 + sym10(a, b)] = 0.02 * M * (1.0 + 0.05 * i);
    }
    for (int i = 0; i < N; ++i) for (int a = 0; a < 4; ++a) fb.cel_orb[(t * N + i) * 14 + 10 + a] = vol / 4.0 * 0.01 * (1.0 + 0.1 * i);
    for (int s = 0; s < 20; ++s) c.h_tri[t * 20 + s] = vol * (0.01 + 0.005 * s / 20.0);
  }
  fb.ptF.resize(nH * N); fb.ptW.resize(nH * N); fb.ptM.resize(nH * N); fb.ptK.resize(nH * N);
  for (int64_t k = 0; k < nH * N; ++k) { fb.ptF[k] = 0.01 * U(rng); fb.ptW[k] = 0.005 * U(rng); fb.ptM[k] = 0.002 * U(rng); fb.ptK[k] = 0.01 * U(rng); }
  fb.utF.assign(N * N, 0.0); fb.utW.assign(N * N, 0.0); fb.utM.assign(N * N, 0.0); fb.utK.assign(N * N, 0.0);
  for (int i = 0; i < N; ++i) { fb.utF[i * N + i] = -0.3 + 0.02 * i; fb.utW[i * N + i] = 0.1; fb.utM[i * N + i] = 1.0; fb.utK[i * N + i] = 2.0; }
  fb.d.resize(nH); fb.liftH.resize(nH);
  for (int64_t k = 0; k < nH; ++k) { fb.d[k] = 1e-3 * U(rng); fb.liftH[k] = 1e-3 * U(rng); }
  fb.zeta = 1.0; fb.liftT = 1e-3;
  c.occ.assign(N, 2.0);
  if (zero_occ)
    for (int i = 0; i < N; ++i)
      if (i % 3 == 1) c.occ[i] = 0.0;
  c.opt.n_extra = 8; c.opt.inner_maxit = 6; c.opt.inner_mix_history = 6; c.opt.inner_mix_beta = 0.5; c.opt.inner_tol = 1e-12;
  InnerOut out;
  mlc_status st = inner_loop(&c, fb, out);
  std::FILE* f = std::fopen(out_path, "wb");
  std::fwrite(&st, sizeof st, 1, f);
  std::fwrite(out.lam.data(), 8, out.lam.size(), f);
  std::fwrite(out.phiH.data(), 8, out.phiH.size(), f);
  std::fwrite(out.theta2.data(), 8, out.theta2.size(), f);
  std::fwrite(out.wH.data(), 8, out.wH.size(), f);
  std::fwrite(&out.theta1, 8, 1, f);
  std::fwrite(&out.last_diff, 8, 1, f);
  std::fwrite(&out.iters, sizeof out.iters, 1, f);
  std::fclose(f);
  printf("nH=%lld N=%d status %d iters %d last_diff %.3e theta1 %.6f lam0 %.8f lam_last %.8f ms %.1f %s\n", (long long)nH, N,
         (int)st, out.iters, out.last_diff, out.theta1, out.lam.empty() ? 0.0 : out.lam[0], out.lam.empty() ? 0.0 : out.lam[N - 1], out.ms, c.err.c_str());
}
