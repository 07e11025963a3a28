// Device helpers shared by the P1 kernels (kernels.hip) and the P2 kernels
// (p2.hip): pointwise exchange-correlation and external potential, coarse
// barycentric coordinates and the ordered block sums.
#pragma once

#include <hip/hip_runtime.h>

namespace mlc {
namespace {

// Exchange-correlation: LDA = Slater exchange + Perdew-Zunger 1981 correlation
// with the constants printed in Section 4; V_xc = eps + rho d eps/d rho in the
// closed forms eps_x * 4/3 and, for correlation,
//   r_s >= 1: v_c = eps_c (1 + 7/6 b1 sqrt(rs) + 4/3 b2 rs) / (1 + b1 sqrt(rs) + b2 rs)
//   r_s <  1: v_c = A ln rs + (B - A/3) + (2/3) C rs ln rs + (2D - C)/3 rs.
// X-alpha: v = -3/2 alpha (3 rho / pi)^(1/3), eps = 3/4 v.
__device__ __forceinline__ void xc_point(int kind, double xalpha, double rho, double* eps, double* v) {
  if (kind == 0 || !(rho > 1e-30)) {
    *eps = 0.0;
    *v = 0.0;
    return;
  }
  const double pi = 3.14159265358979323846;
  double c13 = cbrt(rho);
  if (kind == 2) {
    double vv = -1.5 * xalpha * cbrt(3.0 / pi) * c13;
    *v = vv;
    *eps = 0.75 * vv;
    return;
  }
  double ex = -0.75 * cbrt(3.0 / pi) * c13;
  double vx = ex * (4.0 / 3.0);
  double rs = cbrt(3.0 / (4.0 * pi * rho));
  double ec, vc;
  if (rs >= 1.0) {
    const double g = -0.1423, b1 = 1.0529, b2 = 0.3334;
    double sq = sqrt(rs);
    double den = 1.0 + b1 * sq + b2 * rs;
    ec = g / den;
    vc = ec * (1.0 + (7.0 / 6.0) * b1 * sq + (4.0 / 3.0) * b2 * rs) / den;
  } else {
    const double A = 0.0311, B = -0.048, C = 0.0020, D = -0.0116;
    double lr = log(rs);
    ec = A * lr + B + C * rs * lr + D * rs;
    vc = A * lr + (B - A / 3.0) + (2.0 / 3.0) * C * rs * lr + ((2.0 * D - C) / 3.0) * rs;
  }
  *eps = ex + ec;
  *v = vx + vc;
}

// ---------------------------------------------------------------------------
// V_ext at a point: -sum Z erf(r/rc)/r (its r -> 0 limit -2Z/(sqrt(pi) rc)),
// the bare -sum Z/r, or the harmonic 1/2 omega^2 |x|^2.
__device__ __forceinline__ double vext_point(double x, double y, double z, int n_nuclei, const double* __restrict__ RZ,
                                             int kind, double rc, double omega) {
  if (kind == 2) return 0.5 * omega * omega * (x * x + y * y + z * z);
  double v = 0.0;
  for (int k = 0; k < n_nuclei; ++k) {
    double dx = x - RZ[4 * k], dy = y - RZ[4 * k + 1], dz = z - RZ[4 * k + 2], Zk = RZ[4 * k + 3];
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    if (kind == 1) {
      v -= Zk / r;
    } else {
      if (r < 1e-12)
        v -= Zk * 1.12837916709551257390 / rc;
      else
        v -= Zk * erf(r / rc) / r;
    }
  }
  return v;
}

__device__ __forceinline__ void coarse_bary(const double* __restrict__ cg, const double* __restrict__ xyz, int v,
                                            double b[4]) {
  double dx = xyz[3 * v] - cg[0], dy = xyz[3 * v + 1] - cg[1], dz = xyz[3 * v + 2] - cg[2];
  b[1] = cg[3] * dx + cg[4] * dy + cg[5] * dz;
  b[2] = cg[6] * dx + cg[7] * dy + cg[8] * dz;
  b[3] = cg[9] * dx + cg[10] * dy + cg[11] * dz;
  b[0] = 1.0 - b[1] - b[2] - b[3];
}

// Block-wide ordered sum of v over the 256 threads; result returned to all.
// Block sums of K values per thread (TPB = 256, four waves): every value's
// wave sum, then one barrier; thread k < K returns the block sum of value k
// (the four wave sums added as (w0 + w1) + (w2 + w3)), the others 0.
// ws: 4 K doubles.
template <int K>
__device__ __forceinline__ double block_sums(const double (&v)[K], double* ws) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double x = v[k];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if (lane == 0) ws[wid * K + k] = x;
  }
  __syncthreads();
  const int t = threadIdx.x;
  const double r = t < K ? (ws[t] + ws[K + t]) + (ws[2 * K + t] + ws[3 * K + t]) : 0.0;
  __syncthreads();  // ws may be reused at once
  return r;
}

}  // namespace
}  // namespace mlc
