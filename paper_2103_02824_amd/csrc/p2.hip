// gfx950 element kernels of the P2 (quadratic) fine space: the same
// quantities as the P1 kernels of kernels.hip (fields at quadrature points,
// element matrices in slot order, load vectors, coarse-pattern integrals,
// energy pieces), on 10-node tets with the 27-point rule of p2.h. The rule's
// points, weights, basis values and element-matrix pieces come from one
// table in device memory (read with wave-uniform addresses). One thread per
// fine tet, except the coarse-pattern kernels (one workgroup per coarse
// tet). Every reduction is ordered; no atomics.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mlc_internal.h"
#include "p2.h"
#include "pointwise.h"

namespace mlc {

namespace {

constexpr int TPB = 256;
constexpr int NE = P2_NE, NQ = P2_NQ;

inline unsigned nb(int64_t work) { return (unsigned)((work + TPB - 1) / TPB); }

__device__ __forceinline__ int pair_index(int a, int b) {  // a <= b
  return a * NE - (a * (a - 1)) / 2 + (b - a);
}

// The 10 products grad lambda_c . grad lambda_d (c <= d) of a tet.
__device__ __forceinline__ void grad_products(const double* __restrict__ G, double gg[10]) {
  int k = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int d = c; d < 4; ++d, ++k)
      gg[k] = G[1 + 3 * c] * G[1 + 3 * d] + G[2 + 3 * c] * G[2 + 3 * d] + G[3 + 3 * c] * G[3 + 3 * d];
}

// K_ab / |T| of the tet from its gradient products.
__device__ __forceinline__ double stiff_entry(const double* __restrict__ tab, int p, const double gg[10]) {
  const double* sk = tab + P2_T_SK + 10 * p;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 10; ++k) s += sk[k] * gg[k];
  return s;
}

// rho at the 27 points of tet t: sum_i f_i (sum_a phi_a(q) u_ia)^2.
__device__ __forceinline__ void tet_density_p2(const int32_t* __restrict__ el, const int32_t* __restrict__ v2d,
                                               const double* __restrict__ X, int N, const double* __restrict__ occ,
                                               const double* __restrict__ tab, int64_t t, double rho[NQ]) {
  int dof[NE];
#pragma unroll
  for (int a = 0; a < NE; ++a) dof[a] = v2d[el[NE * t + a]];
#pragma unroll
  for (int q = 0; q < NQ; ++q) rho[q] = 0.0;
  for (int i = 0; i < N; ++i) {
    double u[NE];
#pragma unroll
    for (int a = 0; a < NE; ++a) u[a] = dof[a] >= 0 ? X[(int64_t)dof[a] * N + i] : 0.0;
    const double f = occ[i];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const double* B = tab + P2_T_B + NE * q;
      double uq = 0.0;
#pragma unroll
      for (int a = 0; a < NE; ++a) uq += B[a] * u[a];
      rho[q] += f * uq * uq;
    }
  }
}

__global__ void __launch_bounds__(TPB) k_qp_density_p2(int64_t nt, const int32_t* __restrict__ el,
                                                       const int32_t* __restrict__ v2d, const double* __restrict__ X,
                                                       int N, const double* __restrict__ occ,
                                                       const double* __restrict__ tab, double* __restrict__ rho_out) {
  const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= nt) return;
  double rho[NQ];
  tet_density_p2(el, v2d, X, N, occ, tab, t, rho);
#pragma unroll
  for (int q = 0; q < NQ; ++q) rho_out[NQ * t + q] = rho[q];
}

// As k_qp_fields of the P1 kernels: rho^l, V_xc, eps_xc, V_eff at the 27
// points; block partials of the 10 raw multipole moments and of min V_eff.
constexpr int NMOM = 11;
__global__ void __launch_bounds__(TPB) k_qp_fields_p2(int64_t nt, const int32_t* __restrict__ el,
                                                      const int32_t* __restrict__ v2d, const double* __restrict__ Phi,
                                                      int N, const double* __restrict__ occ,
                                                      const double* __restrict__ wnod,
                                                      const double* __restrict__ vext, const double* __restrict__ geo,
                                                      const double* __restrict__ qpx, int xck, double xalpha,
                                                      const double* __restrict__ tab, double* __restrict__ vxc,
                                                      double* __restrict__ exc, double* __restrict__ veff,
                                                      double* __restrict__ rho_out, double* __restrict__ partials) {
  __shared__ double sd[TPB];
  const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  double mom[NMOM];
#pragma unroll
  for (int k = 0; k < NMOM - 1; ++k) mom[k] = 0.0;
  mom[NMOM - 1] = 1e300;
  if (t < nt) {
    double rho[NQ];
    tet_density_p2(el, v2d, Phi, N, occ, tab, t, rho);
    double wv[NE];
#pragma unroll
    for (int a = 0; a < NE; ++a) wv[a] = wnod[el[NE * t + a]];
    const double vol = geo[16 * t];
#pragma unroll 3
    for (int q = 0; q < NQ; ++q) {
      const double* B = tab + P2_T_B + NE * q;
      double wq = 0.0;
#pragma unroll
      for (int a = 0; a < NE; ++a) wq += B[a] * wv[a];
      double e, v;
      xc_point(xck, xalpha, rho[q], &e, &v);
      const int64_t i = NQ * t + q;
      const double ve = vext[i] + wq + v;
      vxc[i] = v;
      exc[i] = e;
      veff[i] = ve;
      rho_out[i] = rho[q];
      const double m = vol * tab[P2_T_W + q] * rho[q];
      const double x = qpx[3 * i], y = qpx[3 * i + 1], z = qpx[3 * i + 2];
      mom[0] += m;
      mom[1] += m * x;
      mom[2] += m * y;
      mom[3] += m * z;
      mom[4] += m * x * x;
      mom[5] += m * y * y;
      mom[6] += m * z * z;
      mom[7] += m * x * y;
      mom[8] += m * x * z;
      mom[9] += m * y * z;
      mom[10] = fmin(mom[10], ve);
    }
  }
  for (int k = 0; k < NMOM; ++k) {
    __syncthreads();
    sd[threadIdx.x] = mom[k];
    for (int s = TPB / 2; s > 0; s >>= 1) {
      __syncthreads();
      if ((int)threadIdx.x < s) {
        if (k == NMOM - 1)
          sd[threadIdx.x] = fmin(sd[threadIdx.x], sd[threadIdx.x + s]);
        else
          sd[threadIdx.x] += sd[threadIdx.x + s];
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * NMOM + k] = sd[0];
  }
}

// out(t,q) = sum_a phi_a(q) val(node a) + add1(t,q) + add2(t,q), with
// val(v) = nod[v] (if nod) + dofv[v2d[v]] (if dofv and v is interior).
__global__ void __launch_bounds__(TPB) k_field_p2(int64_t nt, const int32_t* __restrict__ el,
                                                  const double* __restrict__ nod, const int32_t* __restrict__ v2d,
                                                  const double* __restrict__ dofv, const double* __restrict__ add1,
                                                  const double* __restrict__ add2, const double* __restrict__ tab,
                                                  double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= nt) return;
  double u[NE];
#pragma unroll
  for (int a = 0; a < NE; ++a) {
    const int v = el[NE * t + a];
    double x = nod ? nod[v] : 0.0;
    if (dofv) {
      const int d = v2d[v];
      if (d >= 0) x += dofv[d];
    }
    u[a] = x;
  }
#pragma unroll 3
  for (int q = 0; q < NQ; ++q) {
    const double* B = tab + P2_T_B + NE * q;
    double o = 0.0;
#pragma unroll
    for (int a = 0; a < NE; ++a) o += B[a] * u[a];
    const int64_t i = NQ * t + q;
    if (add1) o += add1[i];
    if (add2) o += add2[i];
    out[i] = o;
  }
}

// Element entries of op1 = cK1 K + M_{f1} + cM1 M and op2 = cK2 K + M_{f2}
// (55 symmetric local pairs), each written to its slot-order position
// pos = slot_of[100 t + 10 a + b] (-1: skipped), as the P1 k_elem.
template <bool TWO>
__global__ void __launch_bounds__(TPB) k_elem_p2(int64_t nt, const double* __restrict__ geo, double cK1,
                                                 const double* __restrict__ f1, double cM1, double cK2,
                                                 const double* __restrict__ f2, const int32_t* __restrict__ slot_of,
                                                 const double* __restrict__ tab, double* __restrict__ esl) {
  const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= nt) return;
  const double* G = geo + 16 * t;
  const double vol = G[0];
  double gg[10];
  grad_products(G, gg);
  double w1[NQ], w2[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double wq = vol * tab[P2_T_W + q];
    w1[q] = f1 ? wq * f1[NQ * t + q] : 0.0;
    w2[q] = (TWO && f2) ? wq * f2[NQ * t + q] : 0.0;
  }
  const int32_t* pos = slot_of + (int64_t)NE * NE * t;
  double2* esl2 = reinterpret_cast<double2*>(esl);
  for (int a = 0; a < NE; ++a)
    for (int b = a; b < NE; ++b) {
      const int p = pair_index(a, b);
      const double kv = vol * stiff_entry(tab, p, gg);
      double m1 = 0.0, m2 = 0.0;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const double* B = tab + P2_T_B + NE * q;
        const double bb = B[a] * B[b];
        m1 += w1[q] * bb;
        if (TWO) m2 += w2[q] * bb;
      }
      const double mm = vol * tab[P2_T_MM + p];
      const double e1 = cK1 * kv + m1 + cM1 * mm;
      const double e2 = cK2 * kv + m2;
      const int pab = pos[NE * a + b], pba = pos[NE * b + a];
      if (TWO) {
        if (pab >= 0) esl2[pab] = make_double2(e1, e2);
        if (b != a && pba >= 0) esl2[pba] = make_double2(e1, e2);
      } else {
        if (pab >= 0) esl[pab] = e1;
        if (b != a && pba >= 0) esl[pba] = e1;
      }
    }
}

// Load vector, element pass: L_a = scale sum_q |T| W_q f(q) phi_a(q) and the
// lift l_a = sum over the tet's boundary nodes b of K_ab g_b, into
// e[20 t + a] and e[20 t + 10 + a] (the DoF pass is the P1 one with stride 10).
__global__ void __launch_bounds__(TPB) k_load_elem_p2(int64_t nt, const int32_t* __restrict__ el,
                                                      const double* __restrict__ geo, const double* __restrict__ f,
                                                      double scale, const double* __restrict__ gnod,
                                                      const int32_t* __restrict__ v2d, const double* __restrict__ tab,
                                                      double* __restrict__ e) {
  const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= nt) return;
  const double* G = geo + 16 * t;
  const double vol = G[0];
  double gg[10];
  grad_products(G, gg);
  double fw[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) fw[q] = vol * tab[P2_T_W + q] * f[NQ * t + q];
  bool bnd[NE];
  double gv[NE];
#pragma unroll
  for (int b = 0; b < NE; ++b) {
    const int v = el[NE * t + b];
    bnd[b] = gnod && v2d[v] < 0;
    gv[b] = bnd[b] ? gnod[v] : 0.0;
  }
  for (int a = 0; a < NE; ++a) {
    double load = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) load += fw[q] * tab[P2_T_B + NE * q + a];
    double lift = 0.0;
    for (int b = 0; b < NE; ++b)
      if (bnd[b]) lift += vol * stiff_entry(tab, a <= b ? pair_index(a, b) : pair_index(b, a), gg) * gv[b];
    e[2 * NE * t + a] = scale * load;
    e[2 * NE * t + NE + a] = lift;
  }
}

// Coarse hats of the parent at the 27 points of each fine tet in
// coarse-group order e: chat[(4 q + j) ng + e]; its volume at chat[108 ng + e].
// The points are affine in the fine tet's vertices, and the coarse hats are
// linear, so psi_j(q) = sum_c L[q][c] psi_j(vertex c).
__global__ void __launch_bounds__(TPB) k_coarse_hats_p2(int64_t cnt, int64_t ng, const int32_t* __restrict__ grp_ptr,
                                                        const int32_t* __restrict__ grp_tet,
                                                        const int32_t* __restrict__ el,
                                                        const double* __restrict__ geo,
                                                        const double* __restrict__ xyz,
                                                        const double* __restrict__ cgeo,
                                                        const double* __restrict__ tab, double* __restrict__ chat) {
  const int64_t C = blockIdx.x;
  const double* cg = cgeo + 12 * C;
  for (int e = grp_ptr[C] + threadIdx.x; e < grp_ptr[C + 1]; e += TPB) {
    const int64_t t = grp_tet[e];
    double Bc[4][4];
#pragma unroll
    for (int c = 0; c < 4; ++c) coarse_bary(cg, xyz, el[NE * t + c], Bc[c]);
    for (int q = 0; q < NQ; ++q) {
      const double* L = tab + P2_T_L + 4 * q;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        chat[(int64_t)(4 * q + j) * ng + e] = L[0] * Bc[0][j] + L[1] * Bc[1][j] + L[2] * Bc[2][j] + L[3] * Bc[3][j];
    }
    chat[(int64_t)(4 * NQ) * ng + e] = geo[16 * t];
  }
}

__device__ __forceinline__ void coarse_grads(const double* __restrict__ cg, double g[4][3]) {
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    g[1][x] = cg[3 + x];
    g[2][x] = cg[6 + x];
    g[3][x] = cg[9 + x];
    g[0][x] = -(g[1][x] + g[2][x] + g[3][x]);
  }
}

// [A_fix = 1/2 K + M_{fA}] [M_{fW}] [M] [K] in the coarse hats, 40 values per
// coarse tet, summed over its fine tets and their 27 points.
__global__ void __launch_bounds__(TPB) k_coarse_ops_p2(int64_t cnt, int64_t ng, const int32_t* __restrict__ grp_ptr,
                                                       const int32_t* __restrict__ grp_tet,
                                                       const double* __restrict__ chat,
                                                       const double* __restrict__ cgeo,
                                                       const double* __restrict__ fA, const double* __restrict__ fW,
                                                       const double* __restrict__ tab, double* __restrict__ out) {
  __shared__ double ws[4 * 40];
  const int64_t C = blockIdx.x;
  double acc[40];
#pragma unroll
  for (int k = 0; k < 40; ++k) acc[k] = 0.0;
  double gc[4][3];
  coarse_grads(cgeo + 12 * C, gc);
  for (int e = grp_ptr[C] + threadIdx.x; e < grp_ptr[C + 1]; e += TPB) {
    const int64_t t = grp_tet[e];
    const double vol = chat[(int64_t)(4 * NQ) * ng + e];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int m = j; m < 4; ++m) {
        const int k = j * 4 - (j * (j - 1)) / 2 + (m - j);
        const double kv = vol * (gc[j][0] * gc[m][0] + gc[j][1] * gc[m][1] + gc[j][2] * gc[m][2]);
        acc[k] += 0.5 * kv;
        acc[30 + k] += kv;
      }
    for (int q = 0; q < NQ; ++q) {
      const double wq = vol * tab[P2_T_W + q];
      const double wA = fA ? wq * fA[NQ * t + q] : 0.0;
      const double wW = fW ? wq * fW[NQ * t + q] : 0.0;
      double ps[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) ps[j] = chat[(int64_t)(4 * q + j) * ng + e];
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int m = j; m < 4; ++m) {
          const int k = j * 4 - (j * (j - 1)) / 2 + (m - j);
          const double pp = ps[j] * ps[m];
          acc[k] += wA * pp;
          acc[10 + k] += wW * pp;
          acc[20 + k] += wq * pp;
        }
    }
  }
  const double v = block_sums<40>(acc, ws);
  if (threadIdx.x < 40) out[40 * C + threadIdx.x] = v;
}

// Per orbital i and coarse tet: the 10 entries (u_i psi_j, psi_m) and the 4
// entries (u_i^2, psi_j), as the P1 k_coarse_orb: one block per coarse tet,
// fine tets in LDS tiles (their hat values, volumes and DoFs), lane l of each
// wave owns orbital i0 + l, the 4 waves take every 4th tet of a tile, and
// the 4 partial sums per orbital are added in a fixed order.
constexpr int ORB2_TILE = 32;
constexpr int ORB2_STRIDE = 4 * NQ + 1;
__global__ void __launch_bounds__(256) k_coarse_orb_p2(int64_t cnt, int64_t ng, const int32_t* __restrict__ grp_ptr,
                                                       const int32_t* __restrict__ grp_dof,
                                                       const double* __restrict__ chat,
                                                       const double* __restrict__ U, int N,
                                                       const double* __restrict__ tab, double* __restrict__ out) {
  __shared__ double sh[ORB2_TILE * ORB2_STRIDE];
  __shared__ int32_t sdof[ORB2_TILE * NE];
  __shared__ double red[3 * 14 * 64];
  const int64_t C = blockIdx.x;
  const int lane = threadIdx.x & 63, slot = threadIdx.x >> 6;
  const int e0 = grp_ptr[C], e1 = grp_ptr[C + 1];
  for (int i0 = 0; i0 < N; i0 += 64) {
    const int i = i0 + lane;
    const int ic = i < N ? i : N - 1;  // lanes past N repeat the last orbital (never stored)
    double acc[14];
#pragma unroll
    for (int k = 0; k < 14; ++k) acc[k] = 0.0;
    for (int t0 = e0; t0 < e1; t0 += ORB2_TILE) {
      const int ne = e1 - t0 < ORB2_TILE ? e1 - t0 : ORB2_TILE;
      __syncthreads();
      for (int k = threadIdx.x; k < ORB2_STRIDE * ne; k += 256) {
        const int q = k / ne, t = k - q * ne;
        sh[t * ORB2_STRIDE + q] = chat[(int64_t)q * ng + t0 + t];
      }
      for (int k = threadIdx.x; k < NE * ne; k += 256) sdof[k] = grp_dof[(int64_t)NE * t0 + k];
      __syncthreads();
      for (int t = slot; t < ne; t += 4) {
        double u[NE];
#pragma unroll
        for (int a = 0; a < NE; ++a) {
          const int dof = sdof[NE * t + a];
          const double v = U[(int64_t)(dof >= 0 ? dof : 0) * N + ic];
          u[a] = dof >= 0 ? v : 0.0;
        }
        const double* h = sh + t * ORB2_STRIDE;
        const double vol = h[4 * NQ];
#pragma unroll 3
        for (int q = 0; q < NQ; ++q) {
          const double* B = tab + P2_T_B + NE * q;
          double uq = 0.0;
#pragma unroll
          for (int a = 0; a < NE; ++a) uq += B[a] * u[a];
          const double wu = vol * tab[P2_T_W + q] * uq;
          double ps[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) ps[j] = h[4 * q + j];
#pragma unroll
          for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int m = j; m < 4; ++m) acc[j * 4 - (j * (j - 1)) / 2 + (m - j)] += wu * ps[j] * ps[m];
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[10 + j] += wu * uq * ps[j];
        }
      }
    }
    __syncthreads();
    if (slot > 0)
#pragma unroll
      for (int k = 0; k < 14; ++k) red[((slot - 1) * 14 + k) * 64 + lane] = acc[k];
    __syncthreads();
    if (slot == 0 && i < N) {
#pragma unroll
      for (int k = 0; k < 14; ++k) {
        const double v = ((acc[k] + red[k * 64 + lane]) + red[(14 + k) * 64 + lane]) + red[(28 + k) * 64 + lane];
        out[14 * (C * N + i) + k] = v;
      }
    }
  }
}

// Trilinear tensor T_jkm = int psi_j psi_k psi_m (fine 27-point rule), 20
// entries (j <= k <= m) per coarse tet.
__global__ void __launch_bounds__(TPB) k_coarse_tri_p2(int64_t cnt, const int32_t* __restrict__ grp_ptr,
                                                       const int32_t* __restrict__ grp_tet,
                                                       const int32_t* __restrict__ el,
                                                       const double* __restrict__ geo,
                                                       const double* __restrict__ xyz,
                                                       const double* __restrict__ cgeo,
                                                       const double* __restrict__ tab, double* __restrict__ out) {
  __shared__ double ws[4 * 20];
  const int64_t C = blockIdx.x;
  double acc[20];
#pragma unroll
  for (int k = 0; k < 20; ++k) acc[k] = 0.0;
  const double* cg = cgeo + 12 * C;
  for (int e = grp_ptr[C] + threadIdx.x; e < grp_ptr[C + 1]; e += TPB) {
    const int64_t t = grp_tet[e];
    const double vol = geo[16 * t];
    double Bc[4][4];
#pragma unroll
    for (int c = 0; c < 4; ++c) coarse_bary(cg, xyz, el[NE * t + c], Bc[c]);
    for (int q = 0; q < NQ; ++q) {
      const double* L = tab + P2_T_L + 4 * q;
      double ps[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) ps[j] = L[0] * Bc[0][j] + L[1] * Bc[1][j] + L[2] * Bc[2][j] + L[3] * Bc[3][j];
      const double w = vol * tab[P2_T_W + q];
      int k = 0;
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int m = j; m < 4; ++m)
#pragma unroll
          for (int l = m; l < 4; ++l, ++k) acc[k] += w * ps[j] * ps[m] * ps[l];
    }
  }
  const double v = block_sums<20>(acc, ws);
  if (threadIdx.x < 20) out[20 * C + threadIdx.x] = v;
}

// Energy pieces per block: [int rho, int (-1/2 w rho + rho (eps_xc(rho) - v_xc^l))].
__global__ void __launch_bounds__(TPB) k_energy_p2(int64_t nt, const int32_t* __restrict__ el,
                                                   const int32_t* __restrict__ v2d, const double* __restrict__ Phi,
                                                   int N, const double* __restrict__ occ,
                                                   const double* __restrict__ wnod,
                                                   const double* __restrict__ vxc_old,
                                                   const double* __restrict__ geo, int xck, double xalpha,
                                                   const double* __restrict__ tab, double* __restrict__ partials) {
  __shared__ double sd[TPB];
  const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (t < nt) {
    double rho[NQ];
    tet_density_p2(el, v2d, Phi, N, occ, tab, t, rho);
    double wv[NE];
#pragma unroll
    for (int a = 0; a < NE; ++a) wv[a] = wnod[el[NE * t + a]];
    const double vol = geo[16 * t];
#pragma unroll 3
    for (int q = 0; q < NQ; ++q) {
      const double* B = tab + P2_T_B + NE * q;
      double wq = 0.0;
#pragma unroll
      for (int a = 0; a < NE; ++a) wq += B[a] * wv[a];
      double e, vx;
      xc_point(xck, xalpha, rho[q], &e, &vx);
      const double w = vol * tab[P2_T_W + q];
      v[0] += w * rho[q];
      v[1] += w * (-0.5 * wq * rho[q] + rho[q] * (e - vxc_old[NQ * t + q]));
    }
  }
  for (int k = 0; k < 2; ++k) {
    __syncthreads();
    sd[threadIdx.x] = v[k];
    for (int s = TPB / 2; s > 0; s >>= 1) {
      __syncthreads();
      if ((int)threadIdx.x < s) sd[threadIdx.x] += sd[threadIdx.x + s];
    }
    __syncthreads();
    if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * 2 + k] = sd[0];
  }
}

}  // namespace

void launch_qp_density_p2(hipStream_t s, int64_t nt, const int32_t* el, const int32_t* v2d, const double* X, int N,
                          const double* occ, const double* tab, double* rho_out) {
  hipLaunchKernelGGL(k_qp_density_p2, dim3(nb(nt)), dim3(TPB), 0, s, nt, el, v2d, X, N, occ, tab, rho_out);
}
void launch_qp_fields_p2(hipStream_t s, int64_t nt, const int32_t* el, const int32_t* v2d, const double* Phi, int N,
                         const double* occ, const double* wnod, const double* vext, const double* geo,
                         const double* qpx, int xck, double xalpha, const double* tab, double* vxc, double* exc,
                         double* veff, double* rho, double* partials) {
  hipLaunchKernelGGL(k_qp_fields_p2, dim3(nb(nt)), dim3(TPB), 0, s, nt, el, v2d, Phi, N, occ, wnod, vext, geo, qpx,
                     xck, xalpha, tab, vxc, exc, veff, rho, partials);
}
void launch_field_p2(hipStream_t s, int64_t nt, const int32_t* el, const double* nod, const int32_t* v2d,
                     const double* dofv, const double* add1, const double* add2, const double* tab, double* out) {
  hipLaunchKernelGGL(k_field_p2, dim3(nb(nt)), dim3(TPB), 0, s, nt, el, nod, v2d, dofv, add1, add2, tab, out);
}
void launch_assemble2_p2(hipStream_t s, int64_t nt, int64_t n, int64_t nnz, const double* geo,
                         const int32_t* slot_ptr, const int32_t* slot_of, const int32_t* diag_slot, double* esl,
                         double cK1, const double* f1, double cM1, double* val1, double* dinv1, double cK2,
                         const double* f2, double* val2, const double* tab) {
  if (val2)
    hipLaunchKernelGGL(k_elem_p2<true>, dim3(nb(nt)), dim3(TPB), 0, s, nt, geo, cK1, f1, cM1, cK2, f2, slot_of, tab,
                       esl);
  else
    hipLaunchKernelGGL(k_elem_p2<false>, dim3(nb(nt)), dim3(TPB), 0, s, nt, geo, cK1, f1, cM1, cK2, f2, slot_of, tab,
                       esl);
  launch_slot_sum(s, nnz, slot_ptr, esl, val1, val2);
  if (dinv1) launch_diag_inv(s, n, diag_slot, val1, dinv1);
}
void launch_load_p2(hipStream_t s, int64_t n, int64_t nt, const int32_t* adj_ptr, const int32_t* adj_tet,
                    const int8_t* adj_loc, const int32_t* el, const double* geo, const double* f_qp, double scale,
                    const double* gnod, const int32_t* v2d, const double* tab, double* scratch, double* b,
                    double* lvec) {
  hipLaunchKernelGGL(k_load_elem_p2, dim3(nb(nt)), dim3(TPB), 0, s, nt, el, geo, f_qp, scale, gnod, v2d, tab,
                     scratch);
  launch_load_gather(s, n, NE, adj_ptr, adj_tet, adj_loc, scratch, b, lvec);
}
void launch_coarse_hats_p2(hipStream_t s, int64_t cnt, int64_t ng, const int32_t* grp_ptr, const int32_t* grp_tet,
                           const int32_t* el, const double* geo, const double* xyz, const double* cgeo,
                           const double* tab, double* chat) {
  hipLaunchKernelGGL(k_coarse_hats_p2, dim3((unsigned)cnt), dim3(TPB), 0, s, cnt, ng, grp_ptr, grp_tet, el, geo, xyz,
                     cgeo, tab, chat);
}
void launch_coarse_ops_p2(hipStream_t s, int64_t cnt, int64_t ng, const int32_t* grp_ptr, const int32_t* grp_tet,
                          const double* chat, const double* cgeo, const double* fA, const double* fW,
                          const double* tab, double* out) {
  hipLaunchKernelGGL(k_coarse_ops_p2, dim3((unsigned)cnt), dim3(TPB), 0, s, cnt, ng, grp_ptr, grp_tet, chat, cgeo, fA,
                     fW, tab, out);
}
void launch_coarse_orb_p2(hipStream_t s, int64_t cnt, int64_t ng, const int32_t* grp_ptr, const int32_t* grp_dof,
                          const double* chat, const double* U, int N, const double* tab, double* out) {
  hipLaunchKernelGGL(k_coarse_orb_p2, dim3((unsigned)cnt), dim3(256), 0, s, cnt, ng, grp_ptr, grp_dof, chat, U, N,
                     tab, out);
}
void launch_coarse_tri_p2(hipStream_t s, int64_t cnt, const int32_t* grp_ptr, const int32_t* grp_tet,
                          const int32_t* el, const double* geo, const double* xyz, const double* cgeo,
                          const double* tab, double* out) {
  hipLaunchKernelGGL(k_coarse_tri_p2, dim3((unsigned)cnt), dim3(TPB), 0, s, cnt, grp_ptr, grp_tet, el, geo, xyz, cgeo,
                     tab, out);
}
void launch_energy_p2(hipStream_t s, int64_t nt, const int32_t* el, const int32_t* v2d, const double* Phi, int N,
                      const double* occ, const double* wnod, const double* vxc_old, const double* geo, int xck,
                      double xalpha, const double* tab, double* partials) {
  hipLaunchKernelGGL(k_energy_p2, dim3(nb(nt)), dim3(TPB), 0, s, nt, el, v2d, Phi, N, occ, wnod, vxc_old, geo, xck,
                     xalpha, tab, partials);
}

}  // namespace mlc
