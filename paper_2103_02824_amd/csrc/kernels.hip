// gfx950 kernels of the fine-mesh correction step.
//
// Layouts (all device memory comes from the caller's workspace):
//   orbital blocks  n x N row-major, orbital index fastest, so the N values of
//                   one DoF are one contiguous 8N-byte segment;
//   fields at quadrature points  nt x 4 (4-point rule, barycentric (a,b,b,b));
//   operators       CSR over interior DoFs, int32 indices, FP64 values.
//
// Every reduction is two-stage and ordered (block partials, then one block
// summing partials in block order), so results are bitwise reproducible from
// run to run. The kernels of this file use no atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "mlc_internal.h"
#include "pointwise.h"

namespace mlc {

namespace {

constexpr int TPB = 256;

__device__ __forceinline__ double Lq(int q, int j) { return q == j ? QA : QB; }

// Ordered in-block reduction of R rows x N columns held in sd[row*N + col];
// leaves the column sums in sd[col].
__device__ __forceinline__ void block_reduce_cols(double* sd, int R, int N) {
  int t = threadIdx.x;
  int m = R;
  while (m > 1) {
    int h = (m + 1) >> 1;
    __syncthreads();
    if (t < (m - h) * N) sd[t] += sd[t + h * N];
    m = h;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(TPB) k_vext(int64_t npts, const double* __restrict__ qpx, int n_nuclei,
                                              const double* __restrict__ RZ, int kind, double rc,
                                              double omega, double* __restrict__ vext) {
  int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= npts) return;
  vext[i] = vext_point(qpx[3 * i], qpx[3 * i + 1], qpx[3 * i + 2], n_nuclei, RZ, kind, rc, omega);
}

// rho(q) = sum_i f_i phi_i(q)^2 for one tet; phi from nodal interior values.
__device__ __forceinline__ void tet_density(const int32_t* __restrict__ tets, const int32_t* __restrict__ v2d,
                                            const double* __restrict__ X, int N, const double* __restrict__ occ,
                                            int64_t t, double rho[4]) {
  int dof[4];
  for (int j = 0; j < 4; ++j) dof[j] = v2d[tets[4 * t + j]];
  for (int q = 0; q < 4; ++q) rho[q] = 0.0;
  for (int i = 0; i < N; ++i) {
    double u[4];
    for (int j = 0; j < 4; ++j) u[j] = dof[j] >= 0 ? X[(int64_t)dof[j] * N + i] : 0.0;
    double s = u[0] + u[1] + u[2] + u[3];
    double f = occ[i];
    for (int q = 0; q < 4; ++q) {
      double uq = QB * s + (QA - QB) * u[q];
      rho[q] += f * uq * uq;
    }
  }
}

__global__ void __launch_bounds__(TPB) k_qp_density(int64_t nt, const int32_t* __restrict__ tets,
                                                    const int32_t* __restrict__ v2d, const double* __restrict__ X,
                                                    int N, const double* __restrict__ occ,
                                                    double* __restrict__ rho_out) {
  int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= nt) return;
  double rho[4];
  tet_density(tets, v2d, X, N, occ, t, rho);
  for (int q = 0; q < 4; ++q) rho_out[4 * t + q] = rho[q];
}

// Per tet: rho^l, V_xc, eps_xc, V_eff = V_ext + w^l + V_xc at the 4 points;
// block partials of the multipole raw moments (10) and of min V_eff.
constexpr int NMOM = 11;  // Q, Dx,Dy,Dz, Sxx,Syy,Szz,Sxy,Sxz,Syz, min veff
__global__ void __launch_bounds__(TPB) k_qp_fields(int64_t nt, const int32_t* __restrict__ tets,
                                                   const int32_t* __restrict__ v2d, const double* __restrict__ Phi,
                                                   int N, const double* __restrict__ occ,
                                                   const double* __restrict__ wnod, const double* __restrict__ vext,
                                                   const double* __restrict__ geo, const double* __restrict__ qpx,
                                                   int xck, double xalpha, double* __restrict__ vxc,
                                                   double* __restrict__ exc, double* __restrict__ veff,
                                                   double* __restrict__ rho_out, double* __restrict__ partials) {
  __shared__ double sd[TPB];
  int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  double mom[NMOM];
  for (int k = 0; k < NMOM - 1; ++k) mom[k] = 0.0;
  mom[NMOM - 1] = 1e300;
  if (t < nt) {
    double rho[4];
    tet_density(tets, v2d, Phi, N, occ, t, rho);
    double wv[4];
    for (int j = 0; j < 4; ++j) wv[j] = wnod[tets[4 * t + j]];
    double ws = wv[0] + wv[1] + wv[2] + wv[3];
    double wq4 = 0.25 * geo[16 * t];
    for (int q = 0; q < 4; ++q) {
      double e, v;
      xc_point(xck, xalpha, rho[q], &e, &v);
      double wq = QB * ws + (QA - QB) * wv[q];
      double ve = vext[4 * t + q] + wq + v;
      vxc[4 * t + q] = v;
      exc[4 * t + q] = e;
      veff[4 * t + q] = ve;
      rho_out[4 * t + q] = rho[q];
      double m = wq4 * rho[q];
      double x = qpx[12 * t + 3 * q], y = qpx[12 * t + 3 * q + 1], z = qpx[12 * t + 3 * q + 2];
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

// Sum (or min for the last value when minlast) over nblk partial rows.
__global__ void __launch_bounds__(TPB) k_reduce_rows(const double* __restrict__ partials, int nblk, int nvals,
                                                     int minlast, double* __restrict__ out) {
  __shared__ double sd[TPB];
  for (int k = 0; k < nvals; ++k) {
    bool mn = minlast && k == nvals - 1;
    double acc = mn ? 1e300 : 0.0;
    for (int b = threadIdx.x; b < nblk; b += TPB) {
      double v = partials[(int64_t)b * nvals + k];
      acc = mn ? fmin(acc, v) : acc + v;
    }
    __syncthreads();
    sd[threadIdx.x] = acc;
    for (int s = TPB / 2; s > 0; s >>= 1) {
      __syncthreads();
      if ((int)threadIdx.x < s) sd[threadIdx.x] = mn ? fmin(sd[threadIdx.x], sd[threadIdx.x + s]) : sd[threadIdx.x] + sd[threadIdx.x + s];
    }
    __syncthreads();
    if (threadIdx.x == 0) out[k] = sd[0];
  }
}

// Multipole Dirichlet data at boundary vertices from raw moments about the
// origin, shifted to the charge centroid c:
//   g = Q/r + p.r/r^3 + 1/2 r.Qt.r / r^5, Qt traceless, r = x - c.
__global__ void __launch_bounds__(TPB) k_boundary_g(int64_t nb, const int32_t* __restrict__ bverts,
                                                    const double* __restrict__ xyz, const double* __restrict__ mom,
                                                    double* __restrict__ g) {
  int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= nb) return;
  double Q = mom[0];
  double c[3] = {mom[1] / Q, mom[2] / Q, mom[3] / Q};
  double p[3] = {mom[1] - Q * c[0], mom[2] - Q * c[1], mom[3] - Q * c[2]};
  double S[3][3] = {{mom[4], mom[7], mom[8]}, {mom[7], mom[5], mom[9]}, {mom[8], mom[9], mom[6]}};
  double Sc[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Sc[a][b] = S[a][b] - c[a] * mom[1 + b] - c[b] * mom[1 + a] + Q * c[a] * c[b];
  double tr = Sc[0][0] + Sc[1][1] + Sc[2][2];
  int v = bverts[i];
  double r[3] = {xyz[3 * v] - c[0], xyz[3 * v + 1] - c[1], xyz[3 * v + 2] - c[2]};
  double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
  double rn = sqrt(r2);
  double quad = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) quad += r[a] * (3.0 * Sc[a][b] - (a == b ? tr : 0.0)) * r[b];
  double pr = p[0] * r[0] + p[1] * r[1] + p[2] * r[2];
  g[v] = Q / rn + pr / (r2 * rn) + 0.5 * quad / (r2 * r2 * rn);
}

// out(t,q) = sum_j L[q][j] val(v_j) + add1(t,q) + add2(t,q), with
// val(v) = nod[v] (if nod) + dofv[v2d[v]] (if dofv and v is interior).
__global__ void __launch_bounds__(TPB) k_field(int64_t nt, const int32_t* __restrict__ tets,
                                               const double* __restrict__ nod, const int32_t* __restrict__ v2d,
                                               const double* __restrict__ dofv, const double* __restrict__ add1,
                                               const double* __restrict__ add2, double* __restrict__ out) {
  int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= nt) return;
  double u[4];
  for (int j = 0; j < 4; ++j) {
    int v = tets[4 * t + j];
    double a = nod ? nod[v] : 0.0;
    if (dofv) {
      int d = v2d[v];
      if (d >= 0) a += dofv[d];
    }
    u[j] = a;
  }
  double s = u[0] + u[1] + u[2] + u[3];
  for (int q = 0; q < 4; ++q) {
    double o = QB * s + (QA - QB) * u[q];
    if (add1) o += add1[4 * t + q];
    if (add2) o += add2[4 * t + q];
    out[4 * t + q] = o;
  }
}

// Element entries (10 symmetric local pairs, order (0,0)(0,1)..(3,3)) of
//   op1 = cK1 K + M_{f1} + cM1 M  and  op2 = cK2 K + M_{f2}
// for one tet per thread (the mass parts use the 4-point rule), each written
// to its slot-order position pos = slot_of[16 t + 4 a + b] (-1: skipped):
// with TWO the pair (op1, op2) as one 16-byte store at esl2[pos], otherwise
// op1 alone at esl[pos].
template <bool TWO>
__global__ void __launch_bounds__(TPB) k_elem(int64_t nt, const double* __restrict__ geo, double cK1,
                                              const double* __restrict__ f1, double cM1, double cK2,
                                              const double* __restrict__ f2, const int32_t* __restrict__ slot_of,
                                              double* __restrict__ esl) {
  int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= nt) return;
  int32_t pos[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) pos[k] = slot_of[16 * t + k];
  const double* G = geo + 16 * t;
  double vol = G[0];
  double g[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int x = 0; x < 3; ++x) g[a][x] = G[1 + 3 * a + x];
  double w1[4], w2[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    w1[q] = 0.25 * vol * (f1 ? f1[4 * t + q] : 0.0);
    w2[q] = 0.25 * vol * (f2 ? f2[4 * t + q] : 0.0);
  }
  double2* esl2 = reinterpret_cast<double2*>(esl);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a; b < 4; ++b) {
      double kv = vol * (g[a][0] * g[b][0] + g[a][1] * g[b][1] + g[a][2] * g[b][2]);
      double m1 = 0.0, m2 = 0.0, mm = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double ll = Lq(q, a) * Lq(q, b);
        m1 += w1[q] * ll;
        m2 += w2[q] * ll;
        mm += 0.25 * vol * ll;
      }
      const double e1 = cK1 * kv + m1 + cM1 * mm;
      const double e2 = cK2 * kv + m2;
      const int pab = pos[4 * a + b], pba = pos[4 * b + a];
      if (TWO) {
        if (pab >= 0) esl2[pab] = make_double2(e1, e2);
        if (b != a && pba >= 0) esl2[pba] = make_double2(e1, e2);
      } else {
        if (pab >= 0) esl[pab] = e1;
        if (b != a && pba >= 0) esl[pba] = e1;
      }
    }
}

// CSR values: each slot's contiguous run of element entries summed in order.
template <bool TWO>
__global__ void __launch_bounds__(TPB) k_slot_sum(int64_t nnz, const int32_t* __restrict__ slot_ptr,
                                                  const double* __restrict__ esl, double* __restrict__ val1,
                                                  double* __restrict__ val2) {
  int64_t j = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (j >= nnz) return;
  const int e0 = slot_ptr[j], e1 = slot_ptr[j + 1];
  double s1 = 0.0, s2 = 0.0;
  if (TWO) {
    const double2* esl2 = reinterpret_cast<const double2*>(esl);
    for (int e = e0; e < e1; ++e) {
      const double2 v = esl2[e];
      s1 += v.x;
      s2 += v.y;
    }
    val1[j] = s1;
    val2[j] = s2;
  } else {
    for (int e = e0; e < e1; ++e) s1 += esl[e];
    val1[j] = s1;
  }
}

__global__ void __launch_bounds__(TPB) k_diag_inv(int64_t n, const int32_t* __restrict__ diag_slot,
                                                  const double* __restrict__ val, double* __restrict__ dinv) {
  int64_t a = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (a >= n) return;
  dinv[a] = 1.0 / val[diag_slot[a]];
}

// Load vector in two passes. Per tet (one thread): the local load
//   L_a = scale * |T|/4 sum_q f(q) lambda_a(q)
// and the lift of the boundary data, l_a = sum_{boundary vertices b of T} K^T_ab g_b,
// into e[8t + a] and e[8t + 4 + a]. Per interior DoF (one thread): the sums
// over its adjacent tets in tet order, b = L - l and lvec = l.
__global__ void __launch_bounds__(TPB) k_load_elem(int64_t nt, const int32_t* __restrict__ tets,
                                                   const double* __restrict__ geo, const double* __restrict__ f,
                                                   double scale, const double* __restrict__ gnod,
                                                   const int32_t* __restrict__ v2d, double* __restrict__ e) {
  int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= nt) return;
  const double* G = geo + 16 * t;
  const double vol = G[0];
  double fq[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) fq[q] = f[4 * t + q];
  bool bnd[4];
  double gv[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    int v = tets[4 * t + b];
    bnd[b] = gnod && v2d[v] < 0;
    gv[b] = bnd[b] ? gnod[v] : 0.0;
  }
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    double load = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) load += 0.25 * vol * fq[q] * Lq(q, a);
    double lift = 0.0;
#pragma unroll
    for (int b = 0; b < 4; ++b)
      if (bnd[b])
        lift += vol * (G[1 + 3 * a] * G[1 + 3 * b] + G[2 + 3 * a] * G[2 + 3 * b] + G[3 + 3 * a] * G[3 + 3 * b]) *
                gv[b];
    e[8 * t + a] = scale * load;
    e[8 * t + 4 + a] = lift;
  }
}

// (ne: nodes per tet; the element pass wrote 2 ne values per tet)
__global__ void __launch_bounds__(TPB) k_load_gather(int64_t n, int ne, const int32_t* __restrict__ adj_ptr,
                                                     const int32_t* __restrict__ adj_tet,
                                                     const int8_t* __restrict__ adj_loc, const double* __restrict__ e,
                                                     double* __restrict__ b, double* __restrict__ lvec) {
  int64_t a = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (a >= n) return;
  double load = 0.0, lift = 0.0;
  for (int k = adj_ptr[a]; k < adj_ptr[a + 1]; ++k) {
    int64_t o = 2 * ne * (int64_t)adj_tet[k] + adj_loc[k];
    load += e[o];
    lift += e[o + ne];
  }
  b[a] = load - lift;
  if (lvec) lvec[a] = lift;
}

// Y[r,c] = s[c] * X[r,c]
__global__ void __launch_bounds__(TPB) k_scale_cols_to(int64_t total, int N, const double* __restrict__ X,
                                                       const double* __restrict__ s, double* __restrict__ Y) {
  int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= total) return;
  Y[i] = s[i % N] * X[i];
}

// Per-column block partials of sum_r X[r,c] Y[r,c].
__global__ void __launch_bounds__(TPB) k_coldot(int64_t n, int N, int R, const double* __restrict__ X,
                                                const double* __restrict__ Y, double* __restrict__ partial) {
  __shared__ double sd[TPB];
  int t = threadIdx.x;
  int rl = t / N, c = t - rl * N;
  int64_t r = (int64_t)blockIdx.x * R + rl;
  double v = 0.0;
  if (rl < R && r < n) v = X[r * N + c] * Y[r * N + c];
  sd[t] = v;
  block_reduce_cols(sd, R, N);
  if (t < N) partial[(int64_t)blockIdx.x * N + t] = sd[t];
}

// out[c] = sum over blocks of partial[b*N + c] (ordered); one block per column.
__global__ void __launch_bounds__(TPB) k_reduce_cols(int N, int nblk, const double* __restrict__ partial,
                                                     double* __restrict__ out) {
  __shared__ double sd[TPB];
  const int c = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += TPB) acc += partial[(int64_t)b * N + c];
  sd[threadIdx.x] = acc;
  for (int s = TPB / 2; s > 0; s >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < s) sd[threadIdx.x] += sd[threadIdx.x + s];
  }
  if (threadIdx.x == 0) out[c] = sd[0];
}

// X[:,c] /= sqrt(s[c])
__global__ void __launch_bounds__(TPB) k_normalize_cols(int64_t total, int N, const double* __restrict__ s,
                                                        double* __restrict__ X) {
  int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i >= total) return;
  X[i] = X[i] / sqrt(s[i % N]);
}

// Chunked restriction P^T Y. Each block takes one chunk of RESTRICT_CHUNK
// consecutive fine rows: it copies the chunk's rows of Y (contiguous, RCOL
// columns at a time) into LDS with coalesced loads, then each wavefront sums
// the chunk's segments (all entries of one coarse DoF within the chunk, in
// row order) with a lane per column, reading the rows from LDS. Every row of Y
// is read from HBM once; the four coarse parents of a row read it from LDS.
constexpr int RCOL = 64;
constexpr int RENT_MAX = 4 * RESTRICT_CHUNK;  // entries of one chunk: at most four coarse parents per row
__global__ void __launch_bounds__(TPB) k_restrict_chunks(int64_t n, int N, const int32_t* __restrict__ rch_seg,
                                                         const int32_t* __restrict__ rseg_ptr,
                                                         const int32_t* __restrict__ rent_row,
                                                         const double* __restrict__ rent_w,
                                                         const double* __restrict__ Y, double* __restrict__ part) {
  __shared__ double yl[RESTRICT_CHUNK * RCOL];
  __shared__ double ew[RENT_MAX];
  __shared__ int32_t er[RENT_MAX];
  const int64_t r0 = (int64_t)blockIdx.x * RESTRICT_CHUNK;
  const int nr = (int)(n - r0 < RESTRICT_CHUNK ? n - r0 : RESTRICT_CHUNK);
  const int s0 = rch_seg[blockIdx.x], s1 = rch_seg[blockIdx.x + 1];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  // the tile's row stride in LDS: N when one tile holds every column (the
  // chunk's rows of Y are then one contiguous block, copied as such)
  const int ld = N <= RCOL ? N : RCOL;
  const int e00 = rseg_ptr[s0], ne = rseg_ptr[s1] - e00;
  for (int t = threadIdx.x; t < ne; t += TPB) {
    er[t] = rent_row[e00 + t] * ld;
    ew[t] = rent_w[e00 + t];
  }
  for (int c0 = 0; c0 < N; c0 += RCOL) {
    const int nc = N - c0 < RCOL ? N - c0 : RCOL;
    if (N <= RCOL) {
      // contiguous copy, four loads in flight per thread
      const double* src = Y + r0 * N;
      const int tot = nr * N;
      for (int t = threadIdx.x; t < tot; t += 4 * TPB) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = t + u * TPB < tot ? src[t + u * TPB] : 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (t + u * TPB < tot) yl[t + u * TPB] = v[u];
      }
    } else {
      const double* src = Y + r0 * N + c0;
      for (int r = threadIdx.x / RCOL; r < nr; r += TPB / RCOL) {
        const int q = threadIdx.x % RCOL;
        if (q < nc) yl[r * RCOL + q] = src[(int64_t)r * N + q];
      }
    }
    __syncthreads();
    if (lane < nc)
      for (int g = s0 + wid; g < s1; g += TPB / 64) {
        const int e0 = rseg_ptr[g] - e00, e1 = rseg_ptr[g + 1] - e00;
        double acc = 0.0;
        int e = e0;
        for (; e + 4 <= e1; e += 4) {
          const double y0 = yl[er[e] + lane], y1 = yl[er[e + 1] + lane], y2 = yl[er[e + 2] + lane],
                       y3 = yl[er[e + 3] + lane];
          acc += ew[e] * y0;
          acc += ew[e + 1] * y1;
          acc += ew[e + 2] * y2;
          acc += ew[e + 3] * y3;
        }
        for (; e < e1; ++e) acc += ew[e] * yl[er[e] + lane];
        part[(int64_t)g * N + c0 + lane] = acc;
      }
    __syncthreads();
  }
}

// The chunked restriction of one column (N = 1): the chunk's 128 values in
// LDS, a wavefront per segment with its lanes over the segment's entries and
// a fixed shuffle tree for the sum.
__global__ void __launch_bounds__(TPB) k_restrict_chunks1(int64_t n, const int32_t* __restrict__ rch_seg,
                                                          const int32_t* __restrict__ rseg_ptr,
                                                          const int32_t* __restrict__ rent_row,
                                                          const double* __restrict__ rent_w,
                                                          const double* __restrict__ Y, double* __restrict__ part) {
  __shared__ double yl[RESTRICT_CHUNK];
  const int64_t r0 = (int64_t)blockIdx.x * RESTRICT_CHUNK;
  const int nr = (int)(n - r0 < RESTRICT_CHUNK ? n - r0 : RESTRICT_CHUNK);
  const int s0 = rch_seg[blockIdx.x], s1 = rch_seg[blockIdx.x + 1];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int t = threadIdx.x; t < nr; t += TPB) yl[t] = Y[r0 + t];
  __syncthreads();
  for (int g = s0 + wid; g < s1; g += TPB / 64) {
    double acc = 0.0;
    for (int e = rseg_ptr[g] + lane; e < rseg_ptr[g + 1]; e += 64) acc += rent_w[e] * yl[rent_row[e]];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) part[g] = acc;
  }
}

// out[k] = sum of the segment partials of coarse DoF k (N = 1): a wavefront per
// coarse DoF, its lanes over the segments, a fixed shuffle tree.
__global__ void __launch_bounds__(TPB) k_restrict_sum1(int64_t nH, const int32_t* __restrict__ kseg_ptr,
                                                       const int32_t* __restrict__ kseg,
                                                       const double* __restrict__ part, double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * (TPB / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k >= nH) return;
  double acc = 0.0;
  for (int j = kseg_ptr[k] + lane; j < kseg_ptr[k + 1]; j += 64) acc += part[kseg[j]];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
  if (lane == 0) out[k] = acc;
}

// out[k, c] = sum of the segment partials of coarse DoF k, in chunk order: one
// wavefront per coarse DoF, a lane per column.
__global__ void __launch_bounds__(TPB) k_restrict_sum(int64_t nH, int N, const int32_t* __restrict__ kseg_ptr,
                                                      const int32_t* __restrict__ kseg,
                                                      const double* __restrict__ part, double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * (TPB / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k >= nH) return;
  const int j0 = kseg_ptr[k], j1 = kseg_ptr[k + 1];
  for (int c = lane; c < N; c += 64) {
    // four segments' loads in flight, summed in segment order
    double acc = 0.0;
    int j = j0;
    for (; j + 4 <= j1; j += 4) {
      const int64_t g0 = kseg[j], g1 = kseg[j + 1], g2 = kseg[j + 2], g3 = kseg[j + 3];
      const double p0 = part[g0 * N + c], p1 = part[g1 * N + c], p2 = part[g2 * N + c], p3 = part[g3 * N + c];
      acc += p0;
      acc += p1;
      acc += p2;
      acc += p3;
    }
    for (; j < j1; ++j) acc += part[(int64_t)kseg[j] * N + c];
    out[k * N + c] = acc;
  }
}

// Gram block U^T Y (N x N) on the FP64 matrix cores (N <= 16): orbitals are
// padded to 16, rows are the reduction index. One v_mfma_f64_16x16x4f64 per 4
// rows: lane l feeds U[row 4q + l/16][orbital l%16] as A (16 x 4, orbital x
// row) and Y[row 4q + l/16][orbital l%16] as B (4 x 16, row x orbital), and
// accumulates D[l/16 + 4 v][l%16] in its register v = 0..3 (the rows of the
// FP64 16x16 result interleave by four across the lane groups, unlike the
// 16-bit 16x16 forms, whose lane groups hold four consecutive rows; measured
// with a one-wave layout probe). Each block sums GRAM_ROWS rows
// (its four waves take interleaved groups of four rows) and writes its N x N
// partial; the partials are summed in block order afterwards.
constexpr int GRAM_ROWS = 1024;
typedef double f64x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(TPB) k_gram_mfma(int64_t n, int N, const double* __restrict__ U,
                                                   const double* __restrict__ Y, double* __restrict__ partial) {
  __shared__ double sd[TPB / 64][16 * 16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int col = lane & 15, rq = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * GRAM_ROWS;
  const int64_t r1 = r0 + GRAM_ROWS < n ? r0 + GRAM_ROWS : n;
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int64_t rb = r0 + 4 * wid; rb < r1; rb += 16) {
    const int64_t r = rb + rq;
    double a = 0.0, b = 0.0;
    if (r < r1 && col < N) {
      a = U[r * N + col];
      b = Y[r * N + col];
    }
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) sd[wid][(rq + 4 * v) * 16 + col] = acc[v];
  __syncthreads();
  for (int p = threadIdx.x; p < N * N; p += TPB) {
    const int i = p / N, j = p - i * N;
    const int o = i * 16 + j;
    partial[(int64_t)blockIdx.x * N * N + p] = (sd[0][o] + sd[1][o]) + (sd[2][o] + sd[3][o]);
  }
}

// Gram block U^T Y for 16 < N <= 64 on the FP64 matrix cores: the N x N block
// is TI x TI tiles of 16 x 16 (orbitals padded to 16 TI). A block of TI waves
// takes GRAM_ROWS rows; wave w owns tile row w, so it accumulates its TI tiles
// (the same v_mfma_f64_16x16x4f64 lane layout as k_gram_mfma) over all the
// block's rows and writes them to the block's N x N partial directly. Few
// accumulator registers per wave keep several waves per SIMD in flight.
template <int TI>
__global__ void __launch_bounds__(64 * TI) k_gram_mfma_tiles(int64_t n, int N, const double* __restrict__ U,
                                                             const double* __restrict__ Y,
                                                             double* __restrict__ partial) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int col = lane & 15, rq = lane >> 4;
  const int64_t r0 = (int64_t)blockIdx.x * GRAM_ROWS;
  const int64_t r1 = r0 + GRAM_ROWS < n ? r0 + GRAM_ROWS : n;
  f64x4 acc[TI];
#pragma unroll
  for (int bj = 0; bj < TI; ++bj) acc[bj] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int ca = 16 * w + col;
  for (int64_t rb = r0; rb < r1; rb += 4) {
    const int64_t r = rb + rq;
    const bool okr = r < r1;
    const double a = (okr && ca < N) ? U[r * N + ca] : 0.0;
    double b[TI];
#pragma unroll
    for (int bj = 0; bj < TI; ++bj) {
      const int c = 16 * bj + col;
      b[bj] = (okr && c < N) ? Y[r * N + c] : 0.0;
    }
#pragma unroll
    for (int bj = 0; bj < TI; ++bj) acc[bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[bj], acc[bj], 0, 0, 0);
  }
#pragma unroll
  for (int bj = 0; bj < TI; ++bj)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * w + rq + 4 * v, j = 16 * bj + col;
      if (i < N && j < N) partial[(int64_t)blockIdx.x * N * N + (int64_t)i * N + j] = acc[bj][v];
    }
}

// Gram block for N > 16: thread (row, j) with the N products per row in a
// loop, per-block partials by an in-block column reduction per i.
__global__ void __launch_bounds__(TPB) k_gram_wide(int64_t n, int N, const double* __restrict__ U,
                                                   const double* __restrict__ Y, double* __restrict__ partial) {
  __shared__ double sd[TPB];
  const int R = TPB / N;
  const int t = threadIdx.x;
  const int rl = t / N, j = t - rl * N;
  const int64_t r0 = (int64_t)blockIdx.x * GRAM_ROWS;
  const int64_t r1 = r0 + GRAM_ROWS < n ? r0 + GRAM_ROWS : n;
  for (int i = 0; i < N; ++i) {
    double acc = 0.0;
    if (rl < R)
      for (int64_t r = r0 + rl; r < r1; r += R) acc += U[r * N + i] * Y[r * N + j];
    __syncthreads();
    sd[t] = rl < R ? acc : 0.0;
    block_reduce_cols(sd, R, N);
    if (t < N) partial[(int64_t)blockIdx.x * N * N + i * N + t] = sd[t];
  }
}

// ---------------------------------------------------------------------------
// Coarse-pattern integrals, one thread per coarse tet, looping over the fine
// tets inside it (nested meshes: coarse hats are linear on every fine tet,
// psi_j = sum_a Bc[a][j] phi_a with Bc the coarse barycentrics of the fine
// vertices). Results are 4x4 symmetric blocks in coarse local numbering,
// stored as the 10 entries (j<=k) in order (0,0)(0,1)(0,2)(0,3)(1,1)...(3,3).
// Operators: [A_fix = 1/2 K + M_{fA}] [M_{fW}] [M] [K] -> 40 values per coarse
// tet. One workgroup per coarse tet; threads stride over its fine tets.
// Per fine tet, in coarse-group order e (fixed per mesh): the four coarse
// hats of its parent at its four quadrature points, chat[(4 q + j) ng + e],
// and its volume, chat[16 ng + e] (ng = number of fine tets; one array per
// value, so that consecutive threads read consecutive addresses).
__global__ void __launch_bounds__(TPB) k_coarse_hats(int64_t cnt, int64_t ng, const int32_t* __restrict__ grp_ptr,
                                                     const int32_t* __restrict__ grp_tet,
                                                     const int32_t* __restrict__ tets, const double* __restrict__ geo,
                                                     const double* __restrict__ xyz, const double* __restrict__ cgeo,
                                                     double* __restrict__ chat) {
  const int64_t C = blockIdx.x;
  const double* cg = cgeo + 12 * C;
  for (int e = grp_ptr[C] + threadIdx.x; e < grp_ptr[C + 1]; e += TPB) {
    const int64_t t = grp_tet[e];
    double Bc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a) coarse_bary(cg, xyz, tets[4 * t + a], Bc[a]);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double sj = Bc[0][j] + Bc[1][j] + Bc[2][j] + Bc[3][j];
#pragma unroll
      for (int q = 0; q < 4; ++q) chat[(int64_t)(4 * q + j) * ng + e] = QB * sj + (QA - QB) * Bc[q][j];
    }
    chat[16 * ng + e] = geo[16 * t];
  }
}

// Gradients of the coarse hats on coarse tet C (constant there).
__device__ __forceinline__ void coarse_grads(const double* __restrict__ cg, double g[4][3]) {
#pragma unroll
  for (int x = 0; x < 3; ++x) {
    g[1][x] = cg[3 + x];
    g[2][x] = cg[6 + x];
    g[3][x] = cg[9 + x];
    g[0][x] = -(g[1][x] + g[2][x] + g[3][x]);
  }
}

__global__ void __launch_bounds__(TPB) k_coarse_ops(int64_t cnt, int64_t ng, const int32_t* __restrict__ grp_ptr,
                                                    const int32_t* __restrict__ grp_tet,
                                                    const double* __restrict__ chat, const double* __restrict__ cgeo,
                                                    const double* __restrict__ fA, const double* __restrict__ fW,
                                                    double* __restrict__ out) {
  __shared__ double ws[4 * 40];
  int64_t C = blockIdx.x;
  double acc[40];
#pragma unroll
  for (int k = 0; k < 40; ++k) acc[k] = 0.0;
  double gc[4][3];
  coarse_grads(cgeo + 12 * C, gc);
  for (int e = grp_ptr[C] + threadIdx.x; e < grp_ptr[C + 1]; e += TPB) {
    const int64_t t = grp_tet[e];
    const double vol = chat[16 * ng + e];
    double pq[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int j = 0; j < 4; ++j) pq[q][j] = chat[(int64_t)(4 * q + j) * ng + e];
    double wA[4], wW[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      wA[q] = 0.25 * vol * (fA ? fA[4 * t + q] : 0.0);
      wW[q] = 0.25 * vol * (fW ? fW[4 * t + q] : 0.0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int m = j; m < 4; ++m) {
        const int k = j * 4 - (j * (j - 1)) / 2 + (m - j);
        double kv = vol * (gc[j][0] * gc[m][0] + gc[j][1] * gc[m][1] + gc[j][2] * gc[m][2]);
        double mA = 0.0, mW = 0.0, mM = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          double pp = pq[q][j] * pq[q][m];
          mA += wA[q] * pp;
          mW += wW[q] * pp;
          mM += 0.25 * vol * pp;
        }
        acc[k] += 0.5 * kv + mA;
        acc[10 + k] += mW;
        acc[20 + k] += mM;
        acc[30 + k] += kv;
      }
  }
  const double v = block_sums<40>(acc, ws);
  if (threadIdx.x < 40) out[40 * C + threadIdx.x] = v;
}

// Per orbital i and coarse tet: the 10 entries (u_i psi_j, psi_m) and the 4
// entries (u_i^2, psi_j). One block per coarse tet; its fine tets (group
// order, DoFs from the per-mesh table grp_dof) in tiles of ORB_TILE whose hat
// values, weights and DoFs are staged in LDS once for all orbitals. Lane l of
// each wave owns orbital i0 + l (64 orbitals per pass); the block's 4 waves
// take every 4th tet of the tile, ORB_BATCH tets at a time (the LDS reads are
// broadcasts, the U reads of a wave one contiguous row segment each, all of a
// batch in flight together). The 4 partial sums per orbital are added in a
// fixed order.
constexpr int ORB_TILE = 64;
constexpr int ORB_BATCH = 4;
__global__ void __launch_bounds__(256) k_coarse_orb(int64_t cnt, int64_t ng, const int32_t* __restrict__ grp_ptr,
                                                    const int32_t* __restrict__ grp_dof,
                                                    const double* __restrict__ chat, const double* __restrict__ U,
                                                    int N, double* __restrict__ out) {
  __shared__ double sh[ORB_TILE * 17];
  __shared__ int32_t sdof[ORB_TILE * 4];
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
    for (int t0 = e0; t0 < e1; t0 += ORB_TILE) {
      const int ne = e1 - t0 < ORB_TILE ? e1 - t0 : ORB_TILE;
      __syncthreads();
      for (int k = threadIdx.x; k < 17 * ne; k += 256) {
        const int q = k / ne, t = k - q * ne;
        sh[t * 17 + q] = chat[(int64_t)q * ng + t0 + t];
      }
      for (int k = threadIdx.x; k < 4 * ne; k += 256) sdof[k] = grp_dof[4 * (int64_t)t0 + k];
      __syncthreads();
      // ORB_BATCH tets per wave at a time: their U values are loaded together
      // (tets past the tile repeat the last one with weight zero)
      for (int t0 = slot; t0 < ne; t0 += 4 * ORB_BATCH) {
        double u[ORB_BATCH][4];
#pragma unroll
        for (int b = 0; b < ORB_BATCH; ++b) {
          const int t = t0 + 4 * b < ne ? t0 + 4 * b : ne - 1;
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            const int dof = sdof[4 * t + a];
            const double v = U[(int64_t)(dof >= 0 ? dof : 0) * N + ic];
            u[b][a] = dof >= 0 ? v : 0.0;
          }
        }
#pragma unroll 1
        for (int b = 0; b < ORB_BATCH; ++b) {
          const int t = t0 + 4 * b < ne ? t0 + 4 * b : ne - 1;
          const double* h = sh + t * 17;
          const double w = t0 + 4 * b < ne ? 0.25 * h[16] : 0.0;
          const double us = u[b][0] + u[b][1] + u[b][2] + u[b][3];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const double uq = QB * us + (QA - QB) * u[b][q];
            const double wu = w * uq;
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
    }
    // the partial sums of waves 1..3 through LDS, added by wave 0 in slot order
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

// Joint-space variant: per coarse tet and orbital pair (j <= l) the 4 entries
// (u_j u_l, psi_m) over the coarse tet's vertices m; PAIR_CHUNK pairs per pass
// over the fine tets (pairs in the order (0,0), (0,1), ..., (0,N-1), (1,1), ...).
constexpr int PAIR_CHUNK = 4;
__global__ void __launch_bounds__(TPB) k_coarse_pairs(int64_t cnt, int64_t ng, const int32_t* __restrict__ grp_ptr,
                                                      const int32_t* __restrict__ grp_dof,
                                                      const double* __restrict__ chat, const double* __restrict__ U,
                                                      int N, const int32_t* __restrict__ pair_jl, int npair,
                                                      double* __restrict__ out) {
  __shared__ double ws[4 * PAIR_CHUNK * 4];
  const int64_t C = blockIdx.x;
  for (int p0 = 0; p0 < npair; p0 += PAIR_CHUNK) {
    const int np = npair - p0 < PAIR_CHUNK ? npair - p0 : PAIR_CHUNK;
    double acc[PAIR_CHUNK * 4];
#pragma unroll
    for (int k = 0; k < PAIR_CHUNK * 4; ++k) acc[k] = 0.0;
    for (int e = grp_ptr[C] + threadIdx.x; e < grp_ptr[C + 1]; e += TPB) {
      const int4 dq = reinterpret_cast<const int4*>(grp_dof)[e];
      const int dof[4] = {dq.x, dq.y, dq.z, dq.w};
      double h[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) h[k] = chat[(int64_t)k * ng + e];
      const double w = 0.25 * chat[16 * ng + e];
#pragma unroll
      for (int o = 0; o < PAIR_CHUNK; ++o) {
        if (o >= np) continue;
        const int jj = pair_jl[2 * (p0 + o)], ll = pair_jl[2 * (p0 + o) + 1];
        double a[4], b[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          a[q] = dof[q] >= 0 ? U[(int64_t)dof[q] * N + jj] : 0.0;
          b[q] = dof[q] >= 0 ? U[(int64_t)dof[q] * N + ll] : 0.0;
        }
        const double as = a[0] + a[1] + a[2] + a[3], bs = b[0] + b[1] + b[2] + b[3];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double aq = QB * as + (QA - QB) * a[q], bq = QB * bs + (QA - QB) * b[q];
#pragma unroll
          for (int m = 0; m < 4; ++m) acc[4 * o + m] += w * aq * bq * h[4 * q + m];
        }
      }
    }
    const double v = block_sums<PAIR_CHUNK * 4>(acc, ws);
    if ((int)threadIdx.x < 4 * np) out[4 * (C * npair + p0) + threadIdx.x] = v;
  }
}

// Joint-space reconstruction: Phi[a, i] = sum_s Pw[a, s] C[Pk[a, s], i] + sum_j U[a, j] D[j, i]
// (C: N_H x N coarse coefficients, D: N x N coefficients of the u_j).
__global__ void __launch_bounds__(TPB) k_reconstruct_joint(int64_t n, int N, const int32_t* __restrict__ Pk,
                                                           const double* __restrict__ Pw,
                                                           const double* __restrict__ Cc, const double* __restrict__ D,
                                                           const double* __restrict__ U, double* __restrict__ Phi) {
  const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= n * N) return;
  const int64_t a = t / N;
  const int i = (int)(t - a * N);
  double v = 0.0;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int k = Pk[4 * a + s];
    if (k >= 0) v += Pw[4 * a + s] * Cc[(int64_t)k * N + i];
  }
  const double* ua = U + a * N;
  for (int j = 0; j < N; ++j) v += ua[j] * D[j * N + i];
  Phi[t] = v;
}

// Trilinear tensor T_jkm = int psi_j psi_k psi_m (fine quadrature), 20 entries
// (j<=k<=m) per coarse tet; one workgroup per coarse tet.
__global__ void __launch_bounds__(TPB) k_coarse_tri(int64_t cnt, const int32_t* __restrict__ grp_ptr,
                                                    const int32_t* __restrict__ grp_tet,
                                                    const int32_t* __restrict__ tets, const double* __restrict__ geo,
                                                    const double* __restrict__ xyz, const double* __restrict__ cgeo,
                                                    double* __restrict__ out) {
  __shared__ double ws[4 * 20];
  int64_t C = blockIdx.x;
  double acc[20];
#pragma unroll
  for (int k = 0; k < 20; ++k) acc[k] = 0.0;
  const double* cg = cgeo + 12 * C;
  for (int e = grp_ptr[C] + threadIdx.x; e < grp_ptr[C + 1]; e += TPB) {
    int64_t t = grp_tet[e];
    double vol = geo[16 * t];
    double Bc[4][4];
    for (int a = 0; a < 4; ++a) coarse_bary(cg, xyz, tets[4 * t + a], Bc[a]);
    for (int q = 0; q < 4; ++q) {
      double ps[4];
      for (int j = 0; j < 4; ++j) {
        double s = Bc[0][j] + Bc[1][j] + Bc[2][j] + Bc[3][j];
        ps[j] = QB * s + (QA - QB) * Bc[q][j];
      }
      double w = 0.25 * vol;
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

// Phi[a,i] = sum_j Pw[a,j] phiH[Pk[a,j], i] + theta2[i] U[a,i]
__global__ void __launch_bounds__(TPB) k_reconstruct(int64_t n, int N, const int32_t* __restrict__ Pk,
                                                     const double* __restrict__ Pw, const double* __restrict__ phiH,
                                                     const double* __restrict__ theta2, const double* __restrict__ U,
                                                     double* __restrict__ Phi) {
  int64_t id = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (id >= n * N) return;
  int64_t a = id / N;
  int i = (int)(id - a * N);
  double s = 0.0;
  for (int j = 0; j < 4; ++j) {
    int k = Pk[4 * a + j];
    if (k >= 0) s += Pw[4 * a + j] * phiH[(int64_t)k * N + i];
  }
  Phi[id] = s + theta2[i] * U[id];
}

// w(v) = g(v) + sum_j Pw[a,j] wH[Pk[a,j]] + theta1 w0[a]   (a = dof of v; boundary: g)
__global__ void __launch_bounds__(TPB) k_hartree_nodal(int64_t nv, const int32_t* __restrict__ v2d,
                                                       const int32_t* __restrict__ Pk, const double* __restrict__ Pw,
                                                       const double* __restrict__ wH, double theta1,
                                                       const double* __restrict__ w0, const double* __restrict__ g,
                                                       double* __restrict__ w) {
  int64_t v = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (v >= nv) return;
  int a = v2d[v];
  double s = g[v];
  if (a >= 0) {
    for (int j = 0; j < 4; ++j) {
      int k = Pk[4 * (int64_t)a + j];
      if (k >= 0) s += Pw[4 * (int64_t)a + j] * wH[k];
    }
    s += theta1 * w0[a];
  }
  w[v] = s;
}

__global__ void __launch_bounds__(TPB) k_rho_nodal(int64_t nv, const int32_t* __restrict__ v2d,
                                                   const double* __restrict__ Phi, int N,
                                                   const double* __restrict__ occ, double* __restrict__ rho) {
  int64_t v = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (v >= nv) return;
  int a = v2d[v];
  double s = 0.0;
  if (a >= 0)
    for (int i = 0; i < N; ++i) {
      double p = Phi[(int64_t)a * N + i];
      s += occ[i] * p * p;
    }
  rho[v] = s;
}

// Row permutation of an n x N block (orbital fastest): gather reads row
// perm[a] of in into row a of out, scatter writes row a of in to row perm[a].
__global__ void __launch_bounds__(TPB) k_permute_rows(int64_t n, int N, const int32_t* __restrict__ perm,
                                                      const double* __restrict__ in, double* __restrict__ out,
                                                      int gather) {
  int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= n * N) return;
  int64_t a = t / N;
  int i = (int)(t - a * N);
  int64_t pa = perm[a];
  if (gather)
    out[t] = in[pa * N + i];
  else
    out[pa * N + i] = in[t];
}

// out[a] = w[d2v[a]]: the interior (DoF) values of a nodal vector.
__global__ void __launch_bounds__(TPB) k_gather_nodal(int64_t n, const int32_t* __restrict__ d2v,
                                                      const double* __restrict__ w, double* __restrict__ out) {
  int64_t a = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (a < n) out[a] = w[d2v[a]];
}

// Count of non-finite values in two arrays (grid-stride; one atomic per wavefront).
__global__ void __launch_bounds__(TPB) k_count_nonfinite(int64_t na, const double* __restrict__ a, int64_t nb_,
                                                         const double* __restrict__ b, int32_t* __restrict__ cnt) {
  int bad = 0;
  const int64_t stride = (int64_t)gridDim.x * TPB;
  for (int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x; t < na + nb_; t += stride) {
    double v = t < na ? a[t] : b[t - na];
    bad += !isfinite(v);
  }
  for (int o = 32; o > 0; o >>= 1) bad += __shfl_xor(bad, o);
  if ((threadIdx.x & 63) == 0 && bad) atomicAdd(cnt, bad);
}

// Energy pieces per block: [int rho, int (-1/2 w rho + rho (eps_xc(rho) - v_xc^l))]
__global__ void __launch_bounds__(TPB) k_energy(int64_t nt, const int32_t* __restrict__ tets,
                                                const int32_t* __restrict__ v2d, const double* __restrict__ Phi,
                                                int N, const double* __restrict__ occ,
                                                const double* __restrict__ wnod, const double* __restrict__ vxc_old,
                                                const double* __restrict__ geo, int xck, double xalpha,
                                                double* __restrict__ partials) {
  __shared__ double sd[TPB];
  int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  double v[2] = {0.0, 0.0};
  if (t < nt) {
    double rho[4];
    tet_density(tets, v2d, Phi, N, occ, t, rho);
    double wv[4];
    for (int j = 0; j < 4; ++j) wv[j] = wnod[tets[4 * t + j]];
    double ws = wv[0] + wv[1] + wv[2] + wv[3];
    double w4 = 0.25 * geo[16 * t];
    for (int q = 0; q < 4; ++q) {
      double e, vx;
      xc_point(xck, xalpha, rho[q], &e, &vx);
      double wq = QB * ws + (QA - QB) * wv[q];
      v[0] += w4 * rho[q];
      v[1] += w4 * (-0.5 * wq * rho[q] + rho[q] * (e - vxc_old[4 * t + q]));
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

// ---------------------------------------------------------------------------
// Lanczos estimate of lambda_max(D^-1 A) for the Chebyshev interval. D^-1 A is
// self-adjoint in <x, y>_D = sum_i x_i y_i / dinv_i; m Lanczos steps from a
// fixed pseudo-random start give the tridiagonal T_m, whose largest
// eigenvalue (a Ritz value, at most lambda_max) is found by bisection on
// Sturm counts. The bound used is min(Gershgorin, safety x that Ritz value).
// Block partial sums are added in a fixed order (one reduction kernel).
constexpr int LZ_BLOCKS = 1024;
__device__ __forceinline__ void lz_block_sum(double v, double* __restrict__ partial) {
  __shared__ double sd[TPB];
  sd[threadIdx.x] = v;
  for (int h = TPB / 2; h > 0; h >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < h) sd[threadIdx.x] += sd[threadIdx.x + h];
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sd[0];
}

// v_i = a pseudo-random value in [-1, 1) (multiplicative hash of i); partial <v, v>_D.
__global__ void __launch_bounds__(TPB) k_lz_init(int64_t n, const double* __restrict__ dinv, double* __restrict__ v,
                                                 double* __restrict__ partial) {
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
    const uint32_t h = (uint32_t)((uint64_t)(i + 1) * 2654435761ull);
    const double x = (double)h * (2.0 / 4294967296.0) - 1.0;
    v[i] = x;
    acc += x * x / dinv[i];
  }
  lz_block_sum(acc, partial);
}
// v /= sqrt(nrm2[0])
__global__ void __launch_bounds__(TPB) k_lz_scale(int64_t n, const double* __restrict__ nrm2, double* __restrict__ v) {
  const double sc = nrm2[0] > 0.0 ? 1.0 / sqrt(nrm2[0]) : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) v[i] *= sc;
}
// w = D^-1 y - beta v_prev (beta = sqrt(beta2[0]), 0 at the first step); partial <w, v>_D.
__global__ void __launch_bounds__(TPB) k_lz_alpha(int64_t n, const double* __restrict__ dinv,
                                                  const double* __restrict__ y, const double* __restrict__ v,
                                                  const double* __restrict__ vprev, const double* __restrict__ beta2,
                                                  double* __restrict__ w, double* __restrict__ partial) {
  const double beta = beta2 ? sqrt(fmax(beta2[0], 0.0)) : 0.0;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
    const double wi = dinv[i] * y[i] - beta * vprev[i];
    w[i] = wi;
    acc += wi * v[i] / dinv[i];
  }
  lz_block_sum(acc, partial);
}
// w -= alpha v; partial <w, w>_D.
__global__ void __launch_bounds__(TPB) k_lz_orth(int64_t n, const double* __restrict__ dinv,
                                                 const double* __restrict__ alpha, const double* __restrict__ v,
                                                 double* __restrict__ w, double* __restrict__ partial) {
  const double a = alpha[0];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
    const double wi = w[i] - a * v[i];
    w[i] = wi;
    acc += wi * wi / dinv[i];
  }
  lz_block_sum(acc, partial);
}
// v_prev = v; v = w / beta (0 when beta vanishes: an invariant subspace was found).
__global__ void __launch_bounds__(TPB) k_lz_next(int64_t n, const double* __restrict__ beta2,
                                                 const double* __restrict__ w, double* __restrict__ v,
                                                 double* __restrict__ vprev) {
  const double b2 = beta2[0];
  const double sc = b2 > 1e-300 ? 1.0 / sqrt(b2) : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
    vprev[i] = v[i];
    v[i] = w[i] * sc;
  }
}
// Largest eigenvalue of T (diagonal alpha[0..m), off-diagonal sqrt(beta2[1..m))) by bisection on the
// number of eigenvalues below x (Sturm sequence of the LDL^T pivots); lmax[0] = min(lmax[0], safety x it).
__global__ void k_lz_eig(int m, const double* __restrict__ alpha, const double* __restrict__ beta2, double safety,
                         double* __restrict__ lmax) {
  if (threadIdx.x != 0) return;
  double lo = 1e300, hi = -1e300;
  for (int j = 0; j < m; ++j) {
    const double bl = j > 0 ? sqrt(fmax(beta2[j], 0.0)) : 0.0, br = j + 1 < m ? sqrt(fmax(beta2[j + 1], 0.0)) : 0.0;
    lo = fmin(lo, alpha[j] - bl - br);
    hi = fmax(hi, alpha[j] + bl + br);
  }
  if (!(hi > lo) || !(hi < 1e300)) return;
  for (int it = 0; it < 200; ++it) {
    const double x = 0.5 * (lo + hi);
    int below = 0;
    double q = alpha[0] - x;
    if (q < 0.0) ++below;
    for (int j = 1; j < m; ++j) {
      if (q == 0.0) q = 1e-300;
      q = (alpha[j] - x) - fmax(beta2[j], 0.0) / q;
      if (q < 0.0) ++below;
    }
    if (below == m) hi = x;  // every eigenvalue below x
    else lo = x;
  }
  const double est = safety * hi;
  if (est > 0.0 && est < lmax[0]) lmax[0] = est;
}

inline unsigned nb(int64_t work) { return (unsigned)((work + TPB - 1) / TPB); }

// ---------------------------------------------------------------------------
// Learned initial guess of step 5 (the features, the start x0 = phi + s y, the
// per-column residual judge and the training-sample sink).

// Per-block column maxima of |X| (thread (row, column) layout).
__global__ void __launch_bounds__(TPB) k_colmax_abs(int64_t n, int N, int R, const double* __restrict__ X,
                                                    double* __restrict__ partial) {
  __shared__ double sd[TPB];
  int t = threadIdx.x;
  int rl = t / N, c = t - rl * N;
  double v = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * R + rl; rl < R && r < n; r += (int64_t)gridDim.x * R)
    v = fmax(v, fabs(X[r * N + c]));
  sd[t] = v;
  int m = R;
  while (m > 1) {
    int h = (m + 1) >> 1;
    __syncthreads();
    if (t < (m - h) * N) sd[t] = fmax(sd[t], sd[t + h * N]);
    m = h;
  }
  __syncthreads();
  if (t < N) partial[(int64_t)blockIdx.x * N + t] = sd[t];
}

// out[c] = max over blocks (1 where the column is zero).
__global__ void __launch_bounds__(TPB) k_colmax_final(int N, int nblk, const double* __restrict__ partial,
                                                      double* __restrict__ out) {
  for (int c = threadIdx.x; c < N; c += TPB) {
    double v = 0.0;
    for (int b = 0; b < nblk; ++b) v = fmax(v, partial[(int64_t)b * N + c]);
    out[c] = v > 0.0 ? v : 1.0;
  }
}

// Row (i N + c): [V_eff (clipped to +-50), phi/s, D^-1 (b - A phi)/s, d1/10, d2/10, d3/10].
__global__ void __launch_bounds__(TPB) k_features(int64_t n, int N, const int32_t* __restrict__ d2v,
                                                  const double* __restrict__ xyz, const double* __restrict__ w,
                                                  const double* __restrict__ Phi, const double* __restrict__ AX,
                                                  const double* __restrict__ B, const double* __restrict__ dinv,
                                                  const double* __restrict__ occ, const double* __restrict__ RZ,
                                                  int n_nuclei, int pot, double rc, double omega, int xck,
                                                  double xalpha, double diag, const double* __restrict__ scale,
                                                  float* __restrict__ F) {
  int64_t q = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (q >= n * N) return;
  int64_t i = q / N;
  int c = (int)(q - i * N);
  int v = d2v[i];
  double x = xyz[3 * v], y = xyz[3 * v + 1], z = xyz[3 * v + 2];
  double rho = 0.0;
  for (int k = 0; k < N; ++k) rho += occ[k] * Phi[i * N + k] * Phi[i * N + k];
  double eps = 0.0, vxc = 0.0;
  xc_point(xck, xalpha, rho, &eps, &vxc);
  double ve = vext_point(x, y, z, n_nuclei, RZ, pot, rc, omega) + w[v] + vxc;
  ve = fmin(50.0, fmax(-50.0, ve));
  double d1 = diag, d2 = diag, d3 = diag;
  if (pot != 2) {
    for (int k = 0; k < n_nuclei; ++k) {
      double dx = x - RZ[4 * k], dy = y - RZ[4 * k + 1], dz = z - RZ[4 * k + 2];
      double r = sqrt(dx * dx + dy * dy + dz * dz);
      if (r < d1) {
        d3 = d2;
        d2 = d1;
        d1 = r;
      } else if (r < d2) {
        d3 = d2;
        d2 = r;
      } else if (r < d3) {
        d3 = r;
      }
    }
  }
  double sc = scale[c];
  float* f = F + q * 6;
  f[0] = (float)ve;
  f[1] = (float)(Phi[q] / sc);
  f[2] = (float)(dinv[i] * (B[q] - AX[q]) / sc);
  f[3] = (float)(d1 / 10.0);
  f[4] = (float)(d2 / 10.0);
  f[5] = (float)(d3 / 10.0);
}

// delta = s * y (the network's correction direction).
__global__ void __launch_bounds__(TPB) k_guess_delta(int64_t total, int N, const double* __restrict__ scale,
                                                     const float* __restrict__ Y, double* __restrict__ D) {
  int64_t q = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (q >= total) return;
  D[q] = scale[q % N] * (double)Y[q];
}

// Per-block column sums of [phi.A phi, phi.A delta, delta.A delta, b.phi, b.delta].
__global__ void __launch_bounds__(TPB) k_guess_dots(int64_t n, int N, int R, const double* __restrict__ Phi,
                                                    const double* __restrict__ D, const double* __restrict__ AP,
                                                    const double* __restrict__ AD, const double* __restrict__ B,
                                                    double* __restrict__ partial) {
  __shared__ double sd[TPB];
  int t = threadIdx.x;
  int rl = t / N, c = t - rl * N;
  int64_t r = (int64_t)blockIdx.x * R + rl;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (rl < R && r < n) {
    int64_t q = r * N + c;
    v[0] = Phi[q] * AP[q];
    v[1] = Phi[q] * AD[q];
    v[2] = D[q] * AD[q];
    v[3] = B[q] * Phi[q];
    v[4] = B[q] * D[q];
  }
  for (int k = 0; k < 5; ++k) {
    __syncthreads();
    sd[t] = v[k];
    block_reduce_cols(sd, R, N);
    if (t < N) partial[(int64_t)blockIdx.x * 5 * N + k * N + t] = sd[t];
  }
}

// Minimiser of J(x) = 1/2 x.Ax - b.x over span{phi, delta} for column c
// from the five sums g = [phi.A phi, phi.A delta, delta.A delta, b.phi,
// b.delta]; (1, 0) where the 2 x 2 system is singular or J does not drop.
__device__ __forceinline__ bool galerkin_coef(const double* g, int N, int c, double* a, double* b) {
  double g00 = g[c], g01 = g[N + c], g11 = g[2 * N + c], r0 = g[3 * N + c], r1 = g[4 * N + c];
  double det = g00 * g11 - g01 * g01;
  *a = 1.0;
  *b = 0.0;
  if (!(det > 1e-12 * g00 * g11)) return false;
  double aa = (r0 * g11 - r1 * g01) / det, bb = (g00 * r1 - g01 * r0) / det;
  double jphi = 0.5 * g00 - r0;
  double jnew = 0.5 * (aa * aa * g00 + 2.0 * aa * bb * g01 + bb * bb * g11) - (aa * r0 + bb * r1);
  if (!(jnew < jphi)) return false;
  *a = aa;
  *b = bb;
  return true;
}

// Per-block column sums of |b - A x0|^2 (x0 the span minimiser, phi where it
// is not defined) and |b - A phi|^2 (A x0 = a A phi + b A delta).
__global__ void __launch_bounds__(TPB) k_guess_resid(int64_t n, int N, int R, const double* __restrict__ AP,
                                                     const double* __restrict__ AD, const double* __restrict__ B,
                                                     const double* __restrict__ g, double* __restrict__ partial) {
  __shared__ double sd[TPB];
  int t = threadIdx.x;
  int rl = t / N, c = t - rl * N;
  int64_t r = (int64_t)blockIdx.x * R + rl;
  double v[2] = {0.0, 0.0};
  if (rl < R && r < n) {
    double a, b;
    galerkin_coef(g, N, c, &a, &b);
    int64_t q = r * N + c;
    double el = B[q] - (a * AP[q] + b * AD[q]);
    double ep = B[q] - AP[q];
    v[0] = el * el;
    v[1] = ep * ep;
  }
  for (int k = 0; k < 2; ++k) {
    __syncthreads();
    sd[t] = v[k];
    block_reduce_cols(sd, R, N);
    if (t < N) partial[(int64_t)blockIdx.x * 2 * N + k * N + t] = sd[t];
  }
}

// X = a phi + b delta per column where the span minimiser is defined, lowers J
// and its residual does not exceed phi's; X = phi elsewhere (X holds delta on
// entry). sel: [used (N), |b - A x0|^2 (N), |b - A phi|^2 (N), |b - A X|^2 of
// the start taken (N)]; the middle two are read, block 0 writes the others.
__global__ void __launch_bounds__(TPB) k_guess_apply(int64_t n, int N, int R, const double* __restrict__ Phi,
                                                     const double* __restrict__ g, double* __restrict__ sel,
                                                     double* __restrict__ X) {
  int t = threadIdx.x;
  int rl = t / N, c = t - rl * N;
  if (rl >= R) return;
  double a, b;
  const bool ok = galerkin_coef(g, N, c, &a, &b) && sel[N + c] <= sel[2 * N + c];
  if (blockIdx.x == 0 && rl == 0) {
    sel[c] = ok ? 1.0 : 0.0;
    sel[3 * N + c] = ok ? sel[N + c] : sel[2 * N + c];
  }
  for (int64_t r = (int64_t)blockIdx.x * R + rl; r < n; r += (int64_t)gridDim.x * R) {
    int64_t q = r * N + c;
    X[q] = ok ? a * Phi[q] + b * X[q] : Phi[q];
  }
}

// eta^2 of each fine tet for the residual estimator of the adaptive loop:
// h_T^2 sum_i sum_q |T|/4 ((V_eff(q) - lambda_i) phi_i(q))^2 plus, for each
// face a (opposite vertex a) with a tet t' on its other side,
// h_e |e| sum_i J_i^2 with J_i = 1/2 (grad phi_i|t - grad phi_i|t') . nu,
// nu = -grad lambda_a / |grad lambda_a| the outward normal, |e| = 3 |t|
// |grad lambda_a|, h_e the face's longest edge. One thread per tet, the
// orbitals in a loop; written at the caller's index of the tet.
__global__ void __launch_bounds__(TPB) k_estimate(int64_t nt, int N, const int32_t* __restrict__ tets,
                                                  const int32_t* __restrict__ v2d, const double* __restrict__ Phi,
                                                  const double* __restrict__ lam, const double* __restrict__ veff,
                                                  const double* __restrict__ geo, const double* __restrict__ xyz,
                                                  const int32_t* __restrict__ nbr, const int32_t* __restrict__ tord,
                                                  double* __restrict__ eta2) {
  const int64_t t = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (t >= nt) return;
  int vt[4], dof[4];
  double x[4][3];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    vt[a] = tets[4 * t + a];
    dof[a] = v2d[vt[a]];
#pragma unroll
    for (int k = 0; k < 3; ++k) x[a][k] = xyz[3 * (int64_t)vt[a] + k];
  }
  const double* G = geo + 16 * t;
  const double vol = G[0];
  double h2 = 0.0;
  for (int a = 0; a < 4; ++a)
    for (int b = a + 1; b < 4; ++b) {
      double e2 = 0.0;
#pragma unroll
      for (int k = 0; k < 3; ++k) e2 += (x[a][k] - x[b][k]) * (x[a][k] - x[b][k]);
      h2 = fmax(h2, e2);
    }
  // faces: outward normal, h_e |e| (0 on the boundary), the neighbour's DoFs and gradients
  double nu[4][3], wf[4];
  int64_t tn[4];
  for (int a = 0; a < 4; ++a) {
    const int32_t o = nbr[4 * t + a];
    tn[a] = o;
    const double g0 = G[1 + 3 * a], g1 = G[2 + 3 * a], g2 = G[3 + 3 * a];
    const double gn = sqrt(g0 * g0 + g1 * g1 + g2 * g2);
    nu[a][0] = -g0 / gn;
    nu[a][1] = -g1 / gn;
    nu[a][2] = -g2 / gn;
    double he2 = 0.0;
    for (int b = 0; b < 4; ++b)
      for (int c = b + 1; c < 4; ++c) {
        if (b == a || c == a) continue;
        double e2 = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) e2 += (x[b][k] - x[c][k]) * (x[b][k] - x[c][k]);
        he2 = fmax(he2, e2);
      }
    wf[a] = o >= 0 ? sqrt(he2) * 3.0 * vol * gn : 0.0;
  }
  double elem = 0.0, face = 0.0;
  for (int i = 0; i < N; ++i) {
    double u[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) u[a] = dof[a] >= 0 ? Phi[(int64_t)dof[a] * N + i] : 0.0;
    const double us = u[0] + u[1] + u[2] + u[3];
    const double li = lam[i];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double r = (veff[4 * t + q] - li) * (QB * us + (QA - QB) * u[q]);
      elem += 0.25 * vol * r * r;
    }
    double g[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int k = 0; k < 3; ++k) g[k] += u[a] * G[1 + 3 * a + k];
    for (int a = 0; a < 4; ++a) {
      if (tn[a] < 0) continue;
      const int64_t o = tn[a];
      const double* Go = geo + 16 * o;
      double go[3] = {0.0, 0.0, 0.0};
      for (int b = 0; b < 4; ++b) {
        const int db = v2d[tets[4 * o + b]];
        const double ub = db >= 0 ? Phi[(int64_t)db * N + i] : 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) go[k] += ub * Go[1 + 3 * b + k];
      }
      const double J = 0.5 * ((g[0] - go[0]) * nu[a][0] + (g[1] - go[1]) * nu[a][1] + (g[2] - go[2]) * nu[a][2]);
      face += wf[a] * J * J;
    }
  }
  eta2[tord[t]] = h2 * elem + face;
}

// Nodal values of the vertices one bisection batch created: the mean of the
// two ends of each one's edge (rows of ncols values).
__global__ void __launch_bounds__(TPB) k_transfer(int64_t m, int64_t first, int64_t nv_old,
                                                  const int64_t* __restrict__ parents, int ncols,
                                                  double* __restrict__ values) {
  const int64_t id = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (id >= m * ncols) return;
  const int64_t j = first + id / ncols;
  const int c = (int)(id - (id / ncols) * ncols);
  const int64_t lo = parents[2 * j], hi = parents[2 * j + 1];
  values[(nv_old + j) * ncols + c] = 0.5 * (values[lo * ncols + c] + values[hi * ncols + c]);
}

// Sample rows of every stride-th DoF: features and (u - phi)/s.
__global__ void __launch_bounds__(TPB) k_collect(int64_t n, int N, int stride, const float* __restrict__ F,
                                                 const double* __restrict__ U, const double* __restrict__ Phi,
                                                 const double* __restrict__ scale, int64_t offset, int64_t cap,
                                                 float* __restrict__ ox, float* __restrict__ ot) {
  int64_t k = (int64_t)blockIdx.x * TPB + threadIdx.x;  // sample index over (selected DoF, column)
  int64_t nsel = (n + stride - 1) / stride;
  if (k >= nsel * N) return;
  int64_t is = k / N;
  int c = (int)(k - is * N);
  int64_t i = is * stride;
  int64_t row = offset + k;
  if (row >= cap) return;
  int64_t q = i * N + c;
  for (int a = 0; a < 6; ++a) ox[row * 6 + a] = F[q * 6 + a];
  ot[row] = (float)((U[q] - Phi[q]) / scale[c]);
}

}  // namespace

// ============================================================================
// Launchers
int spmm_rows_per_block(int N) { return TPB / N; }
int elem_blocks(int64_t n, int N) { return (int)((n + spmm_rows_per_block(N) - 1) / spmm_rows_per_block(N)); }
int qp_blocks(int64_t nt) { return (int)nb(nt); }
int gram_blocks(int64_t n) { return (int)((n + GRAM_ROWS - 1) / GRAM_ROWS); }

void launch_vext(hipStream_t s, int64_t npts, const double* qpx, const double* RZ, int n_nuclei, int kind,
                 double rc, double omega, double* vext) {
  hipLaunchKernelGGL(k_vext, dim3(nb(npts)), dim3(TPB), 0, s, npts, qpx, n_nuclei, RZ, kind, rc, omega, vext);
}
void launch_qp_density(hipStream_t s, int64_t nt, const int32_t* tets, const int32_t* v2d, const double* X, int N,
                       const double* occ, double* rho_out) {
  hipLaunchKernelGGL(k_qp_density, dim3(nb(nt)), dim3(TPB), 0, s, nt, tets, v2d, X, N, occ, rho_out);
}
void launch_qp_fields(hipStream_t s, int64_t nt, const int32_t* tets, const int32_t* v2d, const double* Phi, int N,
                      const double* occ, const double* wnod, const double* vext, const double* geo,
                      const double* qpx, int xck, double xalpha, double* vxc, double* exc, double* veff,
                      double* rho, double* partials) {
  hipLaunchKernelGGL(k_qp_fields, dim3(nb(nt)), dim3(TPB), 0, s, nt, tets, v2d, Phi, N, occ, wnod, vext, geo, qpx,
                     xck, xalpha, vxc, exc, veff, rho, partials);
}
int nmom() { return NMOM; }
void launch_reduce_rows(hipStream_t s, const double* partials, int nblk, int nvals, int minlast, double* out) {
  hipLaunchKernelGGL(k_reduce_rows, dim3(1), dim3(TPB), 0, s, partials, nblk, nvals, minlast, out);
}
void launch_boundary_g(hipStream_t s, int64_t nbv, const int32_t* bverts, const double* xyz, const double* mom,
                       double* g) {
  if (nbv == 0) return;
  hipLaunchKernelGGL(k_boundary_g, dim3(nb(nbv)), dim3(TPB), 0, s, nbv, bverts, xyz, mom, g);
}
void launch_field(hipStream_t s, int64_t nt, const int32_t* tets, const double* nod, const int32_t* v2d,
                  const double* dofv, const double* add1, const double* add2, double* out) {
  hipLaunchKernelGGL(k_field, dim3(nb(nt)), dim3(TPB), 0, s, nt, tets, nod, v2d, dofv, add1, add2, out);
}
void launch_assemble2(hipStream_t s, int64_t nt, int64_t n, int64_t nnz, const double* geo, const int32_t* slot_ptr,
                      const int32_t* slot_of, int64_t ns, const int32_t* diag_slot, double* esl, double cK1,
                      const double* f1, double cM1, double* val1, double* dinv1, double cK2, const double* f2,
                      double* val2) {
  (void)ns;
  if (val2) {
    hipLaunchKernelGGL(k_elem<true>, dim3(nb(nt)), dim3(TPB), 0, s, nt, geo, cK1, f1, cM1, cK2, f2, slot_of, esl);
    hipLaunchKernelGGL(k_slot_sum<true>, dim3(nb(nnz)), dim3(TPB), 0, s, nnz, slot_ptr, esl, val1, val2);
  } else {
    hipLaunchKernelGGL(k_elem<false>, dim3(nb(nt)), dim3(TPB), 0, s, nt, geo, cK1, f1, cM1, cK2, f2, slot_of, esl);
    hipLaunchKernelGGL(k_slot_sum<false>, dim3(nb(nnz)), dim3(TPB), 0, s, nnz, slot_ptr, esl, val1, nullptr);
  }
  if (dinv1) hipLaunchKernelGGL(k_diag_inv, dim3(nb(n)), dim3(TPB), 0, s, n, diag_slot, val1, dinv1);
}
void launch_load(hipStream_t s, int64_t n, int64_t nt, const int32_t* adj_ptr, const int32_t* adj_tet,
                 const int8_t* adj_loc, const int32_t* tets, const double* geo, const double* f_qp, double scale,
                 const double* gnod, const int32_t* v2d, double* scratch, double* b, double* lvec) {
  hipLaunchKernelGGL(k_load_elem, dim3(nb(nt)), dim3(TPB), 0, s, nt, tets, geo, f_qp, scale, gnod, v2d, scratch);
  launch_load_gather(s, n, 4, adj_ptr, adj_tet, adj_loc, scratch, b, lvec);
}
void launch_load_gather(hipStream_t s, int64_t n, int ne, const int32_t* adj_ptr, const int32_t* adj_tet,
                        const int8_t* adj_loc, const double* scratch, double* b, double* lvec) {
  hipLaunchKernelGGL(k_load_gather, dim3(nb(n)), dim3(TPB), 0, s, n, ne, adj_ptr, adj_tet, adj_loc, scratch, b, lvec);
}
void launch_slot_sum(hipStream_t s, int64_t nnz, const int32_t* slot_ptr, const double* esl, double* val1,
                     double* val2) {
  if (val2)
    hipLaunchKernelGGL(k_slot_sum<true>, dim3(nb(nnz)), dim3(TPB), 0, s, nnz, slot_ptr, esl, val1, val2);
  else
    hipLaunchKernelGGL(k_slot_sum<false>, dim3(nb(nnz)), dim3(TPB), 0, s, nnz, slot_ptr, esl, val1, nullptr);
}
void launch_diag_inv(hipStream_t s, int64_t n, const int32_t* diag_slot, const double* val, double* dinv) {
  hipLaunchKernelGGL(k_diag_inv, dim3(nb(n)), dim3(TPB), 0, s, n, diag_slot, val, dinv);
}
void launch_scale_cols_to(hipStream_t s, int64_t n, int N, const double* X, const double* sc, double* Y) {
  hipLaunchKernelGGL(k_scale_cols_to, dim3(nb(n * N)), dim3(TPB), 0, s, n * N, N, X, sc, Y);
}
void launch_coldot(hipStream_t s, int64_t n, int N, const double* X, const double* Y, double* partial) {
  int R = spmm_rows_per_block(N);
  hipLaunchKernelGGL(k_coldot, dim3(elem_blocks(n, N)), dim3(TPB), 0, s, n, N, R, X, Y, partial);
}
void launch_reduce_cols(hipStream_t s, int N, int nblk, const double* partial, double* out) {
  hipLaunchKernelGGL(k_reduce_cols, dim3(N), dim3(TPB), 0, s, N, nblk, partial, out);
}
void launch_lanczos_lmax(hipStream_t s, int64_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                         const double* dinv, int m, double safety, double* work, double* partial, double* scal,
                         double* lmax) {
  if (m < 2 || n < 2) return;
  const int g = (int)std::min<int64_t>(LZ_BLOCKS, std::max<int64_t>(1, (n + TPB - 1) / TPB));
  double *v = work, *vprev = work + n, *w = work + 2 * n;
  double *alpha = scal, *beta2 = scal + m + 1;  // beta2[j]: squared norm after step j - 1 (beta2[0] unused)
  hipLaunchKernelGGL(k_lz_init, dim3(g), dim3(TPB), 0, s, n, dinv, v, partial);
  hipLaunchKernelGGL(k_reduce_cols, dim3(1), dim3(TPB), 0, s, 1, g, partial, beta2);
  hipLaunchKernelGGL(k_lz_scale, dim3(g), dim3(TPB), 0, s, n, beta2, v);
  for (int j = 0; j < m; ++j) {
    launch_spmm2(s, n, 1, rowptr, col, val, v, w, nullptr, nullptr);
    hipLaunchKernelGGL(k_lz_alpha, dim3(g), dim3(TPB), 0, s, n, dinv, w, v, vprev, j > 0 ? beta2 + j : nullptr, w,
                       partial);
    hipLaunchKernelGGL(k_reduce_cols, dim3(1), dim3(TPB), 0, s, 1, g, partial, alpha + j);
    hipLaunchKernelGGL(k_lz_orth, dim3(g), dim3(TPB), 0, s, n, dinv, alpha + j, v, w, partial);
    hipLaunchKernelGGL(k_reduce_cols, dim3(1), dim3(TPB), 0, s, 1, g, partial, beta2 + j + 1);
    if (j + 1 < m) hipLaunchKernelGGL(k_lz_next, dim3(g), dim3(TPB), 0, s, n, beta2 + j + 1, w, v, vprev);
  }
  hipLaunchKernelGGL(k_lz_eig, dim3(1), dim3(64), 0, s, m, alpha, beta2, safety, lmax);
}
void launch_normalize_cols(hipStream_t s, int64_t n, int N, const double* sc, double* X) {
  hipLaunchKernelGGL(k_normalize_cols, dim3(nb(n * N)), dim3(TPB), 0, s, n * N, N, sc, X);
}
void launch_restrict_chunks(hipStream_t s, int64_t n, int64_t nH, int N, const Dev& d, const double* Y,
                            double* out, double* part) {
  const int64_t nch = (n + RESTRICT_CHUNK - 1) / RESTRICT_CHUNK;
  if (!part) part = d.rpart;
  const dim3 gs((unsigned)((nH + TPB / 64 - 1) / (TPB / 64)));
  if (N == 1) {
    if (nch > 0)
      hipLaunchKernelGGL(k_restrict_chunks1, dim3((unsigned)nch), dim3(TPB), 0, s, n, d.rch_seg, d.rseg_ptr,
                         d.rent_row, d.rent_w, Y, part);
    if (nH > 0) hipLaunchKernelGGL(k_restrict_sum1, gs, dim3(TPB), 0, s, nH, d.kseg_ptr, d.kseg, part, out);
    return;
  }
  if (nch > 0)
    hipLaunchKernelGGL(k_restrict_chunks, dim3((unsigned)nch), dim3(TPB), 0, s, n, N, d.rch_seg, d.rseg_ptr,
                       d.rent_row, d.rent_w, Y, part);
  if (nH > 0)
    hipLaunchKernelGGL(k_restrict_sum, gs, dim3(TPB), 0, s, nH, N, d.kseg_ptr, d.kseg, part, out);
}
void launch_gram(hipStream_t s, int64_t n, int N, const double* U, const double* Y, double* partial) {
  const dim3 g(gram_blocks(n)), b(TPB);
  if (N <= 16)
    hipLaunchKernelGGL(k_gram_mfma, g, b, 0, s, n, N, U, Y, partial);
  else if (N <= 32)
    hipLaunchKernelGGL(k_gram_mfma_tiles<2>, g, dim3(128), 0, s, n, N, U, Y, partial);
  else if (N <= 48)
    hipLaunchKernelGGL(k_gram_mfma_tiles<3>, g, dim3(192), 0, s, n, N, U, Y, partial);
  else if (N <= 64)
    hipLaunchKernelGGL(k_gram_mfma_tiles<4>, g, dim3(256), 0, s, n, N, U, Y, partial);
  else
    hipLaunchKernelGGL(k_gram_wide, g, b, 0, s, n, N, U, Y, partial);
}
void launch_coarse_hats(hipStream_t s, int64_t cnt, int64_t ng, const int32_t* grp_ptr, const int32_t* grp_tet,
                        const int32_t* tets, const double* geo, const double* xyz, const double* cgeo, double* chat) {
  hipLaunchKernelGGL(k_coarse_hats, dim3((unsigned)cnt), dim3(TPB), 0, s, cnt, ng, grp_ptr, grp_tet, tets, geo, xyz,
                     cgeo, chat);
}
void launch_coarse_ops(hipStream_t s, int64_t cnt, int64_t ng, const int32_t* grp_ptr, const int32_t* grp_tet,
                       const double* chat, const double* cgeo, const double* fA, const double* fW, double* out) {
  hipLaunchKernelGGL(k_coarse_ops, dim3((unsigned)cnt), dim3(TPB), 0, s, cnt, ng, grp_ptr, grp_tet, chat, cgeo, fA,
                     fW, out);
}
void launch_coarse_orb(hipStream_t s, int64_t cnt, int64_t ng, const int32_t* grp_ptr, const int32_t* grp_dof,
                       const double* chat, const double* U, int N, double* out) {
  hipLaunchKernelGGL(k_coarse_orb, dim3((unsigned)cnt), dim3(256), 0, s, cnt, ng, grp_ptr, grp_dof, chat, U, N,
                     out);
}
void launch_coarse_pairs(hipStream_t s, int64_t cnt, int64_t ng, const int32_t* grp_ptr, const int32_t* grp_dof,
                         const double* chat, const double* U, int N, const int32_t* pair_jl, int npair, double* out) {
  hipLaunchKernelGGL(k_coarse_pairs, dim3((unsigned)cnt), dim3(TPB), 0, s, cnt, ng, grp_ptr, grp_dof, chat, U, N,
                     pair_jl, npair, out);
}
void launch_reconstruct_joint(hipStream_t s, int64_t n, int N, const int32_t* Pk, const double* Pw, const double* Cc,
                              const double* D, const double* U, double* Phi) {
  hipLaunchKernelGGL(k_reconstruct_joint, dim3(nb(n * N)), dim3(TPB), 0, s, n, N, Pk, Pw, Cc, D, U, Phi);
}
void launch_coarse_tri(hipStream_t s, int64_t cnt, const int32_t* grp_ptr, const int32_t* grp_tet,
                       const int32_t* tets, const double* geo, const double* xyz, const double* cgeo, double* out) {
  hipLaunchKernelGGL(k_coarse_tri, dim3((unsigned)cnt), dim3(TPB), 0, s, cnt, grp_ptr, grp_tet, tets, geo, xyz, cgeo,
                     out);
}
void launch_reconstruct(hipStream_t s, int64_t n, int N, const int32_t* Pk, const double* Pw, const double* phiH,
                        const double* theta2, const double* U, double* Phi) {
  hipLaunchKernelGGL(k_reconstruct, dim3(nb(n * N)), dim3(TPB), 0, s, n, N, Pk, Pw, phiH, theta2, U, Phi);
}
void launch_hartree_nodal(hipStream_t s, int64_t nv, const int32_t* v2d, const int32_t* Pk, const double* Pw,
                          const double* wH, double theta1, const double* w0, const double* g, double* w) {
  hipLaunchKernelGGL(k_hartree_nodal, dim3(nb(nv)), dim3(TPB), 0, s, nv, v2d, Pk, Pw, wH, theta1, w0, g, w);
}
void launch_rho_nodal(hipStream_t s, int64_t nv, const int32_t* v2d, const double* Phi, int N, const double* occ,
                      double* rho) {
  hipLaunchKernelGGL(k_rho_nodal, dim3(nb(nv)), dim3(TPB), 0, s, nv, v2d, Phi, N, occ, rho);
}
void launch_permute_rows(hipStream_t s, int64_t n, int N, const int32_t* perm, const double* in, double* out,
                         int gather) {
  if (n * N == 0) return;
  hipLaunchKernelGGL(k_permute_rows, dim3(nb(n * N)), dim3(TPB), 0, s, n, N, perm, in, out, gather);
}
void launch_gather_nodal(hipStream_t s, int64_t n, const int32_t* d2v, const double* w, double* out) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_gather_nodal, dim3(nb(n)), dim3(TPB), 0, s, n, d2v, w, out);
}
void launch_count_nonfinite(hipStream_t s, int64_t na, const double* a, int64_t nb_, const double* b, int32_t* cnt) {
  (void)hipMemsetAsync(cnt, 0, sizeof(int32_t), s);
  int64_t blocks = std::min<int64_t>(nb(na + nb_), 2048);
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_count_nonfinite, dim3((unsigned)blocks), dim3(TPB), 0, s, na, a, nb_, b, cnt);
}
void launch_energy(hipStream_t s, int64_t nt, const int32_t* tets, const int32_t* v2d, const double* Phi, int N,
                   const double* occ, const double* wnod, const double* vxc_old, const double* geo, int xck,
                   double xalpha, double* partials) {
  hipLaunchKernelGGL(k_energy, dim3(nb(nt)), dim3(TPB), 0, s, nt, tets, v2d, Phi, N, occ, wnod, vxc_old, geo, xck,
                     xalpha, partials);
}

void launch_colmax_abs(hipStream_t s, int64_t n, int N, const double* X, double* partial, double* out) {
  int R = spmm_rows_per_block(N);
  int nbk = elem_blocks(n, N);
  if (nbk > 1024) nbk = 1024;
  hipLaunchKernelGGL(k_colmax_abs, dim3(nbk), dim3(TPB), 0, s, n, N, R, X, partial);
  hipLaunchKernelGGL(k_colmax_final, dim3(1), dim3(TPB), 0, s, N, nbk, partial, out);
}
void launch_features(hipStream_t s, int64_t n, int N, const int32_t* d2v, const double* xyz, const double* w,
                     const double* Phi, const double* AX, const double* B, const double* dinv, const double* occ,
                     const double* RZ, int n_nuclei, int pot, double rc, double omega, int xck, double xalpha,
                     double diag, const double* scale, float* F) {
  hipLaunchKernelGGL(k_features, dim3(nb(n * N)), dim3(TPB), 0, s, n, N, d2v, xyz, w, Phi, AX, B, dinv, occ, RZ,
                     n_nuclei, pot, rc, omega, xck, xalpha, diag, scale, F);
}
void launch_guess_delta(hipStream_t s, int64_t n, int N, const double* scale, const float* Y, double* D) {
  hipLaunchKernelGGL(k_guess_delta, dim3(nb(n * N)), dim3(TPB), 0, s, n * N, N, scale, Y, D);
}
void launch_guess_galerkin(hipStream_t s, int64_t n, int N, const double* Phi, const double* AP, const double* AD,
                           const double* B, double* X, double* partial, double* gdots, double* gsel) {
  int R = spmm_rows_per_block(N);
  int nbk = elem_blocks(n, N);
  hipLaunchKernelGGL(k_guess_dots, dim3(nbk), dim3(TPB), 0, s, n, N, R, Phi, X, AP, AD, B, partial);
  hipLaunchKernelGGL(k_reduce_cols, dim3(5 * N), dim3(TPB), 0, s, 5 * N, nbk, partial, gdots);
  hipLaunchKernelGGL(k_guess_resid, dim3(nbk), dim3(TPB), 0, s, n, N, R, AP, AD, B, gdots, partial);
  hipLaunchKernelGGL(k_reduce_cols, dim3(2 * N), dim3(TPB), 0, s, 2 * N, nbk, partial, gsel + N);
  hipLaunchKernelGGL(k_guess_apply, dim3(nbk), dim3(TPB), 0, s, n, N, R, Phi, gdots, gsel, X);
}
void launch_estimate(hipStream_t s, int64_t nt, int N, const int32_t* tets, const int32_t* v2d, const double* Phi,
                     const double* lam, const double* veff, const double* geo, const double* xyz, const int32_t* nbr,
                     const int32_t* tord, double* eta2) {
  hipLaunchKernelGGL(k_estimate, dim3(nb(nt)), dim3(TPB), 0, s, nt, N, tets, v2d, Phi, lam, veff, geo, xyz, nbr, tord,
                     eta2);
}
void launch_transfer(hipStream_t s, int64_t m, int64_t first, int64_t nv_old, const int64_t* parents, int ncols,
                     double* values) {
  if (m > 0) hipLaunchKernelGGL(k_transfer, dim3(nb(m * ncols)), dim3(TPB), 0, s, m, first, nv_old, parents, ncols, values);
}
void launch_collect(hipStream_t s, int64_t n, int N, int stride, const float* F, const double* U,
                    const double* Phi, const double* scale, int64_t offset, int64_t cap, float* out_x,
                    float* out_t) {
  int64_t nsel = (n + stride - 1) / stride;
  hipLaunchKernelGGL(k_collect, dim3(nb(nsel * N)), dim3(TPB), 0, s, n, N, stride, F, U, Phi, scale, offset, cap,
                     out_x, out_t);
}

}  // namespace mlc
