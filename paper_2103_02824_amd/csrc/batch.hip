// Batched multi-column Jacobi-PCG over many independent systems (gfx950).
//
// A batch holds K problems of different sizes n_p and column counts N_p (the
// step-5 problems of several systems, or their Hartree problems). Rows of
// every problem are cut into tiles of TR rows; one launch covers the tiles of
// all problems, a table maps tile -> problem. One CG iteration is five
// launches: SpMM (per-tile partials of p.q), alpha (one block per problem sums
// its partials in tile order), update (x, r; partials of r.Dr and r.r), beta
// (one block per problem: beta, the convergence test, the active count) and
// direction. Problems whose columns have all converged skip their tiles.
// Scalars per problem and column live on the device:
//   bs[p * 8 * NB + k * NB + c], k = RZ, RR, BB, ACT, IT, ALPHA, BETA, MASK
// and the active-column count of problem p in flags[p]; flags[K] is set on a
// breakdown (non-positive curvature on an active column, which freezes it).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "batch.h"
#include "row_gather.h"

namespace mlc {

namespace {

constexpr int BS = 256;  // threads per block for every batched kernel

__device__ __forceinline__ double wsum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Column sums over the (rl, c) layout: sd holds R x N values, row-major.
__device__ __forceinline__ void reduce_rc(double* sd, int R, int N) {
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

__device__ __forceinline__ double* sc(double* bs, int p, int NB, int k) { return bs + ((int64_t)p * 8 + k) * NB; }
__device__ __forceinline__ const double* sc(const double* bs, int p, int NB, int k) {
  return bs + ((int64_t)p * 8 + k) * NB;
}

// Chebyshev polynomial preconditioner (the same recurrence as the single-
// system solves: Y. Saad, Iterative Methods for Sparse Linear Systems,
// Algorithm 12.1, over [lmax / ratio, lmax]).
__device__ __forceinline__ double cheb_theta(double lmax, double ratio) { return 0.5 * (lmax + lmax / ratio); }
__device__ __forceinline__ void cheb_coef(double lmax, double ratio, int j, double* cd, double* cr) {
  const double b = lmax, a = lmax / ratio;
  const double theta = 0.5 * (b + a), delta = 0.5 * (b - a);
  const double s1 = theta / delta;
  double rho_prev = 1.0 / s1, rho = rho_prev;
  for (int k = 1; k <= j; ++k) {
    rho_prev = rho;
    rho = 1.0 / (2.0 * s1 - rho_prev);
  }
  *cd = rho * rho_prev;
  *cr = 2.0 * rho / delta;
}

// Rows [r0, r1) of Y = A S for NT <= 8 columns: G lanes per row, every lane
// strides the row's nonzeros by G and keeps the NT sums in registers. With
// dot: per-block column sums of S . Y into sd[0..NT).
// Nonzeros per lane and pass of the tile row gathers (row_gather).
constexpr int tile_unroll(int NT, int G) { return G >= 8 ? 2 : (NT <= 3 ? 4 : 2); }
constexpr int tile_cheb_unroll(int NT, int G) { return G >= 8 ? 1 : (NT <= 3 ? 2 : 1); }

template <int NT, int G, typename T>
__device__ void tile_spmm_small(int64_t r0, int64_t r1, const int32_t* __restrict__ rowptr,
                                const int32_t* __restrict__ col, const T* __restrict__ val, const T* __restrict__ S,
                                T* __restrict__ Y, bool dot, double* sd) {
  constexpr int RB = BS / G;
  const int sub = threadIdx.x % G;
  const int rl = threadIdx.x / G;
  double dp[NT];
#pragma unroll
  for (int c = 0; c < NT; ++c) dp[c] = 0.0;
  for (int64_t rb = r0; rb < r1; rb += RB) {
    int64_t r = rb + rl;
    T acc[NT];
#pragma unroll
    for (int c = 0; c < NT; ++c) acc[c] = T(0);
    if (r < r1) row_gather<NT, G, tile_unroll(NT, G)>(r, sub, rowptr, col, val, S, acc);
#pragma unroll
    for (int c = 0; c < NT; ++c)
#pragma unroll
      for (int off = G / 2; off > 0; off >>= 1) acc[c] += __shfl_xor(acc[c], off, G);
    if (r < r1) {
#pragma unroll
      for (int c = 0; c < NT; ++c)
        if (c % G == sub) {
          Y[r * NT + c] = acc[c];
          if (dot) dp[c] += (double)acc[c] * (double)S[r * NT + c];
        }
    }
  }
  if (!dot) return;
  __shared__ double wpart[BS / 64][8];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NT; ++c) {
    double v = wsum(dp[c]);
    if (lane == 0) wpart[wid][c] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < NT) {
    int c = threadIdx.x;
    double s = 0.0;
    for (int w = 0; w < BS / 64; ++w) s += wpart[w][c];
    sd[c] = s;
  }
  __syncthreads();
}

// Column sums over the block's BS / L row slots of dot[h][v] (column
// (g + L h) V + v) into sd[0..N).
template <int L, int V, int NCH>
__device__ __forceinline__ void tile_cols_lanes(const double (&dot)[NCH][V], int N, double* sd) {
  __shared__ double cs[MLC_MAX_ORBITALS];
  const int g = threadIdx.x % L, rl = threadIdx.x / L;
#pragma unroll
  for (int h = 0; h < NCH; ++h)
#pragma unroll
    for (int v = 0; v < V; ++v) {
      __syncthreads();
      sd[threadIdx.x] = dot[h][v];
      for (int m = BS / L / 2; m > 0; m >>= 1) {
        __syncthreads();
        if (rl < m) sd[threadIdx.x] += sd[threadIdx.x + m * L];
      }
      __syncthreads();
      const int c = (g + L * h) * V + v;
      if (rl == 0 && c < N) cs[c] = sd[g];
    }
  __syncthreads();
  if ((int)threadIdx.x < N) sd[threadIdx.x] = cs[threadIdx.x];
  __syncthreads();
}

// Rows [r0, r1) of Y = A S for N > 8 in the layout of wide_shape(N,
// tile_vmax<T>): V columns per lane, L lanes per row, BS / L rows per pass,
// tile_wu<T> entries per chunk with their gathers issued together (the
// batched kernels hold every system's path, so they keep the register budget
// of the small-N tiles: one column per lane; two FP32 columns per lane made
// the compiler spill the batched Chebyshev kernel). With dot: column sums into
// sd[0..N).
template <typename T>
constexpr int tile_wu() { return sizeof(T) == 8 ? 4 : 8; }
template <typename T>
constexpr int tile_vmax() { return 1; }
template <int L, int V, int NCH, typename T>
__device__ void tile_spmm_lanes(int64_t r0, int64_t r1, int N, const int32_t* __restrict__ rowptr,
                                const int32_t* __restrict__ col, const T* __restrict__ val, const T* __restrict__ S,
                                T* __restrict__ Y, bool dot, double* sd) {
  constexpr int RB = BS / L;
  const int g = threadIdx.x % L, rl = threadIdx.x / L;
  double dp[NCH][V];
#pragma unroll
  for (int h = 0; h < NCH; ++h)
#pragma unroll
    for (int v = 0; v < V; ++v) dp[h][v] = 0.0;
  for (int64_t rb = r0; rb < r1; rb += RB) {
    const int64_t r = rb + rl;
    if (r >= r1) continue;
    T acc[NCH][V];
    row_gather_lanes<L, V, NCH, tile_wu<T>(), false, T>(r, g, N, rowptr[r], rowptr[r + 1], col, val, S, acc);
#pragma unroll
    for (int h = 0; h < NCH; ++h) {
      const int c = (g + L * h) * V;
      if (c < N) {
        const int64_t i = r * N + c;
        store_cols<T, V>(Y + i, acc[h]);
        if (dot) {
          T so[V];
          load_cols<T, V>(S + i, so);
#pragma unroll
          for (int v = 0; v < V; ++v) dp[h][v] += (double)acc[h][v] * (double)so[v];
        }
      }
    }
  }
  if (dot) tile_cols_lanes<L, V, NCH>(dp, N, sd);
}

// Calls f(tag) with the layout of wide_shape(N, tile_vmax<T>()) for N > 8.
template <typename T, typename F>
__device__ __forceinline__ void lanes_dispatch(int N, F&& f) {
  const WideShape w = wide_shape(N, tile_vmax<T>());
  if (w.NCH > 1) {
    f(WideTag<64, 1, 2>{});
    return;
  }
#define TILE_L(V)                             \
  switch (w.L) {                              \
    case 4: f(WideTag<4, V, 1>{}); break;     \
    case 8: f(WideTag<8, V, 1>{}); break;     \
    case 16: f(WideTag<16, V, 1>{}); break;   \
    case 32: f(WideTag<32, V, 1>{}); break;   \
    default: f(WideTag<64, V, 1>{});          \
  }
  if constexpr (tile_vmax<T>() >= 2) {
    if (w.V == 2) {
      TILE_L(2)
      return;
    }
  }
  TILE_L(1)
#undef TILE_L
}

// One Chebyshev step over rows [r0, r1): w = A Zin; d = cd d + cr D^-1 (R - w);
// Zout = Zin + d; with dot, column sums of R . Zout into sd[0..N).
template <int NT, int G, typename T>
__device__ void tile_cheb_small(int64_t r0, int64_t r1, const BProb<T>& D, const T* __restrict__ Zin,
                                T* __restrict__ Zout, T cd, T cr, bool dot, double* sd) {
  constexpr int RB = BS / G;
  const int sub = threadIdx.x % G;
  const int rl = threadIdx.x / G;
  double dp[NT];
#pragma unroll
  for (int c = 0; c < NT; ++c) dp[c] = 0.0;
  for (int64_t rb = r0; rb < r1; rb += RB) {
    int64_t r = rb + rl;
    T acc[NT];
#pragma unroll
    for (int c = 0; c < NT; ++c) acc[c] = T(0);
    if (r < r1) row_gather<NT, G, tile_cheb_unroll(NT, G)>(r, sub, D.rowptr, D.col, D.val, Zin, acc);
#pragma unroll
    for (int c = 0; c < NT; ++c)
#pragma unroll
      for (int off = G / 2; off > 0; off >>= 1) acc[c] += __shfl_xor(acc[c], off, G);
    if (r < r1) {
      const T di = D.dinv[r];
#pragma unroll
      for (int c = 0; c < NT; ++c)
        if (c % G == sub) {
          const int64_t i = r * NT + c;
          const T rv = D.R[i];
          const T dn = cd * D.Dd[i] + cr * (di * (rv - acc[c]));
          D.Dd[i] = dn;
          const T z = Zin[i] + dn;
          Zout[i] = z;
          if (dot) dp[c] += (double)rv * (double)z;
        }
    }
  }
  if (!dot) return;
  __shared__ double wpart[BS / 64][8];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NT; ++c) {
    double v = wsum(dp[c]);
    if (lane == 0) wpart[wid][c] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < NT) {
    int c = threadIdx.x;
    double s = 0.0;
    for (int w = 0; w < BS / 64; ++w) s += wpart[w][c];
    sd[c] = s;
  }
  __syncthreads();
}

// The Chebyshev step over rows [r0, r1) for N > 8 in the same layout.
template <int L, int V, int NCH, typename T>
__device__ void tile_cheb_lanes(int64_t r0, int64_t r1, const BProb<T>& D, const T* __restrict__ Zin,
                                T* __restrict__ Zout, T cd, T cr, bool dot, double* sd) {
  constexpr int RB = BS / L;
  const int N = D.N;
  const int g = threadIdx.x % L, rl = threadIdx.x / L;
  double dp[NCH][V];
#pragma unroll
  for (int h = 0; h < NCH; ++h)
#pragma unroll
    for (int v = 0; v < V; ++v) dp[h][v] = 0.0;
  for (int64_t rb = r0; rb < r1; rb += RB) {
    const int64_t r = rb + rl;
    if (r >= r1) continue;
    T rv[NCH][V], dv[NCH][V], zv[NCH][V];
    const T di = D.dinv[r];
#pragma unroll
    for (int h = 0; h < NCH; ++h) {
      const int c = (g + L * h) * V;
      if (c < N) {
        const int64_t i = r * N + c;
        load_cols<T, V>(D.R + i, rv[h]);
        load_cols<T, V>(D.Dd + i, dv[h]);
        load_cols<T, V>(Zin + i, zv[h]);
      }
    }
    T acc[NCH][V];
    row_gather_lanes<L, V, NCH, tile_wu<T>(), false, T>(r, g, N, D.rowptr[r], D.rowptr[r + 1], D.col, D.val, Zin, acc);
#pragma unroll
    for (int h = 0; h < NCH; ++h) {
      const int c = (g + L * h) * V;
      if (c < N) {
        const int64_t i = r * N + c;
        T dn[V], z[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
          dn[v] = cd * dv[h][v] + cr * (di * (rv[h][v] - acc[h][v]));
          z[v] = zv[h][v] + dn[v];
          if (dot) dp[h][v] += (double)rv[h][v] * (double)z[v];
        }
        store_cols<T, V>(D.Dd + i, dn);
        store_cols<T, V>(Zout + i, z);
      }
    }
  }
  if (dot) tile_cols_lanes<L, V, NCH>(dp, N, sd);
}

// Chebyshev step j >= 1 over all tiles. Step j reads Z[(j-1)&1] and writes
// Z[j&1]; the last step writes P instead when to_p (start of a solve) and the
// per-tile r.z partials. In iterations (to_p false) problems without active
// columns skip their tiles.
template <int G, typename T>
__global__ void __launch_bounds__(BS) kb_cheb(const BProb<T>* __restrict__ probs, const int32_t* __restrict__ tile_prob,
                                              int TR, int NB, int j, int last, int to_p, double ratio,
                                              double* __restrict__ rz_part, const int32_t* __restrict__ flags) {
  __shared__ double sd[BS];
  const int t = blockIdx.x;
  const int p = tile_prob[t];
  if (!to_p && flags[p] == 0) return;
  const BProb<T> D = probs[p];
  const int64_t r0 = (int64_t)(t - D.tile0) * TR;
  const int64_t r1 = r0 + TR < D.n ? r0 + TR : D.n;
  double cdd, crr;
  cheb_coef(*D.lmax, ratio, j, &cdd, &crr);
  const T cd = (T)cdd, cr = (T)crr;
  const T* zin = ((j - 1) & 1) ? D.Z1 : D.Z0;
  T* zout = (last && to_p) ? D.P : ((j & 1) ? D.Z1 : D.Z0);
  const bool dot = last != 0;
  switch (D.N) {
#define CHEB(K)                                                                       \
  case K:                                                                             \
    tile_cheb_small<K, (K == 1 ? 8 : G), T>(r0, r1, D, zin, zout, cd, cr, dot, sd);   \
    break;
    CHEB(1)
    CHEB(2)
    CHEB(3)
    CHEB(4)
    CHEB(5)
    CHEB(6)
    CHEB(7)
    CHEB(8)
#undef CHEB
    default:
      lanes_dispatch<T>(D.N, [=](auto tag) {
        using K = decltype(tag);
        tile_cheb_lanes<K::L, K::V, K::NCH, T>(r0, r1, D, zin, zout, cd, cr, dot, sd);
      });
  }
  if (dot && (int)threadIdx.x < D.N) rz_part[(int64_t)t * NB + threadIdx.x] = sd[threadIdx.x];
}

// SpMM over all tiles. mode 0 (CG): Q = A P with partials of P.Q, tiles of
// problems without active columns skip; mode 1: Q = A X, no partials.
template <int G, typename T>
__global__ void __launch_bounds__(BS, 8) kb_spmm(const BProb<T>* __restrict__ probs, const int32_t* __restrict__ tile_prob,
                                              int TR, int NB, int mode, double* __restrict__ part,
                                              const int32_t* __restrict__ flags) {
  __shared__ double sd[BS];
  const int t = blockIdx.x;
  const int p = tile_prob[t];
  if (mode == 0 && flags[p] == 0) return;
  const BProb<T> D = probs[p];
  const int64_t r0 = (int64_t)(t - D.tile0) * TR;
  const int64_t r1 = r0 + TR < D.n ? r0 + TR : D.n;
  const T* S = mode == 0 ? D.P : D.X;
  const bool dot = mode == 0;
  switch (D.N) {
#define SMALL(K)                                                                            \
  case K:                                                                                   \
    tile_spmm_small<K, (K == 1 ? 8 : G), T>(r0, r1, D.rowptr, D.col, D.val, S, D.Q, dot, sd); \
    break;
    SMALL(1)
    SMALL(2)
    SMALL(3)
    SMALL(4)
    SMALL(5)
    SMALL(6)
    SMALL(7)
    SMALL(8)
#undef SMALL
    default:
      lanes_dispatch<T>(D.N, [=](auto tag) {
        using K = decltype(tag);
        tile_spmm_lanes<K::L, K::V, K::NCH, T>(r0, r1, D.N, D.rowptr, D.col, D.val, S, D.Q, dot, sd);
      });
  }
  if (dot && (int)threadIdx.x < D.N) part[(int64_t)t * NB + threadIdx.x] = sd[threadIdx.x];
}

// Sum over the tiles of problem p of nv partial values per tile (stride
// `stride` per tile), in tile order; one block; result in out[0..nv).
__device__ void sum_tiles(const double* __restrict__ part, int tile0, int ntiles, int stride, int nv, double* out) {
  constexpr int CH = 16;
  __shared__ double ws[BS / 64][CH];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int v0 = 0; v0 < nv; v0 += CH) {
    int nc = nv - v0 < CH ? nv - v0 : CH;
    double acc[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) acc[q] = 0.0;
    for (int b = threadIdx.x; b < ntiles; b += BS) {
      const double* pp = part + (int64_t)(tile0 + b) * stride + v0;
#pragma unroll
      for (int q = 0; q < CH; ++q)
        if (q < nc) acc[q] += pp[q];
    }
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      double v = wsum(acc[q]);
      if (lane == 0) ws[wid][q] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < nc) {
      int q = threadIdx.x;
      out[v0 + q] = (ws[0][q] + ws[1][q]) + (ws[2][q] + ws[3][q]);
    }
    __syncthreads();
  }
}

// One block per problem: alpha_c = rz_c / (p.q)_c on active columns.
template <typename T>
__global__ void __launch_bounds__(BS) kb_alpha(const BProb<T>* __restrict__ probs, int NB,
                                               const double* __restrict__ part, double* __restrict__ bs,
                                               int32_t* __restrict__ flags, int K) {
  const int p = blockIdx.x;
  if (flags[p] == 0) return;
  __shared__ double pq[MLC_MAX_ORBITALS];
  const BProb<T> D = probs[p];
  sum_tiles(part, D.tile0, D.ntiles, NB, D.N, pq);
  for (int c = threadIdx.x; c < D.N; c += BS) {
    double* act = sc(bs, p, NB, 3) + c;
    double a = 0.0;
    if (*act != 0.0) {
      if (pq[c] > 0.0) {
        a = sc(bs, p, NB, 0)[c] / pq[c];
      } else {
        *act = 0.0;
        flags[K] = 1;
      }
    }
    sc(bs, p, NB, 5)[c] = a;
  }
}

// Coarse-space correction of batched Hartree problems (one column each).
// Restriction rH = P^T R, one block per global coarse row.
__global__ void __launch_bounds__(BS) kb_restrict(const BProb<double>* __restrict__ probs,
                                                  const BCoarse* __restrict__ cs, const int32_t* __restrict__ crow_prob,
                                                  const int32_t* __restrict__ flags, int check) {
  __shared__ double ws[BS / 64];
  const int g = blockIdx.x;
  const int p = crow_prob[g];
  if (check && flags[p] == 0) return;
  const BCoarse C = cs[p];
  const double* R = probs[p].R;
  const int64_t k = g - C.row0;
  double acc = 0.0;
  for (int e = C.PTptr[k] + (int)threadIdx.x; e < C.PTptr[k + 1]; e += BS) acc += C.PTw[e] * R[C.PTidx[e]];
  acc = wsum(acc);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) ws[wid] = acc;
  __syncthreads();
  if (threadIdx.x == 0) C.rH[k] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

// eH = KHinv rH, one wavefront per global coarse row.
__global__ void __launch_bounds__(BS) kb_coarse_mv(const BCoarse* __restrict__ cs, const int32_t* __restrict__ crow_prob,
                                                   int64_t nrows, const int32_t* __restrict__ flags, int check) {
  const int64_t g = (int64_t)blockIdx.x * (BS / 64) + (threadIdx.x >> 6);
  if (g >= nrows) return;
  const int p = crow_prob[g];
  if (check && flags[p] == 0) return;
  const BCoarse C = cs[p];
  const int64_t k = g - C.row0;
  const int lane = threadIdx.x & 63;
  const double* a = C.KHinv + k * C.nH;
  double acc = 0.0;
  for (int64_t j = lane; j < C.nH; j += 64) acc += a[j] * C.rH[j];
  acc = wsum(acc);
  if (lane == 0) C.eH[k] = acc;
}

// z = (Zin or D^-1 R) + P eH over a tile into Zout; per-tile r.z partials.
// zsrc: 0 D^-1 R, 1 Z0, 2 Z1 (the polynomial's last block); zdst: 0 P, 1 Z0,
// 2 Z1, 3 the coarse-only buffer Zc.
__global__ void __launch_bounds__(BS) kb_zcoarse(const BProb<double>* __restrict__ probs,
                                                 const BCoarse* __restrict__ cs, const int32_t* __restrict__ tile_prob,
                                                 int TR, int NB, int zsrc, int zdst, double* __restrict__ rz_part,
                                                 const int32_t* __restrict__ flags, int check) {
  __shared__ double ws[BS / 64];
  const int t = blockIdx.x;
  const int p = tile_prob[t];
  if (check && flags[p] == 0) return;
  const BProb<double> D = probs[p];
  const BCoarse C = cs[p];
  const int64_t r0 = (int64_t)(t - D.tile0) * TR;
  const int64_t r1 = r0 + TR < D.n ? r0 + TR : D.n;
  const double* zin = zsrc == 1 ? D.Z0 : (zsrc == 2 ? D.Z1 : nullptr);
  double* zout = zdst == 0 ? D.P : (zdst == 1 ? D.Z0 : (zdst == 2 ? D.Z1 : C.Zc));
  double dot = 0.0;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += BS) {
    double z = zin ? zin[i] : D.dinv[i] * D.R[i];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = C.Pk[4 * i + j];
      if (k >= 0) z += C.Pw[4 * i + j] * C.eH[k];
    }
    zout[i] = z;
    dot += D.R[i] * z;
  }
  dot = wsum(dot);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) ws[wid] = dot;
  __syncthreads();
  if (threadIdx.x == 0) rz_part[(int64_t)t * NB] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

// The start with the polynomial: P already holds p(D^-1 A) D^-1 R; add P eH.
__global__ void __launch_bounds__(BS) kb_zcoarse_p(const BProb<double>* __restrict__ probs,
                                                   const BCoarse* __restrict__ cs, const int32_t* __restrict__ tile_prob,
                                                   int TR, int NB, double* __restrict__ rz_part) {
  __shared__ double ws[BS / 64];
  const int t = blockIdx.x;
  const int p = tile_prob[t];
  const BProb<double> D = probs[p];
  const BCoarse C = cs[p];
  const int64_t r0 = (int64_t)(t - D.tile0) * TR;
  const int64_t r1 = r0 + TR < D.n ? r0 + TR : D.n;
  double dot = 0.0;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += BS) {
    double z = D.P[i];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = C.Pk[4 * i + j];
      if (k >= 0) z += C.Pw[4 * i + j] * C.eH[k];
    }
    D.P[i] = z;
    dot += D.R[i] * z;
  }
  dot = wsum(dot);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) ws[wid] = dot;
  __syncthreads();
  if (threadIdx.x == 0) rz_part[(int64_t)t * NB] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

// X += alpha P, R -= alpha Q over a tile; partials of r.Dr and r.r.
template <typename T>
__global__ void __launch_bounds__(BS) kb_update(const BProb<T>* __restrict__ probs, const int32_t* __restrict__ tile_prob,
                                                int TR, int NB, const double* __restrict__ bs,
                                                const int32_t* __restrict__ flags, double* __restrict__ part,
                                                double ratio) {
  __shared__ double sd[BS];
  const int t = blockIdx.x;
  const int p = tile_prob[t];
  if (flags[p] == 0) return;
  const BProb<T> D = probs[p];
  const int N = D.N;
  const int64_t r0 = (int64_t)(t - D.tile0) * TR;
  const int64_t r1 = r0 + TR < D.n ? r0 + TR : D.n;
  double v0 = 0.0, v1 = 0.0;
  if (N <= BS) {
    const int R = BS / N;
    const int rl = threadIdx.x / N, c = threadIdx.x - rl * N;
    const T a = rl < R ? (T)sc(bs, p, NB, 5)[c] : T(0);
    const T ith = D.lmax ? (T)(1.0 / cheb_theta(*D.lmax, ratio)) : T(0);
    for (int64_t rb = r0; rb < r1; rb += R) {
      int64_t r = rb + rl;
      if (rl < R && r < r1) {
        int64_t i = r * N + c;
        T x = D.X[i] + a * D.P[i];
        T rr = D.R[i] - a * D.Q[i];
        D.X[i] = x;
        D.R[i] = rr;
        if (D.lmax) {
          T z = D.dinv[r] * rr * ith;
          D.Z0[i] = z;
          D.Dd[i] = z;
        }
        v0 += (double)rr * (double)D.dinv[r] * (double)rr;
        v1 += (double)rr * (double)rr;
      }
    }
    sd[threadIdx.x] = rl < R ? v0 : 0.0;
    reduce_rc(sd, R, N);
    if ((int)threadIdx.x < N) part[(int64_t)t * 3 * NB + threadIdx.x] = sd[threadIdx.x];
    __syncthreads();
    sd[threadIdx.x] = rl < R ? v1 : 0.0;
    reduce_rc(sd, R, N);
    if ((int)threadIdx.x < N) part[(int64_t)t * 3 * NB + NB + threadIdx.x] = sd[threadIdx.x];
  }
}

// One block per problem: beta, convergence ||r||^2 <= rtol^2 ||b||^2, counts.
template <typename T>
__global__ void __launch_bounds__(BS) kb_beta(const BProb<T>* __restrict__ probs, int NB,
                                              const double* __restrict__ part, double* __restrict__ bs,
                                              int32_t* __restrict__ flags, double rtol2,
                                              const double* __restrict__ rz_part) {
  const int p = blockIdx.x;
  if (flags[p] == 0) return;
  __shared__ double s2[2 * MLC_MAX_ORBITALS];
  __shared__ int cnt;
  const BProb<T> D = probs[p];
  const int N = D.N;
  // the two partial sets (r.Dr, r.r) sit at offsets 0 and NB of each tile row
  if (rz_part)
    sum_tiles(rz_part, D.tile0, D.ntiles, NB, N, s2);  // r.z of the polynomial preconditioner
  else
    sum_tiles(part, D.tile0, D.ntiles, 3 * NB, N, s2);
  sum_tiles(part + NB, D.tile0, D.ntiles, 3 * NB, N, s2 + MLC_MAX_ORBITALS);
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int c = threadIdx.x; c < N; c += BS) {
    double* act = sc(bs, p, NB, 3) + c;
    bool a = *act != 0.0;
    double rzn = s2[c], rr = s2[MLC_MAX_ORBITALS + c];
    double* rz = sc(bs, p, NB, 0) + c;
    sc(bs, p, NB, 6)[c] = a ? rzn / *rz : 0.0;
    if (a) {
      *rz = rzn;
      sc(bs, p, NB, 1)[c] = rr;
      sc(bs, p, NB, 4)[c] += 1.0;
    }
    bool still = a && rr > rtol2 * sc(bs, p, NB, 2)[c];
    *act = still ? 1.0 : 0.0;
    if (still) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) flags[p] = cnt;
}

// P = Dinv R + beta P over a tile.
template <typename T>
__global__ void __launch_bounds__(BS) kb_direction(const BProb<T>* __restrict__ probs,
                                                   const int32_t* __restrict__ tile_prob, int TR, int NB,
                                                   const double* __restrict__ bs, const int32_t* __restrict__ flags,
                                                   int degree, const BCoarse* __restrict__ cs) {
  const int t = blockIdx.x;
  const int p = tile_prob[t];
  if (flags[p] == 0) return;
  __shared__ T beta[MLC_MAX_ORBITALS];
  const BProb<T> D = probs[p];
  const int N = D.N;
  for (int c = threadIdx.x; c < N; c += BS) beta[c] = (T)sc(bs, p, NB, 6)[c];
  __syncthreads();
  const int64_t r0 = (int64_t)(t - D.tile0) * TR;
  const int64_t r1 = r0 + TR < D.n ? r0 + TR : D.n;
  const T* Zl = degree >= 2 ? (((degree - 1) & 1) ? D.Z1 : D.Z0) : nullptr;
  if constexpr (std::is_same<T, double>::value) {
    if (cs && degree < 2) Zl = cs[p].Zc;  // coarse correction on top of Jacobi
  }
  // tile-local 32-bit indices (no 64-bit division per entry)
  const int m = (int)((r1 - r0) * N);
  for (int li = threadIdx.x; li < m; li += BS) {
    const int lr = li / N;
    const int c = li - lr * N;
    const int64_t r = r0 + lr, i = r0 * N + li;
    D.P[i] = (Zl ? Zl[i] : D.dinv[r] * D.R[i]) + beta[c] * D.P[i];
  }
}

// CG start over a tile: R = B - Q (Q = A X from a mode-1 SpMM), P = Dinv R;
// partials of r.Dr, r.r, b.b.
template <typename T>
__global__ void __launch_bounds__(BS) kb_init(const BProb<T>* __restrict__ probs, const int32_t* __restrict__ tile_prob,
                                              int TR, int NB, double* __restrict__ part, int poly, double ratio) {
  __shared__ double sd[BS];
  const int t = blockIdx.x;
  const int p = tile_prob[t];
  const BProb<T> D = probs[p];
  const int N = D.N;
  const int64_t r0 = (int64_t)(t - D.tile0) * TR;
  const int64_t r1 = r0 + TR < D.n ? r0 + TR : D.n;
  const int R = BS / N;
  const int rl = threadIdx.x / N, c = threadIdx.x - rl * N;
  double v[3] = {0.0, 0.0, 0.0};
  for (int64_t rb = r0; rb < r1; rb += R) {
    int64_t r = rb + rl;
    if (rl < R && r < r1) {
      int64_t i = r * N + c;
      T b = D.B[i];
      T rr = b - D.Q[i];
      T z = D.dinv[r] * rr;
      D.R[i] = rr;
      D.P[i] = z;
      if (poly && D.lmax) {
        T z0 = z * (T)(1.0 / cheb_theta(*D.lmax, ratio));
        D.Z0[i] = z0;
        D.Dd[i] = z0;
      }
      v[0] += (double)rr * (double)z;
      v[1] += (double)rr * (double)rr;
      v[2] += (double)b * (double)b;
    }
  }
  for (int k = 0; k < 3; ++k) {
    __syncthreads();
    sd[threadIdx.x] = rl < R ? v[k] : 0.0;
    reduce_rc(sd, R, N);
    if ((int)threadIdx.x < N) part[(int64_t)t * 3 * NB + k * NB + threadIdx.x] = sd[threadIdx.x];
  }
}

// One block per problem: start scalars; a column is active when
// ||r||^2 > rtol^2 ||b||^2 and, with mask_bs, when it is active there.
template <typename T>
__global__ void __launch_bounds__(BS) kb_start(const BProb<T>* __restrict__ probs, int NB,
                                               const double* __restrict__ part, double* __restrict__ bs,
                                               const double* __restrict__ mask_bs, int32_t* __restrict__ flags,
                                               double rtol2, const double* __restrict__ rz_part) {
  const int p = blockIdx.x;
  __shared__ double s3[3 * MLC_MAX_ORBITALS];
  __shared__ int cnt;
  const BProb<T> D = probs[p];
  const int N = D.N;
  for (int k = 0; k < 3; ++k)
    sum_tiles(part + k * NB, D.tile0, D.ntiles, 3 * NB, N, s3 + k * MLC_MAX_ORBITALS);
  if (rz_part) sum_tiles(rz_part, D.tile0, D.ntiles, NB, N, s3);  // r.z of the polynomial preconditioner
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int c = threadIdx.x; c < N; c += BS) {
    double rz = s3[c], rr = s3[MLC_MAX_ORBITALS + c], bb = s3[2 * MLC_MAX_ORBITALS + c];
    sc(bs, p, NB, 0)[c] = rz;
    sc(bs, p, NB, 1)[c] = rr;
    sc(bs, p, NB, 2)[c] = bb;
    sc(bs, p, NB, 4)[c] = 0.0;
    bool act = rr > rtol2 * bb;
    if (mask_bs) act = act && sc(mask_bs, p, NB, 3)[c] != 0.0;
    sc(bs, p, NB, 3)[c] = act ? 1.0 : 0.0;
    if (act) atomicAdd(&cnt, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) flags[p] = cnt;
}

// Iterative refinement helpers over a tile: op 0: B32 = R64, X32 = 0;
// op 1: X64 += X32.
__global__ void __launch_bounds__(BS) kb_ir(const BProb<double>* __restrict__ p64, const BProb<float>* __restrict__ p32,
                                            const int32_t* __restrict__ tile_prob, int TR, int op) {
  const int t = blockIdx.x;
  const int p = tile_prob[t];
  const BProb<double> D = p64[p];
  const BProb<float> F = p32[p];
  const int N = D.N;
  const int64_t r0 = (int64_t)(t - D.tile0) * TR;
  const int64_t r1 = r0 + TR < D.n ? r0 + TR : D.n;
  for (int64_t i = r0 * N + threadIdx.x; i < r1 * N; i += BS) {
    if (op == 0) {
      const_cast<float*>(F.B)[i] = (float)D.R[i];
      F.X[i] = 0.0f;
    } else {
      D.X[i] += (double)F.X[i];
    }
  }
}

}  // namespace

template <typename T>
void launch_b_spmm(hipStream_t s, const BProb<T>* probs, const int32_t* tile_prob, int ntiles, int TR, int G, int NB,
                   int mode, double* part, const int32_t* flags) {
  switch (G) {
    case 2:
      hipLaunchKernelGGL((kb_spmm<2, T>), dim3(ntiles), dim3(BS), 0, s, probs, tile_prob, TR, NB, mode, part, flags);
      break;
    case 8:
      hipLaunchKernelGGL((kb_spmm<8, T>), dim3(ntiles), dim3(BS), 0, s, probs, tile_prob, TR, NB, mode, part, flags);
      break;
    default:
      hipLaunchKernelGGL((kb_spmm<4, T>), dim3(ntiles), dim3(BS), 0, s, probs, tile_prob, TR, NB, mode, part, flags);
  }
}

template <typename T>
void launch_b_cheb(hipStream_t s, const BProb<T>* probs, const int32_t* tile_prob, int ntiles, int TR, int G, int NB,
                   const BPoly& poly, int to_p, const int32_t* flags) {
  for (int j = 1; j < poly.degree; ++j) {
    const int last = j == poly.degree - 1;
    switch (G) {
      case 2:
        hipLaunchKernelGGL((kb_cheb<2, T>), dim3(ntiles), dim3(BS), 0, s, probs, tile_prob, TR, NB, j, last, to_p,
                           poly.ratio, poly.rz_part, flags);
        break;
      case 8:
        hipLaunchKernelGGL((kb_cheb<8, T>), dim3(ntiles), dim3(BS), 0, s, probs, tile_prob, TR, NB, j, last, to_p,
                           poly.ratio, poly.rz_part, flags);
        break;
      default:
        hipLaunchKernelGGL((kb_cheb<4, T>), dim3(ntiles), dim3(BS), 0, s, probs, tile_prob, TR, NB, j, last, to_p,
                           poly.ratio, poly.rz_part, flags);
    }
  }
}

// The coarse correction after the polynomial steps (or on top of Jacobi):
// restriction, coarse solve, z += P eH with the per-tile r.z partials.
template <typename T>
void launch_b_coarse(hipStream_t s, const BProb<T>* probs, const int32_t* tile_prob, int ntiles, int TR, int NB,
                     const BPoly& poly, const BCoarseSet& cs, const int32_t* flags, bool start) {
  if constexpr (std::is_same<T, double>::value) {
    const int check = start ? 0 : 1;
    const bool pc = poly.degree >= 2;
    const int last = pc ? (((poly.degree - 1) & 1) ? 2 : 1) : 0;
    const int zsrc = start ? (pc ? 3 : 0) : last;  // at the start the polynomial wrote P
    const int zdst = start ? 0 : (pc ? last : 3);
    hipLaunchKernelGGL(kb_restrict, dim3((unsigned)cs.nrows), dim3(BS), 0, s, probs, cs.coarse, cs.crow_prob, flags,
                       check);
    hipLaunchKernelGGL(kb_coarse_mv, dim3((unsigned)((cs.nrows + 3) / 4)), dim3(BS), 0, s, cs.coarse, cs.crow_prob,
                       cs.nrows, flags, check);
    if (zsrc == 3) {
      // the polynomial's result is in P: add the correction in place
      hipLaunchKernelGGL(kb_zcoarse_p, dim3(ntiles), dim3(BS), 0, s, probs, cs.coarse, tile_prob, TR, NB, poly.rz_part);
    } else {
      hipLaunchKernelGGL(kb_zcoarse, dim3(ntiles), dim3(BS), 0, s, probs, cs.coarse, tile_prob, TR, NB, zsrc, zdst,
                         poly.rz_part, flags, check);
    }
  }
}

template <typename T>
void launch_b_iteration(hipStream_t s, const BProb<T>* probs, const int32_t* tile_prob, int ntiles, int K, int TR,
                        int G, int NB, double* part, double* bs, int32_t* flags, double rtol2, const BPoly& poly,
                        const BCoarseSet* cs) {
  const bool pc = poly.degree >= 2;
  const bool cc = cs && cs->coarse;
  launch_b_spmm<T>(s, probs, tile_prob, ntiles, TR, G, NB, 0, part, flags);
  hipLaunchKernelGGL((kb_alpha<T>), dim3(K), dim3(BS), 0, s, probs, NB, part, bs, flags, K);
  hipLaunchKernelGGL((kb_update<T>), dim3(ntiles), dim3(BS), 0, s, probs, tile_prob, TR, NB, bs, flags, part,
                     poly.ratio);
  if (pc) launch_b_cheb<T>(s, probs, tile_prob, ntiles, TR, G, NB, poly, 0, flags);
  if (cc) launch_b_coarse<T>(s, probs, tile_prob, ntiles, TR, NB, poly, *cs, flags, false);
  hipLaunchKernelGGL((kb_beta<T>), dim3(K), dim3(BS), 0, s, probs, NB, part, bs, flags, rtol2,
                     (pc || cc) ? poly.rz_part : nullptr);
  hipLaunchKernelGGL((kb_direction<T>), dim3(ntiles), dim3(BS), 0, s, probs, tile_prob, TR, NB, bs, flags,
                     pc ? poly.degree : 0, cc ? cs->coarse : nullptr);
}

template <typename T>
void launch_b_start(hipStream_t s, const BProb<T>* probs, const int32_t* tile_prob, int ntiles, int K, int TR, int G,
                    int NB, double* part, double* bs, const double* mask_bs, int32_t* flags, double rtol2,
                    const BPoly& poly, const BCoarseSet* cs) {
  const bool pc = poly.degree >= 2;
  const bool cc = cs && cs->coarse;
  launch_b_spmm<T>(s, probs, tile_prob, ntiles, TR, G, NB, 1, part, flags);
  hipLaunchKernelGGL((kb_init<T>), dim3(ntiles), dim3(BS), 0, s, probs, tile_prob, TR, NB, part, pc ? 1 : 0,
                     poly.ratio);
  if (pc) launch_b_cheb<T>(s, probs, tile_prob, ntiles, TR, G, NB, poly, 1, flags);
  if (cc) launch_b_coarse<T>(s, probs, tile_prob, ntiles, TR, NB, poly, *cs, flags, true);
  hipLaunchKernelGGL((kb_start<T>), dim3(K), dim3(BS), 0, s, probs, NB, part, bs, mask_bs, flags, rtol2,
                     (pc || cc) ? poly.rz_part : nullptr);
}

void launch_b_ir(hipStream_t s, const BProb<double>* p64, const BProb<float>* p32, const int32_t* tile_prob,
                 int ntiles, int TR, int op) {
  hipLaunchKernelGGL(kb_ir, dim3(ntiles), dim3(BS), 0, s, p64, p32, tile_prob, TR, op);
}

template void launch_b_spmm<double>(hipStream_t, const BProb<double>*, const int32_t*, int, int, int, int, int,
                                    double*, const int32_t*);
template void launch_b_spmm<float>(hipStream_t, const BProb<float>*, const int32_t*, int, int, int, int, int, double*,
                                   const int32_t*);
template void launch_b_iteration<double>(hipStream_t, const BProb<double>*, const int32_t*, int, int, int, int, int,
                                         double*, double*, int32_t*, double, const BPoly&, const BCoarseSet*);
template void launch_b_iteration<float>(hipStream_t, const BProb<float>*, const int32_t*, int, int, int, int, int,
                                        double*, double*, int32_t*, double, const BPoly&, const BCoarseSet*);
template void launch_b_start<double>(hipStream_t, const BProb<double>*, const int32_t*, int, int, int, int, int,
                                     double*, double*, const double*, int32_t*, double, const BPoly&,
                                     const BCoarseSet*);
template void launch_b_start<float>(hipStream_t, const BProb<float>*, const int32_t*, int, int, int, int, int, double*,
                                    double*, const double*, int32_t*, double, const BPoly&, const BCoarseSet*);

}  // namespace mlc
