// Multi-right-hand-side CSR SpMM and the Jacobi-PCG vector kernels (gfx950).
//
// Orbital blocks are n x N row-major (orbital fastest). Every CG recurrence is
// independent per column (the step-5 problems are independent per orbital,
// Section 3.2): alpha, beta and the convergence flag are per column and live
// on the device.
//
// One CG iteration is three kernels: SpMM q = A p (block partials of p.q),
// update (alpha from the p.q partials; x, r; partials of r.Dr and r.r) and
// direction (beta and the convergence test from those partials; p). Each
// consumer kernel sums the producer's block partials itself, every block in
// the same fixed order, so all blocks obtain bitwise identical scalars without
// a separate reduction launch; grids are capped (rows visited grid-stride) to
// keep those partial sets small. A last-arriving-block reduction would need a
// device-scope fence in every block, which on this multi-die part means an L2
// write-back per block and costs more than it saves. Scalars are double
// buffered by iteration parity so that no kernel reads a value another block
// of the same launch writes.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "mlc_internal.h"
#include "row_gather.h"

namespace mlc {

namespace {

constexpr int TPB = 256;
constexpr int MAXBLK = 1024;       // plain SpMM / init grids
constexpr int SPMM_BS = 1024;      // CG SpMM block size (16 waves per block)
// CG SpMM grid cap (number of p.q partials): 512 blocks of 16 waves fill the
// resident wave slots of the chip once; more blocks (one pass each) measured
// slower, because the blocks past the first round run on a half-empty chip.
constexpr int SPMM_MAXBLK = 512;
constexpr int VEC_MAXBLK = 512;    // update / direction grid cap
constexpr int UPD_UR = 4;          // row passes per loop trip of the V-column update / direction
constexpr int NXCD = 8;            // XCDs of the chip, each with its own L2

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// In-block column sums for the (row, column) thread layout (R rows x N cols);
// leaves column sums in sd[0..N).
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

inline int cap(int64_t needed, int mx) { return (int)(needed < mx ? (needed < 1 ? 1 : needed) : mx); }
// grids of the row-block kernels: a multiple of the XCD count (mx is one)
inline int cap_xcd(int64_t needed, int mx) { return cap((needed + NXCD - 1) / NXCD * NXCD, mx); }

// Row blocks of a grid-stride loop, XCD-aware. Workgroups are dispatched to
// the XCDs round robin (workgroup w runs on XCD w % NXCD) and each XCD has its
// own L2; XCD x takes the contiguous x-th eighth of the nrb row blocks, so
// the rows of X that its blocks gather (neighbours of neighbouring rows)
// stay in that L2. Grids that are not a multiple of NXCD stride plainly.
struct RowBlocks {
  int64_t first, step, end;
  __device__ explicit RowBlocks(int64_t nrb) {
    const int g = (int)gridDim.x;
    if (g % NXCD != 0) {
      first = blockIdx.x;
      step = g;
      end = nrb;
      return;
    }
    const int x = (int)blockIdx.x % NXCD;
    first = nrb * x / NXCD + (int64_t)blockIdx.x / NXCD;
    step = g / NXCD;
    end = nrb * (x + 1) / NXCD;
  }
};


// ---------------------------------------------------------------------------
// SpMM and fused Chebyshev step for N > 8. A lane owns V consecutive columns
// (V = 4 for FP32 and V = 2 for FP64 when N is a multiple of V: one 16-byte
// load per gathered row segment; else V = 1), L lanes share a row (L = the
// smallest power of two >= N / V, at most 64; with V = 1 and N > 64 a lane
// also owns the columns 64 further on), so a wavefront works on 64 / L rows
// at once. BS-thread blocks over XCD-aware row blocks of BS / L rows. A
// row's column indices and values are read WU at a time (the row's L lanes
// read the same addresses: one request) and the WU gathers are issued before
// they are summed, into two accumulators per column; entries past the row end
// repeat the row's last entry with weight zero, so that every chunk issues all
// its loads at once, with no branch. Blocks of n N sizeof(T) < 2^32 bytes are
// gathered through 32-bit offsets (O32).
// Launch shapes, from a standalone harness on the 40-atom matrix (2.0M rows,
// bimodal row lengths 7..27) at N = 52: the gathers are bound by the vector
// memory instructions they issue (each covers 64 / L rows; a pass of WU
// entries costs WU of them whatever the rows' lengths), so the kernels take
// WU = 8 entries per pass in FP32 (-8% against 16) and 4 in FP64 (-15%), and
// the launches without partial sums run 256-thread blocks on up to 256
// blocks per XCD. The producers of per-block partial sums (CG SpMM, last
// polynomial step) keep 512-thread blocks on a grid of at most 512, because
// every consumer block re-reads all partials.
constexpr int WIDE_BS = 512;       // partial producers
constexpr int WIDE_MAXBLK = 512;   // at most cg_max_blocks()
constexpr int WIDE_BS_PLAIN = 256;
constexpr int WIDE_MAXBLK_PLAIN = 2048;
template <typename T>
constexpr int wide_wu() { return sizeof(T) == 4 ? 8 : 4; }

// Grid of the N > 8 partial producers: one block per 64 rows up to the cap,
// whatever the layout (the FP32 and FP64 kernels and the consumers of their
// partials agree on it); blocks past the last row block write zero partials.
inline int wide_blocks_for(int64_t n) { return cap_xcd((n + 63) / 64, WIDE_MAXBLK); }
// Grid of the other N > 8 launches: one block per row block of BS / L rows up to the cap.
inline int wide_plain_blocks(int64_t n, int L) {
  const int64_t rb = WIDE_BS_PLAIN / L;
  return cap_xcd((n + rb - 1) / rb, WIDE_MAXBLK_PLAIN);
}

// Column sums of dot over the block's BS / L row slots into partial[blk, :].
template <int L, int V, int NCH, int BS>
__device__ __forceinline__ void block_cols_lanes(const double (&dot)[NCH][V], int N, double* __restrict__ partial) {
  __shared__ double sd[BS];
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
      if (rl == 0 && c < N) partial[(int64_t)blockIdx.x * N + c] = sd[g];
    }
}

// Y = A X; with partial: per-block column sums of X . Y.
template <int L, int V, int NCH, bool O32, int BS, typename T>
__global__ void __launch_bounds__(BS) k_spmm_rows(int64_t n, int N, const int32_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ col, const T* __restrict__ val,
                                                       const T* __restrict__ X, T* __restrict__ Y,
                                                       double* __restrict__ partial, const int32_t* __restrict__ flags) {
  constexpr int RB = BS / L;
  if (flags && flags[0] == 0) return;
  const int g = threadIdx.x % L, rl = threadIdx.x / L;
  double dot[NCH][V];
#pragma unroll
  for (int h = 0; h < NCH; ++h)
#pragma unroll
    for (int v = 0; v < V; ++v) dot[h][v] = 0.0;
  // the next row's pointers are loaded while this row's gathers are in
  // flight; rows past n are computed as row n - 1 and not stored (no branch
  // in the loop body)
  const RowBlocks rbk((n + RB - 1) / RB);
  int64_t rn = rbk.first * RB + rl;
  rn = rn < n ? rn : n - 1;
  int jb = rowptr[rn], je = rowptr[rn + 1];
  for (int64_t rb = rbk.first; rb < rbk.end; rb += rbk.step) {
    const int64_t r0 = rb * RB + rl;
    const bool live = r0 < n;
    const int64_t r = live ? r0 : n - 1;
    const int jr = jb, jr1 = je;
    rn = (rb + rbk.step) * RB + rl;
    rn = rn < n ? rn : n - 1;
    jb = rowptr[rn];
    je = rowptr[rn + 1];
    T acc[NCH][V];
    row_gather_lanes<L, V, NCH, wide_wu<T>(), O32, T>(r, g, N, jr, jr1, col, val, X, acc);
#pragma unroll
    for (int h = 0; h < NCH; ++h) {
      const int c = (g + L * h) * V;
      if (live && c < N) {
        const int64_t i = r * N + c;
        store_cols<T, V>(Y + i, acc[h]);
        if (partial) {
          T xo[V];
          load_cols<T, V>(X + i, xo);
#pragma unroll
          for (int v = 0; v < V; ++v) dot[h][v] += (double)acc[h][v] * (double)xo[v];
        }
      }
    }
  }
  if (partial) block_cols_lanes<L, V, NCH, BS>(dot, N, partial);
}

// ---------------------------------------------------------------------------
// Chebyshev polynomial preconditioner z = p(D^-1 A) D^-1 r: the first m steps
// of the Chebyshev iteration for A z = r from z = 0 with the Jacobi splitting,
// for eigenvalues of D^-1 A in [lmax / ratio, lmax] (Y. Saad, Iterative
// Methods for Sparse Linear Systems, 2nd ed., Algorithm 12.1):
//   theta = (b + a)/2, delta = (b - a)/2, s1 = theta/delta, rho_0 = 1/s1,
//   step 0:  d = D^-1 r / theta,  z = d
//   step j:  rho_j = 1/(2 s1 - rho_{j-1}),
//            d = rho_j rho_{j-1} d + (2 rho_j / delta) D^-1 (r - A z),  z += d.
// Its residual polynomial is positive and below one on (0, b], so p is
// positive there and p(D^-1 A) D^-1 is symmetric positive definite for CG.
// lmax is a Gershgorin bound of D^-1 A computed on the device.
// The kernels carry the iterates, not d: with z_j the iterate after step j
// (z_{-1} = 0) the previous direction is z_{j-1} - z_{j-2}, so step j reads
// r, z_{j-1} (gathered) and z_{j-2} and writes z_j over z_{j-2}: one block of
// n x N fewer read and one fewer written per step than with d stored.
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

// ---------------------------------------------------------------------------
// SpMM for small N (compile-time NT <= 8): G lanes share a row, each lane
// takes every G-th nonzero and keeps all NT column sums in registers; the G
// partial sums are combined with lane shuffles. Column indices and values are
// read coalesced (G consecutive entries), X rows as NT consecutive doubles.
// Optional CG epilogue: per-block column sums of P . Q.
template <int NT, int G, int U, int BS, int W, typename T>
__global__ void __launch_bounds__(BS, W) k_spmm_small(int64_t n, const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ col, const T* __restrict__ val,
                                                      const T* __restrict__ X, T* __restrict__ Y,
                                                      double* __restrict__ partial, const int32_t* __restrict__ flags) {
  constexpr int RB = BS / G;  // rows per block pass
  if (flags && flags[0] == 0) return;
  __shared__ double sd[BS / 64][NT];
  const int sub = threadIdx.x % G;
  const int rl = threadIdx.x / G;
  double dot[NT];
#pragma unroll
  for (int c = 0; c < NT; ++c) dot[c] = 0.0;
  // rows past n are computed as row n - 1 and not stored (no branch around
  // the gather); the next row's pointers are loaded ahead
  const RowBlocks rbk((n + RB - 1) / RB);
  int64_t rn = rbk.first * RB + rl;
  rn = rn < n ? rn : n - 1;
  int jb = rowptr[rn], je = rowptr[rn + 1];
  for (int64_t rb = rbk.first; rb < rbk.end; rb += rbk.step) {
    const int64_t r0 = rb * RB + rl;
    const int64_t r = r0 < n ? r0 : n - 1;
    const int jr = jb, jr1 = je;
    rn = (rb + rbk.step) * RB + rl;
    rn = rn < n ? rn : n - 1;
    jb = rowptr[rn];
    je = rowptr[rn + 1];
    T acc[NT];
#pragma unroll
    for (int c = 0; c < NT; ++c) acc[c] = T(0);
    row_gather<NT, G, U>(jr, jr1, sub, col, val, X, acc);
#pragma unroll
    for (int c = 0; c < NT; ++c)
#pragma unroll
      for (int off = G / 2; off > 0; off >>= 1) acc[c] += __shfl_xor(acc[c], off, G);
    if (r0 < n) {
#pragma unroll
      for (int c = 0; c < NT; ++c)
        if (c % G == sub) {
          Y[r * NT + c] = acc[c];
          if (partial) dot[c] += (double)acc[c] * (double)X[r * NT + c];
        }
    }
  }
  if (!partial) return;
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NT; ++c) {
    double v = wave_sum(dot[c]);
    if (lane == 0) sd[wid][c] = v;
  }
  __syncthreads();
  if (threadIdx.x < NT) {
    int c = threadIdx.x;
    double s = 0.0;
    for (int w = 0; w < BS / 64; ++w) s += sd[w][c];
    partial[(int64_t)blockIdx.x * NT + c] = s;
  }
}

// One Chebyshev step j >= 1 fused with its SpMM (NT <= 8, G lanes per row):
// w = A Zin; Zout = Zin + cd (Zin - Zprev) + cr D^-1 (R - w) with Zprev = 0
// for j = 1 (Zprev is not read then); optional per-block column sums of
// R . Zout (the r.z of CG after the last step). Zout may be Zprev (each
// entry is read before it is written, by the same lane; Zin is the only
// gathered block). The row's own entries of R, Zprev and Zin are loaded
// before the gather, so that their latency overlaps it. The matrix values may be a narrower copy (MT = float
// for FP64 vectors): the polynomial is then that of the rounded matrix, a
// fixed symmetric positive definite preconditioner all the same.
template <int NT, int G, int U, int BS, int W, typename T, typename MT = T>
__global__ void __launch_bounds__(BS, W) k_cheb_small(int64_t n, const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ col, const MT* __restrict__ val,
                                                      const T* __restrict__ dinv, const T* __restrict__ R,
                                                      const T* __restrict__ Zin, const T* Zprev, T* Zout,
                                                      const double* __restrict__ lmax, double ratio, int j,
                                                      double* __restrict__ partial,
                                                      const int32_t* __restrict__ flags) {
  constexpr int RB = BS / G;
  constexpr int NO = (NT + G - 1) / G;  // columns owned by a lane (c = sub + o G)
  if (flags && flags[0] == 0) return;
  __shared__ double sd[BS / 64][NT];
  double cdd, crr;
  cheb_coef(*lmax, ratio, j, &cdd, &crr);
  const T cd = (T)cdd, cr = (T)crr;
  const int sub = threadIdx.x % G;
  const int rl = threadIdx.x / G;
  double dot[NT];
#pragma unroll
  for (int c = 0; c < NT; ++c) dot[c] = 0.0;
  // rows past n are computed as row n - 1 and not stored: no branch around
  // the gather (and whole lane groups stay active for the shuffles); the next
  // row's pointers are loaded ahead
  const RowBlocks rbk((n + RB - 1) / RB);
  int64_t rn = rbk.first * RB + rl;
  rn = rn < n ? rn : n - 1;
  int jb = rowptr[rn], je = rowptr[rn + 1];
  for (int64_t rb = rbk.first; rb < rbk.end; rb += rbk.step) {
    const int64_t r0 = rb * RB + rl;
    const bool live = r0 < n;
    const int64_t r = live ? r0 : n - 1;
    const int jr = jb, jr1 = je;
    rn = (rb + rbk.step) * RB + rl;
    rn = rn < n ? rn : n - 1;
    jb = rowptr[rn];
    je = rowptr[rn + 1];
    T rv[NO], pv[NO], zv[NO];
    const T di = dinv[r];
    // the row's own entries (lanes past NT load the last column; for j = 1
    // the caller passes Zprev = Zin and the previous iterate is zero)
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      const int c = sub + o * G < NT ? sub + o * G : NT - 1;
      rv[o] = R[r * NT + c];
      zv[o] = Zin[r * NT + c];
      pv[o] = Zprev[r * NT + c];
    }
    T acc[NT];
#pragma unroll
    for (int c = 0; c < NT; ++c) acc[c] = T(0);
    row_gather<NT, G, U>(jr, jr1, sub, col, val, Zin, acc);
#pragma unroll
    for (int c = 0; c < NT; ++c)
#pragma unroll
      for (int off = G / 2; off > 0; off >>= 1) acc[c] += __shfl_xor(acc[c], off, G);
#pragma unroll
    for (int o = 0; o < NO; ++o) {
      const int c = sub + o * G;
      if (live && c < NT) {
        const T dv = j > 1 ? zv[o] - pv[o] : zv[o];
        const T z = zv[o] + (cd * dv + cr * (di * (rv[o] - acc[c])));
        Zout[r * NT + c] = z;
        if (partial) dot[c] += (double)rv[o] * (double)z;
      }
    }
  }
  if (!partial) return;
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < NT; ++c) {
    double v = wave_sum(dot[c]);
    if (lane == 0) sd[wid][c] = v;
  }
  __syncthreads();
  if (threadIdx.x < NT) {
    int c = threadIdx.x;
    double s = 0.0;
    for (int w = 0; w < BS / 64; ++w) s += sd[w][c];
    partial[(int64_t)blockIdx.x * NT + c] = s;
  }
}

// One Chebyshev step j >= 1 for a single FP64 column with FP32 matrix values
// (the Hartree problem's polynomial steps that produce no partial sums), in
// a streaming layout: a one-wavefront block owns 64 consecutive rows, one
// lane per row, and reads the rows' contiguous run of nonzeros [A, B) in
// windows of S1_WIN entries, lane t taking entries t, t + 64, ... of the
// window: every column-index and value load is one contiguous 256-byte
// request, against 16 separate rows' segments with four lanes per row. Each
// lane writes its products a_e x_{col e} to LDS, and after the barrier each
// row's lane sums the products of its own entries that fall in the window, in
// entry order. Entries past B in the last window load entry B - 1 and store a
// zero product, so every load is in bounds. Rows past n (the last block)
// own no entries and are not stored. Zout may be Zprev (each row's entry is
// read before it is written, by its own lane).
constexpr int S1_WIN = 512;
__global__ void __launch_bounds__(64, 8) k_cheb_stream1(int64_t n, const int32_t* __restrict__ rowptr,
                                                        const int32_t* __restrict__ col,
                                                        const float* __restrict__ val,
                                                        const double* __restrict__ dinv,
                                                        const double* __restrict__ R,
                                                        const double* __restrict__ Zin, const double* Zprev,
                                                        double* Zout, const double* __restrict__ lmax, double ratio,
                                                        int j, const int32_t* __restrict__ flags) {
  __shared__ double prod[S1_WIN];
  if (flags && flags[0] == 0) return;
  double cd, cr;
  cheb_coef(*lmax, ratio, j, &cd, &cr);
  const int lane = threadIdx.x;
  const RowBlocks rbk((n + 63) / 64);
  for (int64_t rb = rbk.first; rb < rbk.end; rb += rbk.step) {
    const int64_t r0 = rb * 64;
    const int64_t r = r0 + lane;
    const bool live = r < n;
    const int64_t rr = live ? r : n - 1;
    const int A = rowptr[r0];
    const int B = rowptr[r0 + 64 < n ? r0 + 64 : n];
    const int rs = live ? rowptr[rr] : B;
    const int re = live ? rowptr[rr + 1] : B;
    const double di = dinv[rr], rv = R[rr], zv = Zin[rr], pv = Zprev[rr];
    double s = 0.0;
    for (int wa = A; wa < B; wa += S1_WIN) {
      const int we = wa + S1_WIN < B ? wa + S1_WIN : B;
      int c[S1_WIN / 64];
      float a[S1_WIN / 64];
#pragma unroll
      for (int k = 0; k < S1_WIN / 64; ++k) {
        const int e = wa + lane + 64 * k;
        const int ec = e < we ? e : we - 1;
        c[k] = col[ec];
        const float av = val[ec];
        a[k] = e < we ? av : 0.0f;
      }
      double x[S1_WIN / 64];
#pragma unroll
      for (int k = 0; k < S1_WIN / 64; ++k) x[k] = Zin[c[k]];
#pragma unroll
      for (int k = 0; k < S1_WIN / 64; ++k) prod[lane + 64 * k] = (double)a[k] * x[k];
      __syncthreads();
      const int lo = (rs > wa ? rs : wa) - wa;
      const int hi = (re < we ? re : we) - wa;
      for (int t = lo; t < hi; ++t) s += prod[t];
      __syncthreads();
    }
    if (live) {
      const double dv = j > 1 ? zv - pv : zv;
      Zout[r] = zv + (cd * dv + cr * (di * (rv - s)));
    }
  }
}

// The fused Chebyshev step for N > 8 in the same layout: w = A Zin;
// Zout = Zin + cd (Zin - Zprev) + cr D^-1 (R - w) (Zprev = 0 for j = 1; Zout
// may be Zprev); with PART, per-block column sums of R . Zout into partial (a
// separate instantiation, so that the steps without them do not hold the
// sums in registers). The row's own R, Zprev, Zin entries are loaded before
// the gather.
template <int L, int V, int NCH, bool PART, bool O32, int BS, typename T>
__global__ void __launch_bounds__(BS) k_cheb_rows(int64_t n, int N, const int32_t* __restrict__ rowptr,
                                                       const int32_t* __restrict__ col, const T* __restrict__ val,
                                                       const T* __restrict__ dinv, const T* __restrict__ R,
                                                       const T* __restrict__ Zin, const T* Zprev, T* Zout,
                                                       const double* __restrict__ lmax, double ratio, int j,
                                                       double* __restrict__ partial,
                                                       const int32_t* __restrict__ flags) {
  constexpr int RB = BS / L;
  if (flags && flags[0] == 0) return;
  double cdd, crr;
  cheb_coef(*lmax, ratio, j, &cdd, &crr);
  const T cd = (T)cdd, cr = (T)crr;
  const int g = threadIdx.x % L, rl = threadIdx.x / L;
  double dot[NCH][V];
#pragma unroll
  for (int h = 0; h < NCH; ++h)
#pragma unroll
    for (int v = 0; v < V; ++v) dot[h][v] = 0.0;
  // The next row's pointers are loaded while this row's gathers are in
  // flight. Rows past n (the tail row block) are computed as row n - 1 and
  // not stored, so the loop body has no branch and its loads need no
  // conservative waits.
  const RowBlocks rbk((n + RB - 1) / RB);
  int64_t rn = rbk.first * RB + rl;
  rn = rn < n ? rn : n - 1;
  int jb = rowptr[rn], je = rowptr[rn + 1];
  for (int64_t rb = rbk.first; rb < rbk.end; rb += rbk.step) {
    const int64_t r0 = rb * RB + rl;
    const bool live = r0 < n;
    const int64_t r = live ? r0 : n - 1;
    const int jr = jb, jr1 = je;
    rn = (rb + rbk.step) * RB + rl;
    rn = rn < n ? rn : n - 1;
    jb = rowptr[rn];
    je = rowptr[rn + 1];
    T rv[NCH][V], pv[NCH][V], zv[NCH][V];
    const T di = dinv[r];
    // the row's own entries (lanes past N load the row's last columns); for
    // j = 1 the caller passes Zprev = Zin and the previous iterate is zero
#pragma unroll
    for (int h = 0; h < NCH; ++h) {
      const int64_t i = r * N + lane_col<L, V>(g, h, N);
      load_cols<T, V>(R + i, rv[h]);
      load_cols<T, V>(Zin + i, zv[h]);
      load_cols<T, V>(Zprev + i, pv[h]);
    }
    T acc[NCH][V];
    row_gather_lanes<L, V, NCH, wide_wu<T>(), O32, T>(r, g, N, jr, jr1, col, val, Zin, acc);
#pragma unroll
    for (int h = 0; h < NCH; ++h) {
      const int c = (g + L * h) * V;
      T z[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const T dv = j > 1 ? zv[h][v] - pv[h][v] : zv[h][v];
        z[v] = zv[h][v] + (cd * dv + cr * (di * (rv[h][v] - acc[h][v])));
        if constexpr (PART) dot[h][v] += live && c < N ? (double)rv[h][v] * (double)z[v] : 0.0;
      }
      if (live && c < N) store_cols<T, V>(Zout + r * N + c, z);
    }
  }
  if constexpr (PART) block_cols_lanes<L, V, NCH, BS>(dot, N, partial);
}

// Gershgorin bound of D^-1 A: per-block maxima of dinv_i sum_j |a_ij|, then
// the maximum over blocks (times 1 + 1e-6) into out[0].
__global__ void __launch_bounds__(TPB) k_gersh(int64_t n, const int32_t* __restrict__ rowptr,
                                               const double* __restrict__ val, const double* __restrict__ dinv,
                                               double* __restrict__ partial) {
  __shared__ double sd[TPB];
  double m = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * TPB + threadIdx.x; r < n; r += (int64_t)gridDim.x * TPB) {
    double s = 0.0;
    for (int e = rowptr[r]; e < rowptr[r + 1]; ++e) s += fabs(val[e]);
    m = fmax(m, s * fabs(dinv[r]));
  }
  sd[threadIdx.x] = m;
  for (int h = TPB / 2; h > 0; h >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < h) sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + h]);
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sd[0];
}
__global__ void __launch_bounds__(TPB) k_gersh_final(int nblk, const double* __restrict__ partial,
                                                     double* __restrict__ out) {
  __shared__ double sd[TPB];
  double m = 0.0;
  for (int b = threadIdx.x; b < nblk; b += TPB) m = fmax(m, partial[b]);
  sd[threadIdx.x] = m;
  for (int h = TPB / 2; h > 0; h >>= 1) {
    __syncthreads();
    if ((int)threadIdx.x < h) sd[threadIdx.x] = fmax(sd[threadIdx.x], sd[threadIdx.x + h]);
  }
  if (threadIdx.x == 0) out[0] = sd[0] * (1.0 + 1e-6);
}

// y = A x for a dense m x m matrix (row-major), one wavefront per row.
__global__ void __launch_bounds__(TPB) k_dense_mv(int64_t m, const double* __restrict__ A,
                                                  const double* __restrict__ x, double* __restrict__ y) {
  const int64_t r = (int64_t)blockIdx.x * (TPB / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (r >= m) return;
  const double* a = A + r * m;
  double s = 0.0;
  for (int64_t k = lane; k < m; k += 64) s += a[k] * x[k];
  s = wave_sum(s);
  if (lane == 0) y[r] = s;
}

// Zout = (Zin or D^-1 R) + P eH (four coarse weights per fine DoF), and the
// per-block partials of R . Zout.
__global__ void __launch_bounds__(TPB) k_zcoarse(int64_t n, const double* __restrict__ dinv,
                                                 const double* __restrict__ R, const double* __restrict__ Zin,
                                                 const int32_t* __restrict__ Pk, const double* __restrict__ Pw,
                                                 const double* __restrict__ eH, double* __restrict__ Zout,
                                                 double* __restrict__ partial) {
  __shared__ double ws[TPB / 64];
  double dot = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x; i < n; i += (int64_t)gridDim.x * TPB) {
    double z = Zin ? Zin[i] : dinv[i] * R[i];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = Pk[4 * i + j];
      if (k >= 0) z += Pw[4 * i + j] * eH[k];
    }
    Zout[i] = z;
    dot += R[i] * z;
  }
  dot = wave_sum(dot);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) ws[wid] = dot;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (ws[0] + ws[1]) + (ws[2] + ws[3]);
}

// (row, column) thread layout of the vector kernels
struct RC {
  int R, rl, c;
  __device__ RC(int N) {
    R = TPB / N;
    rl = threadIdx.x / N;
    c = threadIdx.x - rl * N;
  }
};

// CG start: R = B - AX, P = Dinv R; block partials of rz, rr, bb.
template <typename T>
__global__ void __launch_bounds__(TPB) k_cg_init(int64_t n, int N, const T* __restrict__ B,
                                                 const T* __restrict__ AX, const T* __restrict__ dinv,
                                                 T* __restrict__ Rv, T* __restrict__ P,
                                                 double* __restrict__ partial, T* __restrict__ Z0,
                                                 const double* __restrict__ lmax, double ratio) {
  __shared__ double sd[TPB];
  const T ith = Z0 ? (T)(1.0 / cheb_theta(*lmax, ratio)) : T(0);
  RC p(N);
  double v[3] = {0.0, 0.0, 0.0};
  for (int64_t r0 = (int64_t)blockIdx.x * p.R; r0 < n; r0 += (int64_t)gridDim.x * p.R) {
    int64_t r = r0 + p.rl;
    if (p.rl < p.R && r < n) {
      int64_t i = r * N + p.c;
      T b = B[i];
      T rr = b - AX[i];
      T z = dinv[r] * rr;
      Rv[i] = rr;
      P[i] = z;
      if (Z0) Z0[i] = z * ith;
      v[0] += (double)rr * (double)z;
      v[1] += (double)rr * (double)rr;
      v[2] += (double)b * (double)b;
    }
  }
  for (int k = 0; k < 3; ++k) {
    __syncthreads();
    sd[threadIdx.x] = v[k];
    block_reduce_cols(sd, p.R, N);
    if ((int)threadIdx.x < N) partial[((int64_t)blockIdx.x * 3 + k) * N + threadIdx.x] = sd[threadIdx.x];
  }
}

// Column sums of nblk block partials (row b holds nvals values), computed by
// every block of a consumer kernel in the same fixed order. out: shared array.
__device__ void sum_partials(const double* __restrict__ partial, int nblk, int nvals, double* out) {
  constexpr int CH = 16;
  __shared__ double wsum[TPB / 64][CH];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int v0 = 0; v0 < nvals; v0 += CH) {
    int nc = nvals - v0 < CH ? nvals - v0 : CH;
    double acc[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) acc[q] = 0.0;
    for (int b = threadIdx.x; b < nblk; b += TPB) {
      const double* p = partial + (int64_t)b * nvals + v0;
#pragma unroll
      for (int q = 0; q < CH; ++q)
        if (q < nc) acc[q] += p[q];
    }
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      double v = wave_sum(acc[q]);
      if (lane == 0) wsum[wid][q] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < nc) {
      int q = threadIdx.x;
      out[v0 + q] = (wsum[0][q] + wsum[1][q]) + (wsum[2][q] + wsum[3][q]);
    }
    __syncthreads();
  }
}

// scal buffer per column c (two buffers, alternating by iteration parity):
// [0] rz [1] rr [2] bb [3] active [4] iterations.  flags: [0] active count.
enum { C_RZ = 0, C_RR, C_BB, C_ACT, C_IT };

// CG start scalars from the k_cg_init partials [rz, rr, bb] (one block).
__global__ void __launch_bounds__(TPB) k_cg_start(int N, int nblk, const double* __restrict__ partial, double rtol2,
                                                 const double* __restrict__ mask, double* __restrict__ scal,
                                                 int32_t* __restrict__ flags, const double* __restrict__ rz_part,
                                                 int nblk_rz) {
  __shared__ double sums[3 * MLC_MAX_ORBITALS];
  sum_partials(partial, nblk, 3 * N, sums);
  if (rz_part) sum_partials(rz_part, nblk_rz, N, sums);  // r.z of the polynomial preconditioner
  if (threadIdx.x != 0) return;
  int nact = 0;
  for (int c = 0; c < N; ++c) {
    scal[C_RZ * N + c] = sums[c];
    scal[C_RR * N + c] = sums[N + c];
    scal[C_BB * N + c] = sums[2 * N + c];
    scal[C_IT * N + c] = 0.0;
    bool act = sums[N + c] > rtol2 * sums[2 * N + c];
    if (mask) act = act && mask[C_ACT * N + c] != 0.0;
    scal[C_ACT * N + c] = act ? 1.0 : 0.0;
    nact += act;
  }
  flags[0] = nact;
}

// alpha_c = rz_c / (p.q)_c from the SpMM partials; X += alpha P, R -= alpha Q;
// block partials of r.Dr and r.r. A non-positive curvature on an active
// column sets brk and freezes that column (alpha = 0).
template <typename T>
__global__ void __launch_bounds__(TPB) k_cg_update(int64_t n, int N, const T* __restrict__ dinv,
                                                   T* __restrict__ X, T* __restrict__ Rv,
                                                   const T* __restrict__ P, const T* __restrict__ Q,
                                                   const double* __restrict__ pq_part, int nblk_pq,
                                                   const double* __restrict__ scal, const int32_t* __restrict__ flags,
                                                   double* __restrict__ partial, int32_t* __restrict__ brk,
                                                   T* __restrict__ Z0, const double* __restrict__ lmax,
                                                   double ratio) {
  if (flags[0] == 0) return;
  __shared__ double sd[TPB];
  __shared__ double alpha[MLC_MAX_ORBITALS];
  const T ith = Z0 ? (T)(1.0 / cheb_theta(*lmax, ratio)) : T(0);
  sum_partials(pq_part, nblk_pq, N, alpha);
  if ((int)threadIdx.x < N) {
    int c = threadIdx.x;
    double pq = alpha[c];
    bool act = scal[C_ACT * N + c] != 0.0;
    if (act && !(pq > 0.0)) {
      if (blockIdx.x == 0) brk[0] = 1;
      act = false;
    }
    alpha[c] = act ? scal[C_RZ * N + c] / pq : 0.0;
  }
  __syncthreads();
  RC p(N);
  T a = p.rl < p.R ? (T)alpha[p.c] : T(0);
  double v[2] = {0.0, 0.0};
  for (int64_t r0 = (int64_t)blockIdx.x * p.R; r0 < n; r0 += (int64_t)gridDim.x * p.R) {
    int64_t r = r0 + p.rl;
    if (p.rl < p.R && r < n) {
      int64_t i = r * N + p.c;
      T x = X[i] + a * P[i];
      T rr = Rv[i] - a * Q[i];
      X[i] = x;
      Rv[i] = rr;
      if (Z0) Z0[i] = dinv[r] * rr * ith;
      v[0] += (double)rr * (double)dinv[r] * (double)rr;
      v[1] += (double)rr * (double)rr;
    }
  }
  for (int k = 0; k < 2; ++k) {
    __syncthreads();
    sd[threadIdx.x] = v[k];
    block_reduce_cols(sd, p.R, N);
    if ((int)threadIdx.x < N) partial[((int64_t)blockIdx.x * 2 + k) * N + threadIdx.x] = sd[threadIdx.x];
  }
}

// The update for N > 8 with N a multiple of V = 16 / sizeof(T): a thread owns V
// consecutive columns of a row (one 16-byte access per block and row; N / V
// threads per row, TPB / (N / V) rows per block pass); the block's column
// sums go through LDS as R x N and are added row-halving.
template <typename T, int V>
__global__ void __launch_bounds__(TPB) k_cg_update_v(int64_t n, int N, const T* __restrict__ dinv,
                                                     T* __restrict__ X, T* __restrict__ Rv,
                                                     const T* __restrict__ P, const T* __restrict__ Q,
                                                     const double* __restrict__ pq_part, int nblk_pq,
                                                     const double* __restrict__ scal,
                                                     const int32_t* __restrict__ flags, double* __restrict__ partial,
                                                     int32_t* __restrict__ brk, T* __restrict__ Z0,
                                                     const double* __restrict__ lmax, double ratio) {
  if (flags[0] == 0) return;
  __shared__ double sd[2][TPB * V];
  __shared__ double alpha[MLC_MAX_ORBITALS];
  const T ith = Z0 ? (T)(1.0 / cheb_theta(*lmax, ratio)) : T(0);
  sum_partials(pq_part, nblk_pq, N, alpha);
  if ((int)threadIdx.x < N) {
    int c = threadIdx.x;
    double pq = alpha[c];
    bool act = scal[C_ACT * N + c] != 0.0;
    if (act && !(pq > 0.0)) {
      if (blockIdx.x == 0) brk[0] = 1;
      act = false;
    }
    alpha[c] = act ? scal[C_RZ * N + c] / pq : 0.0;
  }
  __syncthreads();
  const int Qn = N / V, R = TPB / Qn;
  const int rl = threadIdx.x / Qn, c0 = (threadIdx.x - rl * Qn) * V;
  const bool lane_on = rl < R;
  T a[V];
  double v0[V], v1[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    a[v] = lane_on ? (T)alpha[c0 + v] : T(0);
    v0[v] = v1[v] = 0.0;
  }
  // UPD_UR row passes per loop trip, their loads issued together (the grid is
  // small, since every consumer block re-reads all partials)
  for (int64_t rq = (int64_t)blockIdx.x * R * UPD_UR; rq < n; rq += (int64_t)gridDim.x * R * UPD_UR) {
    T x[UPD_UR][V], pp[UPD_UR][V], rr[UPD_UR][V], qq[UPD_UR][V];
    T di[UPD_UR];
#pragma unroll
    for (int k = 0; k < UPD_UR; ++k) {
      const int64_t r = rq + k * R + rl;
      if (lane_on && r < n) {
        const int64_t i = r * N + c0;
        load_cols<T, V>(X + i, x[k]);
        load_cols<T, V>(P + i, pp[k]);
        load_cols<T, V>(Rv + i, rr[k]);
        load_cols<T, V>(Q + i, qq[k]);
        di[k] = dinv[r];
      }
    }
#pragma unroll
    for (int k = 0; k < UPD_UR; ++k) {
      const int64_t r = rq + k * R + rl;
      if (lane_on && r < n) {
        const int64_t i = r * N + c0;
        T z[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
          x[k][v] += a[v] * pp[k][v];
          rr[k][v] -= a[v] * qq[k][v];
          z[v] = di[k] * rr[k][v] * ith;
          v0[v] += (double)rr[k][v] * (double)di[k] * (double)rr[k][v];
          v1[v] += (double)rr[k][v] * (double)rr[k][v];
        }
        store_cols<T, V>(X + i, x[k]);
        store_cols<T, V>(Rv + i, rr[k]);
        if (Z0) store_cols<T, V>(Z0 + i, z);
      }
    }
  }
  if (lane_on)
#pragma unroll
    for (int v = 0; v < V; ++v) {
      sd[0][rl * N + c0 + v] = v0[v];
      sd[1][rl * N + c0 + v] = v1[v];
    }
  for (int m = R; m > 1;) {
    const int h = (m + 1) >> 1;
    __syncthreads();
    for (int t = threadIdx.x; t < (m - h) * N; t += TPB) {
      sd[0][t] += sd[0][t + h * N];
      sd[1][t] += sd[1][t + h * N];
    }
    m = h;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < N; c += TPB) {
    partial[((int64_t)blockIdx.x * 2 + 0) * N + c] = sd[0][c];
    partial[((int64_t)blockIdx.x * 2 + 1) * N + c] = sd[1][c];
  }
}

// beta_c = rz'_c / rz_c and the test ||r||^2 <= rtol^2 ||b||^2 from the update
// partials; P = Dinv R + beta P. Block 0 writes the next scalars (the other
// buffer) and the active count.
template <typename T, int V>
__global__ void __launch_bounds__(TPB) k_cg_direction(int64_t n, int N, const T* __restrict__ dinv,
                                                      const T* __restrict__ Rv, T* __restrict__ P,
                                                      const double* __restrict__ upd_part, int nblk_upd,
                                                      const double* __restrict__ scal_in,
                                                      const int32_t* __restrict__ flags_in,
                                                      double* __restrict__ scal_out, int32_t* __restrict__ flags_out,
                                                      double rtol2, const double* __restrict__ rz_part, int nblk_rz,
                                                      const T* __restrict__ Zl) {
  if (flags_in[0] == 0) {
    // converged: carry the scalars to the other buffer so that the parity
    // alternation stays consistent, then do nothing else
    if (blockIdx.x == 0) {
      for (int i = threadIdx.x; i < 5 * N; i += TPB) scal_out[i] = scal_in[i];
      if (threadIdx.x == 0) flags_out[0] = 0;
    }
    return;
  }
  __shared__ double sums[2 * MLC_MAX_ORBITALS];
  __shared__ double beta[MLC_MAX_ORBITALS];
  __shared__ double still[MLC_MAX_ORBITALS];
  sum_partials(upd_part, nblk_upd, 2 * N, sums);
  if (rz_part) sum_partials(rz_part, nblk_rz, N, sums);  // r.z of the polynomial preconditioner
  if ((int)threadIdx.x < N) {
    int c = threadIdx.x;
    bool act = scal_in[C_ACT * N + c] != 0.0;
    double rzn = sums[c], rr = sums[N + c];
    beta[c] = act ? rzn / scal_in[C_RZ * N + c] : 0.0;
    double bb = scal_in[C_BB * N + c];
    still[c] = (act && rr > rtol2 * bb) ? 1.0 : 0.0;
    if (blockIdx.x == 0) {
      scal_out[C_RZ * N + c] = act ? rzn : scal_in[C_RZ * N + c];
      scal_out[C_RR * N + c] = act ? rr : scal_in[C_RR * N + c];
      scal_out[C_BB * N + c] = bb;
      scal_out[C_IT * N + c] = scal_in[C_IT * N + c] + (act ? 1.0 : 0.0);
      scal_out[C_ACT * N + c] = still[c];
    }
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int nact = 0;
    for (int c = 0; c < N; ++c) nact += still[c] != 0.0;
    flags_out[0] = nact;
  }
  // the rows in the update's layout: V consecutive columns per thread (no
  // 64-bit division per entry)
  const int Qn = N / V, R = TPB / Qn;
  const int rl = threadIdx.x / Qn, c0 = (threadIdx.x - rl * Qn) * V;
  const bool lane_on = rl < R;
  T b[V];
#pragma unroll
  for (int v = 0; v < V; ++v) b[v] = lane_on ? (T)beta[c0 + v] : T(0);
  for (int64_t rq = (int64_t)blockIdx.x * R * UPD_UR; rq < n; rq += (int64_t)gridDim.x * R * UPD_UR) {
    T z[UPD_UR][V], pp[UPD_UR][V];
#pragma unroll
    for (int k = 0; k < UPD_UR; ++k) {
      const int64_t r = rq + k * R + rl;
      if (lane_on && r < n) {
        const int64_t i = r * N + c0;
        if (Zl) {
          load_cols<T, V>(Zl + i, z[k]);
        } else {
          load_cols<T, V>(Rv + i, z[k]);
          const T di = dinv[r];
#pragma unroll
          for (int v = 0; v < V; ++v) z[k][v] *= di;
        }
        load_cols<T, V>(P + i, pp[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < UPD_UR; ++k) {
      const int64_t r = rq + k * R + rl;
      if (lane_on && r < n) {
#pragma unroll
        for (int v = 0; v < V; ++v) pp[k][v] = z[k][v] + b[v] * pp[k][v];
        store_cols<T, V>(P + r * N + c0, pp[k]);
      }
    }
  }
}

// Launch shapes of the row-gather kernels (NT <= 8 columns, four lanes per
// row), from measurements on the 4-atom cluster matrix (2.7M nonzeros):
// - producers of per-block partial sums (the CG SpMM and the last polynomial
//   step) run 1024-thread blocks on a grid capped at SPMM_MAXBLK, because
//   every consumer block re-reads all partials;
// - the other polynomial steps and plain products run 256-thread blocks, one
//   per row block (finer load balance), with deeper unrolling.
constexpr int ROW_G = 4;
constexpr int unroll_wide(int NT) { return NT <= 6 ? 4 : 2; }   // 256-thread shape
constexpr int unroll_part(int NT) { return NT <= 3 ? 4 : (NT <= 6 ? 2 : 1); }  // partial producers
// the last polynomial step also holds the row's R, d and Z entries: beyond
// three columns it needs more than 64 VGPRs (one 1024-thread block per CU)
constexpr int unroll_cheb_part(int NT) { return NT <= 3 ? 4 : 2; }
constexpr int waves_cheb_part(int NT) { return NT <= 3 ? 8 : 4; }
constexpr int waves_wide(int NT) { return NT <= 2 ? 8 : 4; }
constexpr int waves_part(int NT) { return NT <= 6 ? 8 : 4; }

template <int NT, typename T>
void spmm_small(hipStream_t s, int64_t n, const int32_t* rowptr, const int32_t* col, const T* val, const T* X, T* Y,
                double* partial, const int32_t* flags) {
  if (partial) {
    const int64_t needed = (n + (SPMM_BS / ROW_G) - 1) / (SPMM_BS / ROW_G);
    hipLaunchKernelGGL((k_spmm_small<NT, ROW_G, unroll_part(NT), SPMM_BS, waves_part(NT), T>),
                       dim3(cap_xcd(needed, SPMM_MAXBLK)), dim3(SPMM_BS), 0, s, n, rowptr, col, val, X, Y, partial,
                       flags);
  } else {
    const int64_t needed = (n + (TPB / ROW_G) - 1) / (TPB / ROW_G);
    hipLaunchKernelGGL((k_spmm_small<NT, ROW_G, unroll_wide(NT), TPB, waves_wide(NT), T>),
                       dim3(cap_xcd(needed, 1 << 30)), dim3(TPB), 0, s, n, rowptr, col, val, X, Y, partial, flags);
  }
}

int vec_blocks(int64_t n, int N) {
  int64_t R = TPB / N;
  return cap((n + R - 1) / R, VEC_MAXBLK);
}
// columns per thread of the update and direction kernels, and their grid
// (UPD_UR row passes per loop trip)
template <typename T>
inline int upd_v(int N) {
  constexpr int V = 16 / (int)sizeof(T);
  return (N > 8 && N % V == 0) ? V : 1;
}
template <typename T>
inline int upd_blocks(int64_t n, int N) {
  const int V = upd_v<T>(N);
  const int64_t R = (int64_t)(TPB / (N / V)) * (V > 1 ? UPD_UR : 1);
  return cap((n + R - 1) / R, VEC_MAXBLK);
}

// FP32 <-> FP64 helpers of the iterative refinement
__global__ void __launch_bounds__(TPB) k_to_f32(int64_t m, const double* __restrict__ a, float* __restrict__ b) {
  int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i < m) b[i] = (float)a[i];
}
__global__ void __launch_bounds__(TPB) k_add_f32(int64_t m, const float* __restrict__ d, double* __restrict__ x) {
  int64_t i = (int64_t)blockIdx.x * TPB + threadIdx.x;
  if (i < m) x[i] += (double)d[i];
}

// The layouts of wide_launch (64-bit gather offsets).
template <typename T, typename F>
void wide_launch_tag(hipStream_t, int64_t n, int N, F&& f) {
  const WideShape w = wide_shape(N, 16 / (int)sizeof(T));
  const dim3 g(wide_blocks_for(n)), b(WIDE_BS);
  if (w.NCH > 1) {
    f(WideTag<64, 1, 2>{}, g, b);
    return;
  }
#define WIDE_L(V)                        \
  switch (w.L) {                         \
    case 4: f(WideTag<4, V, 1>{}, g, b); break;   \
    case 8: f(WideTag<8, V, 1>{}, g, b); break;   \
    case 16: f(WideTag<16, V, 1>{}, g, b); break; \
    case 32: f(WideTag<32, V, 1>{}, g, b); break; \
    default: f(WideTag<64, V, 1>{}, g, b);        \
  }
  if (w.V == 1) {
    WIDE_L(1)
  } else if (w.V == 2) {
    WIDE_L(2)
  } else if constexpr (sizeof(T) == 4) {
    WIDE_L(4)
  }
#undef WIDE_L
}

// Calls f(tag, grid, block) with tag::L, tag::V, tag::NCH the N > 8 layout of
// wide_shape(N, sizeof(T)) and tag::O32 whether an n x N block of T spans
// less than 4 GiB (32-bit gather offsets).
template <typename T, typename F>
void wide_launch(hipStream_t s, int64_t n, int N, F&& f) {
  if ((uint64_t)n * (uint64_t)N * sizeof(T) < (1ull << 32)) {
    wide_launch_tag<T>(s, n, N, [&](auto tag, dim3 g, dim3 b) { f(WideTag32<decltype(tag)>{}, g, b); });
  } else {
    wide_launch_tag<T>(s, n, N, f);
  }
}

template <typename T>
void spmm_any(hipStream_t s, int64_t n, int N, const int32_t* rowptr, const int32_t* col, const T* val, const T* X,
              T* Y, double* partial, const int32_t* flags) {
#define SPMM_CASE(K)                                                  \
  case K:                                                             \
    spmm_small<K, T>(s, n, rowptr, col, val, X, Y, partial, flags); \
    return;
  switch (N) {
    SPMM_CASE(1)
    SPMM_CASE(2)
    SPMM_CASE(3)
    SPMM_CASE(4)
    SPMM_CASE(5)
    SPMM_CASE(6)
    SPMM_CASE(7)
    SPMM_CASE(8)
    default:
      wide_launch<T>(s, n, N, [&](auto tag, dim3 g, dim3 b) {
        using K = decltype(tag);
        if (partial)
          hipLaunchKernelGGL((k_spmm_rows<K::L, K::V, K::NCH, K::O32, WIDE_BS, T>), g, b, 0, s, n, N, rowptr, col, val,
                             X, Y, partial, flags);
        else
          hipLaunchKernelGGL((k_spmm_rows<K::L, K::V, K::NCH, K::O32, WIDE_BS_PLAIN, T>),
                             dim3(wide_plain_blocks(n, K::L)), dim3(WIDE_BS_PLAIN), 0, s, n, N, rowptr, col, val, X, Y,
                             partial, flags);
      });
  }
#undef SPMM_CASE
}

}  // namespace

int cg_blocks(int64_t n, int N) {
  int64_t R = TPB / N;
  return cap((n + R - 1) / R, MAXBLK);
}
int spmm_blocks(int64_t n, int N) {
  if (N <= 8) return cap_xcd((n + (SPMM_BS / ROW_G) - 1) / (SPMM_BS / ROW_G), SPMM_MAXBLK);
  return wide_blocks_for(n);
}
int cg_max_blocks() { return MAXBLK; }

// Y = A X (N columns); with partial: per-block column sums of X . Y (the CG
// variant, 1024-thread blocks); with flags: early exit when no column is active.
void launch_spmm2(hipStream_t s, int64_t n, int N, const int32_t* rowptr, const int32_t* col, const double* val,
                  const double* X, double* Y, double* partial, const int32_t* flags) {
  spmm_any<double>(s, n, N, rowptr, col, val, X, Y, partial, flags);
}
void launch_spmm2_f32(hipStream_t s, int64_t n, int N, const int32_t* rowptr, const int32_t* col, const float* val,
                      const float* X, float* Y, double* partial, const int32_t* flags) {
  spmm_any<float>(s, n, N, rowptr, col, val, X, Y, partial, flags);
}

template <typename T>
void launch_cg_init_t(hipStream_t s, int64_t n, int N, const T* B, const T* AX, const T* dinv, T* Rv, T* P,
                      double* partial, const PolyPC<T>* pc) {
  hipLaunchKernelGGL((k_cg_init<T>), dim3(cg_blocks(n, N)), dim3(TPB), 0, s, n, N, B, AX, dinv, Rv, P, partial,
                     pc ? pc->Z[0] : (T*)nullptr, pc ? pc->lmax : nullptr,
                     pc ? pc->ratio : 1.0);
}
void launch_cg_init2(hipStream_t s, int64_t n, int N, const double* B, const double* AX, const double* dinv,
                     double* Rv, double* P, double* partial) {
  launch_cg_init_t<double>(s, n, N, B, AX, dinv, Rv, P, partial, nullptr);
}
void launch_cg_init2_f32(hipStream_t s, int64_t n, int N, const float* B, const float* AX, const float* dinv,
                         float* Rv, float* P, double* partial) {
  launch_cg_init_t<float>(s, n, N, B, AX, dinv, Rv, P, partial, nullptr);
}

void launch_cg_start2(hipStream_t s, int64_t n, int N, const double* partial, double rtol2, const double* mask,
                      double* scal, int32_t* flags, const double* rz_part) {
  hipLaunchKernelGGL(k_cg_start, dim3(1), dim3(TPB), 0, s, N, cg_blocks(n, N), partial, rtol2, mask, scal, flags,
                     rz_part, spmm_blocks(n, N));
}
void launch_cg_start(hipStream_t s, int64_t n, int N, const double* partial, double rtol2, const double* mask,
                     double* scal, int32_t* flags) {
  launch_cg_start2(s, n, N, partial, rtol2, mask, scal, flags, nullptr);
}

template <typename T>
void launch_cg_update_t(hipStream_t s, int64_t n, int N, const T* dinv, T* X, T* Rv, const T* P, const T* Q,
                        const double* pq_part, const double* scal, const int32_t* flags, double* partial,
                        int32_t* brk, const PolyPC<T>* pc) {
  constexpr int VV = 16 / (int)sizeof(T);
  if (upd_v<T>(N) == VV)
    hipLaunchKernelGGL((k_cg_update_v<T, VV>), dim3(upd_blocks<T>(n, N)), dim3(TPB), 0, s, n, N, dinv, X, Rv, P, Q,
                       pq_part, spmm_blocks(n, N), scal, flags, partial, brk, pc ? pc->Z[0] : (T*)nullptr,
                       pc ? pc->lmax : nullptr, pc ? pc->ratio : 1.0);
  else
    hipLaunchKernelGGL((k_cg_update<T>), dim3(upd_blocks<T>(n, N)), dim3(TPB), 0, s, n, N, dinv, X, Rv, P, Q, pq_part,
                       spmm_blocks(n, N), scal, flags, partial, brk, pc ? pc->Z[0] : (T*)nullptr,
                       pc ? pc->lmax : nullptr, pc ? pc->ratio : 1.0);
}
void launch_cg_update_f(hipStream_t s, int64_t n, int N, const double* dinv, double* X, double* Rv, const double* P,
                        const double* Q, const double* pq_part, const double* scal, const int32_t* flags,
                        double* partial, int32_t* brk) {
  launch_cg_update_t<double>(s, n, N, dinv, X, Rv, P, Q, pq_part, scal, flags, partial, brk, nullptr);
}
void launch_cg_update_f32(hipStream_t s, int64_t n, int N, const float* dinv, float* X, float* Rv, const float* P,
                          const float* Q, const double* pq_part, const double* scal, const int32_t* flags,
                          double* partial, int32_t* brk) {
  launch_cg_update_t<float>(s, n, N, dinv, X, Rv, P, Q, pq_part, scal, flags, partial, brk, nullptr);
}

template <typename T>
void launch_cg_direction_z(hipStream_t s, int64_t n, int N, const T* dinv, const T* Rv, T* P, const double* upd_part,
                           const double* scal_in, const int32_t* flags_in, double* scal_out, int32_t* flags_out,
                           double rtol2, const double* rz_part, const T* Zl) {
  constexpr int VV = 16 / (int)sizeof(T);
  if (upd_v<T>(N) == VV)
    hipLaunchKernelGGL((k_cg_direction<T, VV>), dim3(upd_blocks<T>(n, N)), dim3(TPB), 0, s, n, N, dinv, Rv, P,
                       upd_part, upd_blocks<T>(n, N), scal_in, flags_in, scal_out, flags_out, rtol2, rz_part,
                       spmm_blocks(n, N), Zl);
  else
    hipLaunchKernelGGL((k_cg_direction<T, 1>), dim3(upd_blocks<T>(n, N)), dim3(TPB), 0, s, n, N, dinv, Rv, P,
                       upd_part, upd_blocks<T>(n, N), scal_in, flags_in, scal_out, flags_out, rtol2, rz_part,
                       spmm_blocks(n, N), Zl);
}
template <typename T>
void launch_cg_direction_t(hipStream_t s, int64_t n, int N, const T* dinv, const T* Rv, T* P, const double* upd_part,
                           const double* scal_in, const int32_t* flags_in, double* scal_out, int32_t* flags_out,
                           double rtol2, const PolyPC<T>* pc) {
  launch_cg_direction_z<T>(s, n, N, dinv, Rv, P, upd_part, scal_in, flags_in, scal_out, flags_out, rtol2,
                           pc ? pc->rz_part : nullptr, pc ? pc->Z[(pc->degree - 1) & 1] : nullptr);
}

void launch_dense_mv(hipStream_t s, int64_t m, const double* Ainv, const double* x, double* y) {
  hipLaunchKernelGGL(k_dense_mv, dim3((unsigned)((m + 3) / 4)), dim3(TPB), 0, s, m, Ainv, x, y);
}
void launch_zcoarse(hipStream_t s, int64_t n, const double* dinv, const double* R, const double* Zin,
                    const int32_t* Pk, const double* Pw, const double* eH, double* Zout, double* rz_part) {
  hipLaunchKernelGGL(k_zcoarse, dim3(spmm_blocks(n, 1)), dim3(TPB), 0, s, n, dinv, R, Zin, Pk, Pw, eH, Zout, rz_part);
}
void launch_cg_direction_f(hipStream_t s, int64_t n, int N, const double* dinv, const double* Rv, double* P,
                           const double* upd_part, const double* scal_in, const int32_t* flags_in, double* scal_out,
                           int32_t* flags_out, double rtol2) {
  launch_cg_direction_t<double>(s, n, N, dinv, Rv, P, upd_part, scal_in, flags_in, scal_out, flags_out, rtol2,
                                nullptr);
}
void launch_cg_direction_f32(hipStream_t s, int64_t n, int N, const float* dinv, const float* Rv, float* P,
                             const double* upd_part, const double* scal_in, const int32_t* flags_in, double* scal_out,
                             int32_t* flags_out, double rtol2) {
  launch_cg_direction_t<float>(s, n, N, dinv, Rv, P, upd_part, scal_in, flags_in, scal_out, flags_out, rtol2, nullptr);
}

// Chebyshev step j >= 1: reads Zin (= z_{j-1}) and Zprev (= z_{j-2} for
// j > 1; for j = 1 pass Zin, whose values are then not used); writes Zout
// (which may be Zprev) and, when part is given, the r.z partials.
template <typename T>
void launch_cheb_step_t(hipStream_t s, int64_t n, int N, const int32_t* rowptr, const int32_t* col, const T* val,
                        const T* dinv, const T* Rv, const PolyPC<T>& pc, int j, const T* zin, const T* zprev,
                        T* zout, double* part, const int32_t* flags) {
  if constexpr (std::is_same<T, double>::value) {
    if (pc.val32 && N == 1) {
      // one FP64 column with FP32 matrix values (the Hartree problem's polynomial)
      if (part) {
        const int64_t needed = (n + (SPMM_BS / ROW_G) - 1) / (SPMM_BS / ROW_G);
        hipLaunchKernelGGL((k_cheb_small<1, ROW_G, unroll_cheb_part(1), SPMM_BS, waves_cheb_part(1), T, float>),
                           dim3(cap_xcd(needed, SPMM_MAXBLK)), dim3(SPMM_BS), 0, s, n, rowptr, col, pc.val32, dinv,
                           Rv, zin, zprev, zout, pc.lmax, pc.ratio, j, part, flags);
      } else {
        hipLaunchKernelGGL(k_cheb_stream1, dim3(cap_xcd((n + 63) / 64, 1 << 30)), dim3(64), 0, s, n, rowptr, col,
                           pc.val32, dinv, Rv, zin, zprev, zout, pc.lmax, pc.ratio, j, flags);
      }
      return;
    }
  }
  if (N <= 8) {
#define CHEB_CASE(K)                                                                                             \
  case K:                                                                                                        \
    if (part) {                                                                                                  \
      const int64_t needed = (n + (SPMM_BS / ROW_G) - 1) / (SPMM_BS / ROW_G);                                    \
      hipLaunchKernelGGL((k_cheb_small<K, ROW_G, unroll_cheb_part(K), SPMM_BS, waves_cheb_part(K), T>),          \
                         dim3(cap_xcd(needed, SPMM_MAXBLK)), dim3(SPMM_BS), 0, s, n, rowptr, col, val, dinv, Rv, \
                         zin, zprev, zout, pc.lmax, pc.ratio, j, part, flags);                                   \
    } else {                                                                                                     \
      const int64_t needed = (n + (TPB / ROW_G) - 1) / (TPB / ROW_G);                                            \
      hipLaunchKernelGGL((k_cheb_small<K, ROW_G, unroll_wide(K), TPB, waves_wide(K), T>),                        \
                         dim3(cap_xcd(needed, 1 << 30)), dim3(TPB), 0, s, n, rowptr, col, val, dinv, Rv, zin,    \
                         zprev, zout, pc.lmax, pc.ratio, j, part, flags);                                        \
    }                                                                                                            \
    break;
    switch (N) {
      CHEB_CASE(1)
      CHEB_CASE(2)
      CHEB_CASE(3)
      CHEB_CASE(4)
      CHEB_CASE(5)
      CHEB_CASE(6)
      CHEB_CASE(7)
      CHEB_CASE(8)
    }
#undef CHEB_CASE
  } else {
    wide_launch<T>(s, n, N, [&](auto tag, dim3 g, dim3 b) {
      using K = decltype(tag);
      if (part)
        hipLaunchKernelGGL((k_cheb_rows<K::L, K::V, K::NCH, true, K::O32, WIDE_BS, T>), g, b, 0, s, n, N, rowptr, col,
                           val, dinv, Rv, zin, zprev, zout, pc.lmax, pc.ratio, j, part, flags);
      else
        hipLaunchKernelGGL((k_cheb_rows<K::L, K::V, K::NCH, false, K::O32, WIDE_BS_PLAIN, T>),
                           dim3(wide_plain_blocks(n, K::L)), dim3(WIDE_BS_PLAIN), 0, s, n, N, rowptr, col, val, dinv, Rv,
                           zin, zprev, zout, pc.lmax, pc.ratio, j, part, flags);
    });
  }
}

// Chebyshev steps 1..degree-1 from z_0 in Z[0] (written by the init or update
// kernel): step j reads Z[(j-1)&1] and Z[j&1] and writes Z[j&1]; the last step
// writes last_out instead when given, and the r.z partials.
template <typename T>
void launch_cheb_steps_t(hipStream_t s, int64_t n, int N, const int32_t* rowptr, const int32_t* col, const T* val,
                         const T* dinv, const T* Rv, const PolyPC<T>& pc, T* last_out, const int32_t* flags) {
  for (int j = 1; j < pc.degree; ++j) {
    const bool last = j == pc.degree - 1;
    const T* zin = pc.Z[(j - 1) & 1];
    T* zprev = pc.Z[j & 1];
    T* zout = last && last_out ? last_out : zprev;
    launch_cheb_step_t<T>(s, n, N, rowptr, col, val, dinv, Rv, pc, j, zin, j > 1 ? zprev : zin, zout,
                          last ? pc.rz_part : nullptr, flags);
  }
}

void launch_gershgorin(hipStream_t s, int64_t n, const int32_t* rowptr, const double* val, const double* dinv,
                       double* partial, double* out) {
  int nbk = (int)((n + TPB - 1) / TPB);
  if (nbk > 1024) nbk = 1024;
  if (nbk < 1) nbk = 1;
  hipLaunchKernelGGL(k_gersh, dim3(nbk), dim3(TPB), 0, s, n, rowptr, val, dinv, partial);
  hipLaunchKernelGGL(k_gersh_final, dim3(1), dim3(TPB), 0, s, nbk, partial, out);
}

template void launch_cg_init_t<double>(hipStream_t, int64_t, int, const double*, const double*, const double*, double*,
                                       double*, double*, const PolyPC<double>*);
template void launch_cg_init_t<float>(hipStream_t, int64_t, int, const float*, const float*, const float*, float*,
                                      float*, double*, const PolyPC<float>*);
template void launch_cg_update_t<double>(hipStream_t, int64_t, int, const double*, double*, double*, const double*,
                                         const double*, const double*, const double*, const int32_t*, double*,
                                         int32_t*, const PolyPC<double>*);
template void launch_cg_update_t<float>(hipStream_t, int64_t, int, const float*, float*, float*, const float*,
                                        const float*, const double*, const double*, const int32_t*, double*, int32_t*,
                                        const PolyPC<float>*);
template void launch_cg_direction_t<double>(hipStream_t, int64_t, int, const double*, const double*, double*,
                                            const double*, const double*, const int32_t*, double*, int32_t*, double,
                                            const PolyPC<double>*);
template void launch_cg_direction_t<float>(hipStream_t, int64_t, int, const float*, const float*, float*,
                                           const double*, const double*, const int32_t*, double*, int32_t*, double,
                                           const PolyPC<float>*);
template void launch_cg_direction_z<double>(hipStream_t, int64_t, int, const double*, const double*, double*,
                                            const double*, const double*, const int32_t*, double*, int32_t*, double,
                                            const double*, const double*);
template void launch_cg_direction_z<float>(hipStream_t, int64_t, int, const float*, const float*, float*,
                                           const double*, const double*, const int32_t*, double*, int32_t*, double,
                                           const double*, const float*);
template void launch_cheb_steps_t<double>(hipStream_t, int64_t, int, const int32_t*, const int32_t*, const double*,
                                          const double*, const double*, const PolyPC<double>&, double*,
                                          const int32_t*);
template void launch_cheb_steps_t<float>(hipStream_t, int64_t, int, const int32_t*, const int32_t*, const float*,
                                         const float*, const float*, const PolyPC<float>&, float*, const int32_t*);
template void launch_cheb_step_t<double>(hipStream_t, int64_t, int, const int32_t*, const int32_t*, const double*,
                                         const double*, const double*, const PolyPC<double>&, int, const double*,
                                         const double*, double*, double*, const int32_t*);
template void launch_cheb_step_t<float>(hipStream_t, int64_t, int, const int32_t*, const int32_t*, const float*,
                                        const float*, const float*, const PolyPC<float>&, int, const float*,
                                        const float*, float*, double*, const int32_t*);

void launch_to_f32(hipStream_t s, int64_t m, const double* a, float* b) {
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((m + TPB - 1) / TPB)), dim3(TPB), 0, s, m, a, b);
}
void launch_add_f32(hipStream_t s, int64_t m, const float* d, double* x) {
  hipLaunchKernelGGL(k_add_f32, dim3((unsigned)((m + TPB - 1) / TPB)), dim3(TPB), 0, s, m, d, x);
}

}  // namespace mlc
