// Row gathers of the CSR SpMM kernels (single-context and batched).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mlc {

// acc[c] += sum over this lane's nonzeros of row r (every G-th from
// rowptr[r] + sub) of a_rj X[j][c]; U nonzeros per pass have their column
// and value loads issued together, then their gathers. Entries past the row
// end repeat the row's last entry with a zero weight (the same terms in the
// same order as a plain loop, since adding +0 changes nothing), so every load
// is in bounds and issued unconditionally: no branch inside the pass, and all
// U gathers are in flight at once.
// The matrix values may be stored in a narrower type VT than the vectors (T):
// each value is widened before its product.
// (jb, j1: the row's entry range, loaded by the caller.)
template <int NT, int G, int U, typename VT, typename T>
__device__ __forceinline__ void row_gather(int jb, int j1, int sub, const int32_t* __restrict__ col,
                                           const VT* __restrict__ val, const T* __restrict__ X, T (&acc)[NT]) {
  for (int j = jb + sub; j < j1; j += G * U) {
    int cc[U];
    T vv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = j + u * G;
      const uint32_t ec = (uint32_t)(e < j1 ? e : j1 - 1);
      cc[u] = col[ec];
      const T a = (T)val[ec];
      vv[u] = e < j1 ? a : T(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const T* xr = X + (int64_t)cc[u] * NT;
#pragma unroll
      for (int c = 0; c < NT; ++c) acc[c] += vv[u] * xr[c];
    }
  }
}
template <int NT, int G, int U, typename VT, typename T>
__device__ __forceinline__ void row_gather(int64_t r, int sub, const int32_t* __restrict__ rowptr,
                                           const int32_t* __restrict__ col, const VT* __restrict__ val,
                                           const T* __restrict__ X, T (&acc)[NT]) {
  row_gather<NT, G, U>(rowptr[r], rowptr[r + 1], sub, col, val, X, acc);
}

// Layout of the kernels for N > 8 orbitals: a lane owns V consecutive columns
// (V = 4, 2 or 1: the largest that divides N, up to vmax), L lanes share a row
// (the smallest power of two >= N / V, from 4 up to 64), and a lane owns NCH
// column groups (2 only for V = 1 and N > 64).
struct WideShape {
  int V, L, NCH;
};
__host__ __device__ inline WideShape wide_shape(int N, int vmax) {
  int V = (vmax >= 4 && N % 4 == 0) ? 4 : ((vmax >= 2 && N % 2 == 0) ? 2 : 1);
  const int groups = (N + V - 1) / V;
  int L = 4;
  while (L < groups && L < 64) L *= 2;
  return {V, L, (groups + L - 1) / L};
}
template <int L_, int V_, int NCH_>
struct WideTag {
  static constexpr int L = L_, V = V_, NCH = NCH_;
  static constexpr bool O32 = false;
};
// the same layout with 32-bit gather offsets
template <typename Tag>
struct WideTag32 : Tag {
  static constexpr bool O32 = true;
};

template <typename T, int V>
__device__ __forceinline__ void load_cols(const T* __restrict__ p, T (&o)[V]) {
  if constexpr (V == 1) {
    o[0] = p[0];
  } else if constexpr (V == 2 && sizeof(T) == 8) {
    const double2 q = *reinterpret_cast<const double2*>(p);
    o[0] = q.x;
    o[1] = q.y;
  } else if constexpr (V == 2) {
    const float2 q = *reinterpret_cast<const float2*>(p);
    o[0] = q.x;
    o[1] = q.y;
  } else {
    const float4 q = *reinterpret_cast<const float4*>(p);
    o[0] = q.x;
    o[1] = q.y;
    o[2] = q.z;
    o[3] = q.w;
  }
}
template <typename T, int V>
__device__ __forceinline__ void store_cols(T* __restrict__ p, const T (&o)[V]) {
  if constexpr (V == 1) {
    p[0] = o[0];
  } else if constexpr (V == 2 && sizeof(T) == 8) {
    *reinterpret_cast<double2*>(p) = make_double2(o[0], o[1]);
  } else if constexpr (V == 2) {
    *reinterpret_cast<float2*>(p) = make_float2(o[0], o[1]);
  } else {
    *reinterpret_cast<float4*>(p) = make_float4(o[0], o[1], o[2], o[3]);
  }
}

// Column offset of the lane's group h, clamped into the row: lanes whose
// group lies past N read the row's last V columns (their sums are never
// stored), so that the loads need no branch.
template <int L, int V>
__device__ __forceinline__ int lane_col(int g, int h, int N) {
  const int c = (g + L * h) * V;
  return c < N ? c : N - V;
}

// acc[h][v] = (A X)[r, lane_col(g, h) + v] for the lane's column group g
// (meaningful where the group lies within N). The row's L lanes load its
// column indices and values cooperatively, CH = max(L, WU) entries per
// chunk (lane g takes entries g, g + L, ...; entries past the row end repeat
// its last entry with weight zero), and pass them to each other with
// width-L shuffles: one load instruction per L entries instead of one per
// entry. Each sub-pass then issues the WU gathers of WU entries with no
// branch inside, so all of them are in flight together; sub-passes wholly
// past the row end are skipped (the same for the row's L lanes). With O32
// (the caller guarantees n N sizeof(T) < 2^32) the gathers address X by a
// 32-bit byte offset from its base: one register per address instead of two.
// The L lanes of a row are consecutive lanes of one wavefront, L dividing 64.
template <int L, int V, int NCH, int WU, bool O32, typename T>
__device__ __forceinline__ void row_gather_lanes(int64_t r, int g, int N, int jb, int j1,
                                                 const int32_t* __restrict__ col, const T* __restrict__ val,
                                                 const T* __restrict__ X, T (&acc)[NCH][V]) {
  constexpr int CH = L > WU ? L : WU;   // entries per cooperative chunk
  constexpr int PER = CH / L;           // entries each lane loads per chunk
  static_assert(CH % L == 0 && CH % WU == 0, "chunk must hold whole lane rounds and sub-passes");
  T a0[NCH][V], a1[NCH][V];
  int coff[NCH];
#pragma unroll
  for (int h = 0; h < NCH; ++h) {
    coff[h] = lane_col<L, V>(g, h, N);
#pragma unroll
    for (int v = 0; v < V; ++v) a0[h][v] = a1[h][v] = T(0);
  }
  const uint32_t rowb = (uint32_t)N * (uint32_t)sizeof(T);
  for (int j = jb; j < j1; j += CH) {
    int kl[PER];
    T wl[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e0 = j + g + L * i;
      const uint32_t e = (uint32_t)(e0 < j1 ? e0 : j1 - 1);
      kl[i] = col[e];
      const T a = val[e];
      wl[i] = e0 < j1 ? a : T(0);
    }
#pragma unroll
    for (int p = 0; p < CH; p += WU) {
      if (j + p >= j1) break;
      int k[WU];
      T w[WU];
#pragma unroll
      for (int u = 0; u < WU; ++u) {
        k[u] = __shfl(kl[(p + u) / L], (p + u) % L, L);
        w[u] = __shfl(wl[(p + u) / L], (p + u) % L, L);
      }
      T x[WU][NCH][V];
#pragma unroll
      for (int u = 0; u < WU; ++u)
#pragma unroll
        for (int h = 0; h < NCH; ++h) {
          if constexpr (O32) {
            const uint32_t off = (uint32_t)k[u] * rowb + (uint32_t)coff[h] * (uint32_t)sizeof(T);
            load_cols<T, V>(reinterpret_cast<const T*>(reinterpret_cast<const char*>(X) + off), x[u][h]);
          } else {
            load_cols<T, V>(X + (int64_t)k[u] * N + coff[h], x[u][h]);
          }
        }
#pragma unroll
      for (int u = 0; u < WU; u += 2)
#pragma unroll
        for (int h = 0; h < NCH; ++h)
#pragma unroll
          for (int v = 0; v < V; ++v) {
            a0[h][v] += w[u] * x[u][h][v];
            a1[h][v] += w[u + 1] * x[u + 1][h][v];
          }
    }
  }
#pragma unroll
  for (int h = 0; h < NCH; ++h)
#pragma unroll
    for (int v = 0; v < V; ++v) acc[h][v] = a0[h][v] + a1[h][v];
}

}  // namespace mlc
