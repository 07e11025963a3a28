// Row gathers of the CSR SpMM kernels (single-context and batched).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mlc {

// acc[c] += sum over this lane's nonzeros of row r (every G-th from
// rowptr[r] + sub) of a_rj X[j][c]; U nonzeros per pass have their column
// and value loads issued together, then their gathers. Entries past the row
// end read row r itself with a zero weight (the same terms in the same order
// as a plain loop, since adding +0 changes nothing).
template <int NT, int G, int U, typename T>
__device__ __forceinline__ void row_gather(int64_t r, int sub, const int32_t* __restrict__ rowptr,
                                           const int32_t* __restrict__ col, const T* __restrict__ val,
                                           const T* __restrict__ X, T (&acc)[NT]) {
  const int j1 = rowptr[r + 1];
  for (int j = rowptr[r] + sub; j < j1; j += G * U) {
    int cc[U];
    T vv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int e = j + u * G;
      const bool ok = e < j1;
      cc[u] = ok ? col[e] : (int)r;
      vv[u] = ok ? val[e] : T(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const T* xr = X + (int64_t)cc[u] * NT;
#pragma unroll
      for (int c = 0; c < NT; ++c) acc[c] += vv[u] * xr[c];
    }
  }
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

// acc[h][v] = (A X)[r, (g + L h) V + v] for the lane's column group g (zero
// where the group lies past N).
template <int L, int V, int NCH, int WU, typename T>
__device__ __forceinline__ void row_gather_lanes(int64_t r, int g, int N, int jb, int j1,
                                                 const int32_t* __restrict__ col, const T* __restrict__ val,
                                                 const T* __restrict__ X, T (&acc)[NCH][V]) {
  T a0[NCH][V], a1[NCH][V];
#pragma unroll
  for (int h = 0; h < NCH; ++h)
#pragma unroll
    for (int v = 0; v < V; ++v) a0[h][v] = a1[h][v] = T(0);
  for (int j = jb; j < j1; j += WU) {
    int k[WU];
    T w[WU];
#pragma unroll
    for (int u = 0; u < WU; ++u) {
      const bool ok = j + u < j1;
      k[u] = ok ? col[j + u] : (int)r;
      w[u] = ok ? val[j + u] : T(0);
    }
    T x[WU][NCH][V];
#pragma unroll
    for (int u = 0; u < WU; ++u)
#pragma unroll
      for (int h = 0; h < NCH; ++h) {
        const int c = (g + L * h) * V;
        if (c < N) {
          load_cols<T, V>(X + (int64_t)k[u] * N + c, x[u][h]);
        } else {
#pragma unroll
          for (int v = 0; v < V; ++v) x[u][h][v] = T(0);
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
#pragma unroll
  for (int h = 0; h < NCH; ++h)
#pragma unroll
    for (int v = 0; v < V; ++v) acc[h][v] = a0[h][v] + a1[h][v];
}

}  // namespace mlc
