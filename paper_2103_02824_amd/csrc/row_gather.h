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

}  // namespace mlc
