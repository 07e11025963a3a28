// Batched CG over independent systems: problem descriptors and launchers.
// Not part of the ABI.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

#include "../../include/mlc.h"

namespace mlc {

// One problem of a batched multi-column CG: n rows, N columns (orbital
// fastest), Jacobi preconditioner dinv, rows cut into ntiles tiles starting at
// global tile tile0.
template <typename T>
struct BProb {
  const int32_t* rowptr;
  const int32_t* col;
  const T* val;
  const T* dinv;
  const T* B;
  T* X;
  T* R;
  T* P;
  T* Q;
  T* Z0;               // Chebyshev preconditioner: ping-pong blocks and the step
  T* Z1;               // difference (n x N each), and the device scalar lmax of
  T* Dd;               // D^-1 A (null: Jacobi)
  const double* lmax;
  int64_t n;
  int32_t N;
  int32_t tile0;
  int32_t ntiles;
  int32_t pad;
};

// Chebyshev polynomial preconditioner of a batched solve (degree 0: Jacobi).
struct BPoly {
  int degree;
  double ratio;
  double* rz_part;  // per-tile r.z partials of the last step (tiles x NB)
};

// Scalar slots per problem: bs[(p * 8 + k) * NB + c].
enum { B_RZ = 0, B_RR, B_BB, B_ACT, B_IT, B_ALPHA, B_BETA, B_MASK };

template <typename T>
void launch_b_spmm(hipStream_t s, const BProb<T>* probs, const int32_t* tile_prob, int ntiles, int TR, int G, int NB,
                   int mode, double* part, const int32_t* flags);
template <typename T>
void launch_b_iteration(hipStream_t s, const BProb<T>* probs, const int32_t* tile_prob, int ntiles, int K, int TR,
                        int G, int NB, double* part, double* bs, int32_t* flags, double rtol2, const BPoly& poly);
template <typename T>
void launch_b_start(hipStream_t s, const BProb<T>* probs, const int32_t* tile_prob, int ntiles, int K, int TR, int G,
                    int NB, double* part, double* bs, const double* mask_bs, int32_t* flags, double rtol2,
                    const BPoly& poly);
void launch_b_ir(hipStream_t s, const BProb<double>* p64, const BProb<float>* p32, const int32_t* tile_prob,
                 int ntiles, int TR, int op);

}  // namespace mlc
