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
  int64_t n;
  int32_t N;
  int32_t tile0;
  int32_t ntiles;
  int32_t pad;
};

// Scalar slots per problem: bs[(p * 8 + k) * NB + c].
enum { B_RZ = 0, B_RR, B_BB, B_ACT, B_IT, B_ALPHA, B_BETA, B_MASK };

template <typename T>
void launch_b_spmm(hipStream_t s, const BProb<T>* probs, const int32_t* tile_prob, int ntiles, int TR, int G, int NB,
                   int mode, double* part, const int32_t* flags);
template <typename T>
void launch_b_iteration(hipStream_t s, const BProb<T>* probs, const int32_t* tile_prob, int ntiles, int K, int TR,
                        int G, int NB, double* part, double* bs, int32_t* flags, double rtol2);
template <typename T>
void launch_b_start(hipStream_t s, const BProb<T>* probs, const int32_t* tile_prob, int ntiles, int K, int TR, int G,
                    int NB, double* part, double* bs, const double* mask_bs, int32_t* flags, double rtol2);
void launch_b_ir(hipStream_t s, const BProb<double>* p64, const BProb<float>* p32, const int32_t* tile_prob,
                 int ntiles, int TR, int op);

}  // namespace mlc
