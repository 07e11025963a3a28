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

// Additive coarse-space correction of one Hartree problem (one column).
struct BCoarse {
  const int32_t* PTptr;
  const int32_t* PTidx;
  const double* PTw;
  const int32_t* Pk;
  const double* Pw;
  const double* KHinv;  // nH x nH
  double* rH;
  double* eH;
  double* Zc;           // z when there is no polynomial preconditioner
  int64_t nH;
  int32_t row0;         // first global coarse row of this problem
  int32_t pad;
};

// The coarse corrections of a batched Hartree solve (coarse == null: none).
struct BCoarseSet {
  const BCoarse* coarse;
  const int32_t* crow_prob;  // global coarse row -> problem
  int64_t nrows;
};

// Scalar slots per problem: bs[(p * 8 + k) * NB + c].
enum { B_RZ = 0, B_RR, B_BB, B_ACT, B_IT, B_ALPHA, B_BETA, B_MASK };

template <typename T>
void launch_b_spmm(hipStream_t s, const BProb<T>* probs, const int32_t* tile_prob, int ntiles, int TR, int G, int NB,
                   int mode, double* part, const int32_t* flags);
template <typename T>
void launch_b_iteration(hipStream_t s, const BProb<T>* probs, const int32_t* tile_prob, int ntiles, int K, int TR,
                        int G, int NB, double* part, double* bs, int32_t* flags, double rtol2, const BPoly& poly,
                        const BCoarseSet* cs = nullptr);
template <typename T>
void launch_b_start(hipStream_t s, const BProb<T>* probs, const int32_t* tile_prob, int ntiles, int K, int TR, int G,
                    int NB, double* part, double* bs, const double* mask_bs, int32_t* flags, double rtol2,
                    const BPoly& poly, const BCoarseSet* cs = nullptr);
void launch_b_ir(hipStream_t s, const BProb<double>* p64, const BProb<float>* p32, const int32_t* tile_prob,
                 int ntiles, int TR, int op);

}  // namespace mlc
