// The per-DoF network of the learned step-5 initial guess: device tables and
// launchers. Not part of the ABI.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace mlc {

// Packed parameter vector (FP32 master copy), offsets in floats:
// W1 (64 x 6, out x in), b1, W2 (64 x 64), b2, W3 (64 x 64), b3, W4 (64), b4.
enum : int {
  NN_W1 = 0,
  NN_B1 = 384,
  NN_W2 = 448,
  NN_B2 = 4544,
  NN_W3 = 4608,
  NN_B3 = 8704,
  NN_W4 = 8768,
  NN_B4 = 8832,
  NN_NPARAM = 8833
};

struct NnDev {
  float* theta = nullptr;           // 8833 FP32 master parameters
  float* m = nullptr;               // Adam first moments
  float* v = nullptr;               // Adam second moments
  float* grad = nullptr;            // reduced gradient
  unsigned short* w1b = nullptr;    // 64 x 16 bf16 (inputs 6..15 zero)
  unsigned short* w2b = nullptr;    // 64 x 64 bf16, [out][in]
  unsigned short* w3b = nullptr;
  unsigned short* w2t = nullptr;    // 64 x 64 bf16, [in][out]
  unsigned short* w3t = nullptr;
  float* gpart = nullptr;           // per-block gradient partials (max blocks x 8833)
  double* lpart = nullptr;          // per-block loss partials
  double* loss = nullptr;           // loss history (max steps)
};

constexpr int NN_GRAD_MAX_BLOCKS = 256;
constexpr int NN_MAX_STEPS = 100000;
constexpr int64_t NN_STATIC_MAX_ROWS = 2147483647;

// bf16 tables from theta (all of them; zero padding of w1b).
void launch_nn_prepare(hipStream_t s, const NnDev& d);
// Y[j] = NN(X[row(j)]) for j < m, row(j) = (start + j * stride) mod M.
void launch_nn_forward(hipStream_t s, const NnDev& d, const float* X, int64_t m, uint64_t start, uint64_t stride,
                       int64_t M, float* Y);
// Gradient of mean((NN(X[row(j)]) - T[row(j)])^2) over j < m into d.grad,
// the loss into d.loss[slot].
void launch_nn_grad(hipStream_t s, const NnDev& d, const float* X, const float* T, int64_t m, uint64_t start,
                    uint64_t stride, int64_t M, int slot);
// The allocation-free loss/gradient call's scratch: a device-resident array of
// nn_static_scratch_bytes() bytes per GPU; sets d->gpart, lpart, grad and loss
// to its parts on the given device (its address is looked up once per device).
size_t nn_static_scratch_bytes();
hipError_t nn_static_scratch(int device, NnDev* d);
// One Adam step with d.grad; c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t).
void launch_nn_adam(hipStream_t s, const NnDev& d, float lr, float beta1, float beta2, float eps, float c1, float c2);

}  // namespace mlc
