// The per-DoF network of the learned step-5 initial guess on gfx950:
// 6 -> 64 -> 64 -> 64 -> 1 with GELU, BF16 matrix products on the matrix
// cores (v_mfma_f32_16x16x16 bf16) with FP32 accumulation, FP32 master
// weights and Adam.
//
// Tiling: a wave handles 16 rows. Every hidden layer is computed transposed,
// H^T = W X^T, with the weights as the MFMA A operand and the activations as
// the B operand: then the accumulator of output block ob (lane l holds
// outputs 16 ob + 4 (l / 16) + i of row l % 16, i = 0..3) is exactly the B
// operand of input block ob of the next layer, and no data moves between
// layers. The backward pass forms dH = W^T dZ the same way; only the weight
// gradients dW = dZ H^T need the row index as the reduction index, for which
// each wave transposes its dZ and H tiles through LDS.
//
// Rounding: the products take bfloat16 operands (x, W1..W3, h1, h2, and in the
// backward pass dz1..dz3 and W2^T, W3^T), rounded to nearest even; GELU, the
// output layer (W4 . h3), the biases and every sum are FP32.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <vector>

#include "nn.h"

namespace mlc {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int BS = 256;  // 4 waves
constexpr float RSQRT2 = 0.70710678118654752440f;
constexpr float RSQRT2PI = 0.39894228040143267794f;

__device__ __forceinline__ short f2bf(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (short)((u >> 16) | 0x40u);  // keep NaN a NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * RSQRT2)); }
__device__ __forceinline__ float gelu_d(float z) {
  return 0.5f * (1.0f + erff(z * RSQRT2)) + z * expf(-0.5f * z * z) * RSQRT2PI;
}

__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x4 lds4(const unsigned short* p) { return *reinterpret_cast<const bf16x4*>(p); }

__device__ __forceinline__ int64_t src_row(int64_t j, uint64_t start, uint64_t stride, int64_t M) {
  return (int64_t)((start + (uint64_t)j * stride) % (uint64_t)M);
}

// Copy n16 16-byte chunks from global to LDS with the whole block.
__device__ __forceinline__ void to_lds(unsigned short* dst, const unsigned short* src, int n16) {
  const uint4* s = reinterpret_cast<const uint4*>(src);
  uint4* d = reinterpret_cast<uint4*>(dst);
  for (int k = threadIdx.x; k < n16; k += BS) d[k] = s[k];
}

// Forward of one 16-row tile by one wave. xb: B operand of the inputs.
// Keeps (if asked) z1..z3, the bf16 activations h1, h2 and h3.
struct Fwd {
  f32x4 z1[4], z2[4], z3[4], h3[4];
  bf16x4 h1b[4], h2b[4];
};

__device__ __forceinline__ void forward_tile(bf16x4 xb, const unsigned short* w1s, const unsigned short* w2s,
                                             const unsigned short* w3s, const float* fb, Fwd& f) {
  const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = mfma(lds4(w1s + (16 * ob + col) * 16 + 4 * grp), xb, acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float z = acc[i] + fb[NN_B1 - NN_B1 + 16 * ob + 4 * grp + i];
      f.z1[ob][i] = z;
      f.h1b[ob][i] = f2bf(gelu(z));
    }
  }
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) acc = mfma(lds4(w2s + (16 * ob + col) * 64 + 16 * kb + 4 * grp), f.h1b[kb], acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float z = acc[i] + fb[64 + 16 * ob + 4 * grp + i];
      f.z2[ob][i] = z;
      f.h2b[ob][i] = f2bf(gelu(z));
    }
  }
#pragma unroll
  for (int ob = 0; ob < 4; ++ob) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) acc = mfma(lds4(w3s + (16 * ob + col) * 64 + 16 * kb + 4 * grp), f.h2b[kb], acc);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float z = acc[i] + fb[128 + 16 * ob + 4 * grp + i];
      f.z3[ob][i] = z;
      f.h3[ob][i] = gelu(z);
    }
  }
}

// y for the tile's rows, in every lane of the row's column (l % 16).
__device__ __forceinline__ float output_tile(const Fwd& f, const float* fb) {
  const int grp = (threadIdx.x & 63) >> 4;
  float p = 0.f;
#pragma unroll
  for (int ob = 0; ob < 4; ++ob)
#pragma unroll
    for (int i = 0; i < 4; ++i) p += fb[192 + 16 * ob + 4 * grp + i] * f.h3[ob][i];
  p += __shfl_xor(p, 16, 64);
  p += __shfl_xor(p, 32, 64);
  return p + fb[256];
}

// B operand of the inputs of the tile row col = l % 16: inputs 4 (l / 16) + i.
__device__ __forceinline__ bf16x4 load_x(const float* __restrict__ X, int64_t src, bool valid) {
  const int grp = (threadIdx.x & 63) >> 4;
  bf16x4 xb = {0, 0, 0, 0};
  if (valid && grp < 2) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      int in = 4 * grp + i;
      if (in < 6) xb[i] = f2bf(X[src * 6 + in]);
    }
  }
  return xb;
}

// FP32 scalars of the tables: b1, b2, b3, W4, b4 (257 values).
__device__ __forceinline__ void load_fb(float* fb, const float* theta) {
  for (int k = threadIdx.x; k < 257; k += BS) {
    float v;
    if (k < 64) v = theta[NN_B1 + k];
    else if (k < 128) v = theta[NN_B2 + k - 64];
    else if (k < 192) v = theta[NN_B3 + k - 128];
    else if (k < 256) v = theta[NN_W4 + k - 192];
    else v = theta[NN_B4];
    fb[k] = v;
  }
}

__global__ void __launch_bounds__(BS) k_nn_prepare(NnDev d) {
  int k = blockIdx.x * BS + threadIdx.x;
  if (k < 64 * 16) {
    int o = k / 16, i = k % 16;
    d.w1b[k] = i < 6 ? (unsigned short)f2bf(d.theta[NN_W1 + o * 6 + i]) : 0;
  }
  if (k < 64 * 64) {
    int o = k / 64, i = k % 64;
    unsigned short a = (unsigned short)f2bf(d.theta[NN_W2 + k]);
    unsigned short b = (unsigned short)f2bf(d.theta[NN_W3 + k]);
    d.w2b[k] = a;
    d.w3b[k] = b;
    d.w2t[i * 64 + o] = a;
    d.w3t[i * 64 + o] = b;
  }
}

__global__ void __launch_bounds__(BS) k_nn_forward(NnDev d, const float* __restrict__ X, int64_t m, uint64_t start,
                                                   uint64_t stride, int64_t M, float* __restrict__ Y) {
  __shared__ __attribute__((aligned(16))) unsigned short w1s[64 * 16];
  __shared__ __attribute__((aligned(16))) unsigned short w2s[64 * 64];
  __shared__ __attribute__((aligned(16))) unsigned short w3s[64 * 64];
  __shared__ float fb[257];
  to_lds(w1s, d.w1b, 64 * 16 / 8);
  to_lds(w2s, d.w2b, 64 * 64 / 8);
  to_lds(w3s, d.w3b, 64 * 64 / 8);
  load_fb(fb, d.theta);
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, col = lane & 15, grp = lane >> 4;
  const int64_t ntiles = (m + 15) / 16;
  for (int64_t tile = (int64_t)blockIdx.x * 4 + wid; tile < ntiles; tile += (int64_t)gridDim.x * 4) {
    const int64_t j = tile * 16 + col;
    const bool valid = j < m;
    const int64_t src = valid ? src_row(j, start, stride, M) : 0;
    Fwd f;
    forward_tile(load_x(X, src, valid), w1s, w2s, w3s, fb, f);
    float y = output_tile(f, fb);
    if (grp == 0 && valid) Y[j] = y;
  }
}

// Gradient partials of one block: all waves walk the block's tiles in step
// (tiles past the end contribute zero), so that the LDS transposes can use
// block barriers.
__global__ void __launch_bounds__(BS) k_nn_grad(NnDev d, const float* __restrict__ X, const float* __restrict__ T,
                                                int64_t m, uint64_t start, uint64_t stride, int64_t M) {
  __shared__ __attribute__((aligned(16))) unsigned short w1s[64 * 16];
  __shared__ __attribute__((aligned(16))) unsigned short w2s[64 * 64];
  __shared__ __attribute__((aligned(16))) unsigned short w3s[64 * 64];
  __shared__ __attribute__((aligned(16))) unsigned short w2t[64 * 64];
  __shared__ __attribute__((aligned(16))) unsigned short w3t[64 * 64];
  __shared__ __attribute__((aligned(16))) unsigned short tdz[4][64 * 16];
  __shared__ __attribute__((aligned(16))) unsigned short th[4][64 * 16];
  __shared__ float fb[257];
  __shared__ float red[NN_NPARAM];
  __shared__ double lred[4];
  to_lds(w1s, d.w1b, 64 * 16 / 8);
  to_lds(w2s, d.w2b, 64 * 64 / 8);
  to_lds(w3s, d.w3b, 64 * 64 / 8);
  to_lds(w2t, d.w2t, 64 * 64 / 8);
  to_lds(w3t, d.w3t, 64 * 64 / 8);
  load_fb(fb, d.theta);
  for (int k = threadIdx.x; k < NN_NPARAM; k += BS) red[k] = 0.f;
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, col = lane & 15, grp = lane >> 4;
  unsigned short* tz = tdz[wid];
  unsigned short* tx = th[wid];
  f32x4 gW1[4], gW2[4][4], gW3[4][4];
  float gb1[16], gb2[16], gb3[16], gW4[16];
  float gb4 = 0.f;
  double lsum = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    gW1[a] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      gW2[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
      gW3[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) gb1[k] = gb2[k] = gb3[k] = gW4[k] = 0.f;
  const float inv_m = 2.0f / (float)m;
  const int64_t ntiles = (m + 15) / 16;
  for (int64_t bt = blockIdx.x; bt * 4 < ntiles; bt += gridDim.x) {
    const int64_t tile = bt * 4 + wid;
    const int64_t j = tile * 16 + col;
    const bool valid = tile < ntiles && j < m;
    const int64_t src = valid ? src_row(j, start, stride, M) : 0;
    Fwd f;
    forward_tile(load_x(X, src, valid), w1s, w2s, w3s, fb, f);
    const float y = output_tile(f, fb);
    const float e = valid ? y - T[src] : 0.f;
    if (grp == 0) lsum += (double)e * (double)e;
    const float dy = e * inv_m;
    if (grp == 0) gb4 += dy;
    // layer 3: dz3 = W4 dy * gelu'(z3)
    bf16x4 dzb[4];
#pragma unroll
    for (int ob = 0; ob < 4; ++ob)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int o = 16 * ob + 4 * grp + i;
        gW4[4 * ob + i] += dy * f.h3[ob][i];
        float dz = fb[192 + o] * dy * gelu_d(f.z3[ob][i]);
        gb3[4 * ob + i] += dz;
        dzb[ob][i] = f2bf(dz);
        tz[o * 16 + col] = (unsigned short)dzb[ob][i];
        tx[o * 16 + col] = (unsigned short)f.h2b[ob][i];
      }
    __syncthreads();
    // gW3 += dz3 h2^T: A[out][row] from tz, B[row][in] from tx
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
      bf16x4 a = lds4(tz + (16 * ob + col) * 16 + 4 * grp);
#pragma unroll
      for (int ib = 0; ib < 4; ++ib) gW3[ob][ib] = mfma(a, lds4(tx + (16 * ib + col) * 16 + 4 * grp), gW3[ob][ib]);
    }
    // layer 2: dz2 = (W3^T dz3) * gelu'(z2)
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) acc = mfma(lds4(w3t + (16 * mb + col) * 64 + 16 * kb + 4 * grp), dzb[kb], acc);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float dz = acc[i] * gelu_d(f.z2[mb][i]);
        gb2[4 * mb + i] += dz;
        f.z2[mb][i] = dz;  // reuse: dz2
      }
    }
    __syncthreads();
#pragma unroll
    for (int ob = 0; ob < 4; ++ob)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int o = 16 * ob + 4 * grp + i;
        dzb[ob][i] = f2bf(f.z2[ob][i]);
        tz[o * 16 + col] = (unsigned short)dzb[ob][i];
        tx[o * 16 + col] = (unsigned short)f.h1b[ob][i];
      }
    __syncthreads();
#pragma unroll
    for (int ob = 0; ob < 4; ++ob) {
      bf16x4 a = lds4(tz + (16 * ob + col) * 16 + 4 * grp);
#pragma unroll
      for (int ib = 0; ib < 4; ++ib) gW2[ob][ib] = mfma(a, lds4(tx + (16 * ib + col) * 16 + 4 * grp), gW2[ob][ib]);
    }
    // layer 1: dz1 = (W2^T dz2) * gelu'(z1)
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) acc = mfma(lds4(w2t + (16 * mb + col) * 64 + 16 * kb + 4 * grp), dzb[kb], acc);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float dz = acc[i] * gelu_d(f.z1[mb][i]);
        gb1[4 * mb + i] += dz;
        f.z1[mb][i] = dz;  // reuse: dz1
      }
    }
    __syncthreads();
#pragma unroll
    for (int ob = 0; ob < 4; ++ob)
#pragma unroll
      for (int i = 0; i < 4; ++i) tz[(16 * ob + 4 * grp + i) * 16 + col] = (unsigned short)f2bf(f.z1[ob][i]);
    __syncthreads();
    // gW1 += dz1 x^T: B[row][in] = x of tile row 4 (l / 16) + i, input l % 16
    {
      bf16x4 bx = {0, 0, 0, 0};
      if (col < 6) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int64_t jr = tile * 16 + 4 * grp + i;
          if (tile < ntiles && jr < m) bx[i] = f2bf(X[src_row(jr, start, stride, M) * 6 + col]);
        }
      }
#pragma unroll
      for (int ob = 0; ob < 4; ++ob) gW1[ob] = mfma(lds4(tz + (16 * ob + col) * 16 + 4 * grp), bx, gW1[ob]);
    }
    __syncthreads();
  }
  // bias and W4 gradients: sum over the 16 rows (lanes of equal l / 16)
#pragma unroll
  for (int k = 0; k < 16; ++k) {
#pragma unroll
    for (int off = 1; off < 16; off <<= 1) {
      gb1[k] += __shfl_xor(gb1[k], off, 64);
      gb2[k] += __shfl_xor(gb2[k], off, 64);
      gb3[k] += __shfl_xor(gb3[k], off, 64);
      gW4[k] += __shfl_xor(gW4[k], off, 64);
    }
  }
  for (int off = 1; off < 64; off <<= 1) {
    gb4 += __shfl_xor(gb4, off, 64);
    lsum += __shfl_xor(lsum, off, 64);
  }
  // the waves add their accumulators into red one after the other
  for (int w = 0; w < 4; ++w) {
    if (wid == w) {
#pragma unroll
      for (int ob = 0; ob < 4; ++ob)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int o = 16 * ob + 4 * grp + i;
          if (col < 6) red[NN_W1 + o * 6 + col] += gW1[ob][i];
#pragma unroll
          for (int ib = 0; ib < 4; ++ib) {
            red[NN_W2 + o * 64 + 16 * ib + col] += gW2[ob][ib][i];
            red[NN_W3 + o * 64 + 16 * ib + col] += gW3[ob][ib][i];
          }
          if (col == 0) {
            red[NN_B1 + o] += gb1[4 * ob + i];
            red[NN_B2 + o] += gb2[4 * ob + i];
            red[NN_B3 + o] += gb3[4 * ob + i];
            red[NN_W4 + o] += gW4[4 * ob + i];
          }
        }
      if (lane == 0) {
        red[NN_B4] += gb4;
        lred[w] = lsum;
      }
    }
    __syncthreads();
  }
  float* gp = d.gpart + (int64_t)blockIdx.x * NN_NPARAM;
  for (int k = threadIdx.x; k < NN_NPARAM; k += BS) gp[k] = red[k];
  if (threadIdx.x == 0) d.lpart[blockIdx.x] = (lred[0] + lred[1]) + (lred[2] + lred[3]);
}

// grad = sum of the block partials in block order; loss[slot] = sum / m.
__global__ void __launch_bounds__(BS) k_nn_reduce(NnDev d, int nblk, int64_t m, int slot) {
  int k = blockIdx.x * BS + threadIdx.x;
  if (k < NN_NPARAM) {
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += d.gpart[(int64_t)b * NN_NPARAM + k];
    d.grad[k] = s;
  }
  if (k == 0) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += d.lpart[b];
    d.loss[slot] = s / (double)m;
  }
}

// Adam on theta with d.grad; refreshes the bf16 tables of the updated entries.
__global__ void __launch_bounds__(BS) k_nn_adam(NnDev d, float lr, float b1, float b2, float eps, float c1,
                                                float c2) {
  int k = blockIdx.x * BS + threadIdx.x;
  if (k >= NN_NPARAM) return;
  float g = d.grad[k];
  float mk = b1 * d.m[k] + (1.0f - b1) * g;
  float vk = b2 * d.v[k] + (1.0f - b2) * g * g;
  d.m[k] = mk;
  d.v[k] = vk;
  float th = d.theta[k] - lr * (mk * c1) / (sqrtf(vk * c2) + eps);
  d.theta[k] = th;
  unsigned short hb = (unsigned short)f2bf(th);
  if (k < NN_B1) {
    d.w1b[(k / 6) * 16 + k % 6] = hb;
  } else if (k >= NN_W2 && k < NN_B2) {
    int q = k - NN_W2, o = q / 64, i = q % 64;
    d.w2b[q] = hb;
    d.w2t[i * 64 + o] = hb;
  } else if (k >= NN_W3 && k < NN_B3) {
    int q = k - NN_W3, o = q / 64, i = q % 64;
    d.w3b[q] = hb;
    d.w3t[i * 64 + o] = hb;
  }
}

inline int grad_blocks(int64_t m) {
  int64_t tiles = (m + 15) / 16;
  int64_t b = (tiles + 3) / 4;
  return (int)(b < 1 ? 1 : (b > NN_GRAD_MAX_BLOCKS ? NN_GRAD_MAX_BLOCKS : b));
}

}  // namespace

void launch_nn_prepare(hipStream_t s, const NnDev& d) {
  hipLaunchKernelGGL(k_nn_prepare, dim3((64 * 64 + BS - 1) / BS), dim3(BS), 0, s, d);
}

void launch_nn_forward(hipStream_t s, const NnDev& d, const float* X, int64_t m, uint64_t start, uint64_t stride,
                       int64_t M, float* Y) {
  if (m <= 0) return;
  // at most four blocks per CU: every block stages the weights in LDS once and
  // its waves then stride over many 16-row tiles
  int64_t tiles = (m + 15) / 16;
  int64_t b = (tiles + 3) / 4;
  int nb = (int)(b > 1024 ? 1024 : b);
  hipLaunchKernelGGL(k_nn_forward, dim3(nb), dim3(BS), 0, s, d, X, m, start, stride, M, Y);
}

void launch_nn_grad(hipStream_t s, const NnDev& d, const float* X, const float* T, int64_t m, uint64_t start,
                    uint64_t stride, int64_t M, int slot) {
  int nb = grad_blocks(m);
  hipLaunchKernelGGL(k_nn_grad, dim3(nb), dim3(BS), 0, s, d, X, T, m, start, stride, M);
  hipLaunchKernelGGL(k_nn_reduce, dim3((NN_NPARAM + BS - 1) / BS), dim3(BS), 0, s, d, nb, m, slot);
}

// ---- device-resident scratch of the allocation-free loss/gradient call ------
// Per-block gradient partials (NN_GRAD_MAX_BLOCKS x NN_NPARAM floats), loss
// partials (NN_GRAD_MAX_BLOCKS doubles), the reduced gradient (NN_NPARAM
// floats) and the loss (one double), each at a 256-byte boundary. Every GPU
// the library runs on holds one copy until the process ends; calls on one GPU
// share it.
namespace {
constexpr size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
constexpr size_t SCR_GPART = 0;
constexpr size_t SCR_LPART = align256(SCR_GPART + sizeof(float) * (size_t)NN_GRAD_MAX_BLOCKS * NN_NPARAM);
constexpr size_t SCR_GRAD = align256(SCR_LPART + sizeof(double) * NN_GRAD_MAX_BLOCKS);
constexpr size_t SCR_LOSS = align256(SCR_GRAD + sizeof(float) * NN_NPARAM);
constexpr size_t SCR_BYTES = align256(SCR_LOSS + sizeof(double));
}  // namespace

static __device__ __align__(256) unsigned char scratch[SCR_BYTES];

size_t nn_static_scratch_bytes() { return SCR_BYTES; }

hipError_t nn_static_scratch(int device, NnDev* d) {
  // the array's address on each device, looked up once per device with that
  // device current (the host-side name is a stand-in, not a device address)
  static std::mutex mu;
  static std::vector<void*> addr;
  std::lock_guard<std::mutex> lock(mu);
  if (device < 0) return hipErrorInvalidDevice;
  if ((int)addr.size() <= device) addr.resize(device + 1, nullptr);
  if (!addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[device] = p;
  }
  char* base = static_cast<char*>(addr[device]);
  d->gpart = reinterpret_cast<float*>(base + SCR_GPART);
  d->lpart = reinterpret_cast<double*>(base + SCR_LPART);
  d->grad = reinterpret_cast<float*>(base + SCR_GRAD);
  d->loss = reinterpret_cast<double*>(base + SCR_LOSS);
  return hipSuccess;
}

void launch_nn_adam(hipStream_t s, const NnDev& d, float lr, float beta1, float beta2, float eps, float c1, float c2) {
  hipLaunchKernelGGL(k_nn_adam, dim3((NN_NPARAM + BS - 1) / BS), dim3(BS), 0, s, d, lr, beta1, beta2, eps, c1, c2);
}

}  // namespace mlc
