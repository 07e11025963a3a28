// The extern "C" entry points of the learned initial guess network.
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "mlc_internal.h"
#include "nn.h"

struct mlc_nn {
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  bool bound = false;
  bool has_params = false;
  int64_t t = 0;  // Adam steps taken
  mlc::NnDev d;
  std::string err;
};

namespace {

using mlc::NnDev;

size_t nn_layout(NnDev* d, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    off = (off + 255) & ~size_t(255);
    char* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  const size_t P = mlc::NN_NPARAM;
  d->theta = reinterpret_cast<float*>(take(P * 4));
  d->m = reinterpret_cast<float*>(take(P * 4));
  d->v = reinterpret_cast<float*>(take(P * 4));
  d->grad = reinterpret_cast<float*>(take(P * 4));
  d->w1b = reinterpret_cast<unsigned short*>(take(64 * 16 * 2));
  d->w2b = reinterpret_cast<unsigned short*>(take(64 * 64 * 2));
  d->w3b = reinterpret_cast<unsigned short*>(take(64 * 64 * 2));
  d->w2t = reinterpret_cast<unsigned short*>(take(64 * 64 * 2));
  d->w3t = reinterpret_cast<unsigned short*>(take(64 * 64 * 2));
  d->gpart = reinterpret_cast<float*>(take((size_t)mlc::NN_GRAD_MAX_BLOCKS * P * 4));
  d->lpart = reinterpret_cast<double*>(take(mlc::NN_GRAD_MAX_BLOCKS * 8));
  d->loss = reinterpret_cast<double*>(take((size_t)mlc::NN_MAX_STEPS * 8));
  return off + 256;
}

mlc_status nfail(mlc_nn* nn, mlc_status s, const std::string& m) {
  nn->err = m;
  return s;
}

#define NCHK(x)                                                                                     \
  do {                                                                                              \
    hipError_t e_ = (x);                                                                            \
    if (e_ != hipSuccess) return nfail(nn, MLC_ERR_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

mlc_status ready(mlc_nn* nn) {
  if (!nn->bound) return nfail(nn, MLC_ERR_STATE, "network not bound");
  if (!nn->has_params) return nfail(nn, MLC_ERR_STATE, "parameters not set");
  return MLC_OK;
}

uint64_t coprime_stride(int64_t M) {
  if (M <= 1) return 1;
  uint64_t s = (uint64_t)(0x9E3779B97F4A7C15ull % (uint64_t)M) | 1ull;
  while (std::gcd(s, (uint64_t)M) != 1) s += 2;
  return s % (uint64_t)M == 0 ? 1 : s;
}

}  // namespace

namespace mlc {
const NnDev* nn_device(const mlc_nn* nn) { return nn && nn->bound && nn->has_params ? &nn->d : nullptr; }
}  // namespace mlc

extern "C" {

mlc_status mlc_nn_create(mlc_nn** out) {
  if (!out) return MLC_ERR_ARG;
  mlc_nn* nn = new mlc_nn();
  nn->ws_bytes = nn_layout(&nn->d, nullptr);
  *out = nn;
  return MLC_OK;
}

mlc_status mlc_nn_workspace_bytes(const mlc_nn* nn, size_t* bytes) {
  if (!nn || !bytes) return MLC_ERR_ARG;
  *bytes = nn->ws_bytes;
  return MLC_OK;
}

mlc_status mlc_nn_bind(mlc_nn* nn, void* workspace, size_t bytes, void* stream) {
  if (!nn || !workspace) return MLC_ERR_ARG;
  if (bytes < nn->ws_bytes) return nfail(nn, MLC_ERR_WORKSPACE, "network workspace too small");
  if ((reinterpret_cast<uintptr_t>(workspace) & 255) != 0)
    return nfail(nn, MLC_ERR_WORKSPACE, "network workspace must be 256-byte aligned");
  nn->ws = static_cast<char*>(workspace);
  nn->stream = static_cast<hipStream_t>(stream);
  nn_layout(&nn->d, nn->ws);
  nn->bound = true;
  nn->has_params = false;
  return MLC_OK;
}

mlc_status mlc_nn_set_params(mlc_nn* nn, const float* theta) {
  if (!nn || !theta) return MLC_ERR_ARG;
  if (!nn->bound) return nfail(nn, MLC_ERR_STATE, "network not bound");
  for (int k = 0; k < mlc::NN_NPARAM; ++k)
    if (!std::isfinite(theta[k])) return nfail(nn, MLC_ERR_NONFINITE, "non-finite parameter");
  hipStream_t s = nn->stream;
  const size_t P = mlc::NN_NPARAM * sizeof(float);
  NCHK(hipMemcpyAsync(nn->d.theta, theta, P, hipMemcpyHostToDevice, s));
  NCHK(hipMemsetAsync(nn->d.m, 0, P, s));
  NCHK(hipMemsetAsync(nn->d.v, 0, P, s));
  mlc::launch_nn_prepare(s, nn->d);
  NCHK(hipGetLastError());
  NCHK(hipStreamSynchronize(s));
  nn->t = 0;
  nn->has_params = true;
  return MLC_OK;
}

mlc_status mlc_nn_get_params(mlc_nn* nn, float* theta) {
  if (!nn || !theta) return MLC_ERR_ARG;
  mlc_status st = ready(nn);
  if (st != MLC_OK) return st;
  NCHK(hipMemcpyAsync(theta, nn->d.theta, mlc::NN_NPARAM * sizeof(float), hipMemcpyDeviceToHost, nn->stream));
  NCHK(hipStreamSynchronize(nn->stream));
  return MLC_OK;
}

mlc_status mlc_nn_forward(mlc_nn* nn, const float* x, int64_t rows, float* y) {
  if (!nn || rows < 0 || (rows > 0 && (!x || !y))) return MLC_ERR_ARG;
  mlc_status st = ready(nn);
  if (st != MLC_OK) return st;
  mlc::launch_nn_forward(nn->stream, nn->d, x, rows, 0, 1, rows > 0 ? rows : 1, y);
  NCHK(hipGetLastError());
  return MLC_OK;
}

mlc_status mlc_nn_loss_grad(mlc_nn* nn, const float* x, const float* t, int64_t rows, double* loss, float* grad) {
  if (!nn || !x || !t || rows < 1 || !loss || !grad) return MLC_ERR_ARG;
  mlc_status st = ready(nn);
  if (st != MLC_OK) return st;
  hipStream_t s = nn->stream;
  mlc::launch_nn_grad(s, nn->d, x, t, rows, 0, 1, rows, 0);
  NCHK(hipGetLastError());
  NCHK(hipMemcpyAsync(grad, nn->d.grad, mlc::NN_NPARAM * sizeof(float), hipMemcpyDeviceToHost, s));
  NCHK(hipMemcpyAsync(loss, nn->d.loss, sizeof(double), hipMemcpyDeviceToHost, s));
  NCHK(hipStreamSynchronize(s));
  return MLC_OK;
}

mlc_status mlc_nn_loss_grad_noalloc(mlc_nn* nn, const float* x, const float* t, int64_t rows, double* loss,
                                    float* grad) {
  if (!nn || !x || !t || rows < 1 || !loss || !grad) return MLC_ERR_ARG;
  if (rows > mlc::NN_STATIC_MAX_ROWS)
    return nfail(nn, MLC_ERR_ARG, "rows above the allocation-free call's limit (2^31 - 1)");
  mlc_status st = ready(nn);
  if (st != MLC_OK) return st;
  hipStream_t s = nn->stream;
  hipDevice_t dev = -1;  // the GPU the network's stream runs on (the null stream: the current device)
  if (s)
    NCHK(hipStreamGetDevice(s, &dev));
  else
    NCHK(hipGetDevice(&dev));
  // the network's parameters and bf16 tables from its workspace; partials,
  // gradient and loss in the device-resident scratch of this GPU
  mlc::NnDev d = nn->d;
  NCHK(mlc::nn_static_scratch(dev, &d));
  mlc::launch_nn_grad(s, d, x, t, rows, 0, 1, rows, 0);
  NCHK(hipGetLastError());
  NCHK(hipMemcpyAsync(grad, d.grad, mlc::NN_NPARAM * sizeof(float), hipMemcpyDeviceToHost, s));
  NCHK(hipMemcpyAsync(loss, d.loss, sizeof(double), hipMemcpyDeviceToHost, s));
  NCHK(hipStreamSynchronize(s));
  return MLC_OK;
}

mlc_status mlc_nn_adam(mlc_nn* nn, const float* grad, double lr, double beta1, double beta2, double eps) {
  if (!nn || !grad || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return MLC_ERR_ARG;
  mlc_status st = ready(nn);
  if (st != MLC_OK) return st;
  hipStream_t s = nn->stream;
  NCHK(hipMemcpyAsync(nn->d.grad, grad, mlc::NN_NPARAM * sizeof(float), hipMemcpyHostToDevice, s));
  ++nn->t;
  const double c1 = 1.0 / (1.0 - std::pow(beta1, (double)nn->t));
  const double c2 = 1.0 / (1.0 - std::pow(beta2, (double)nn->t));
  mlc::launch_nn_adam(s, nn->d, (float)lr, (float)beta1, (float)beta2, (float)eps, (float)c1, (float)c2);
  NCHK(hipGetLastError());
  NCHK(hipStreamSynchronize(s));
  return MLC_OK;
}

mlc_status mlc_nn_train(mlc_nn* nn, const float* x, const float* t, int64_t rows, int32_t steps, int32_t batch,
                        double lr, float* loss_history) {
  if (!nn || !x || !t || rows < 1 || steps < 1 || steps > mlc::NN_MAX_STEPS || batch < 1 || !(lr > 0))
    return MLC_ERR_ARG;
  mlc_status st = ready(nn);
  if (st != MLC_OK) return st;
  hipStream_t s = nn->stream;
  const uint64_t stride = coprime_stride(rows);
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  for (int k = 0; k < steps; ++k) {
    // sample g = k * batch + j of the run is row (g * stride) mod rows: every
    // row once per pass over the data, in a scattered order
    const uint64_t g0 = (uint64_t)k * (uint64_t)batch % (uint64_t)rows;
    const uint64_t start = (uint64_t)((unsigned __int128)g0 * stride % (uint64_t)rows);
    mlc::launch_nn_grad(s, nn->d, x, t, batch, start, stride, rows, k);
    ++nn->t;
    const double c1 = 1.0 / (1.0 - std::pow(b1, (double)nn->t));
    const double c2 = 1.0 / (1.0 - std::pow(b2, (double)nn->t));
    mlc::launch_nn_adam(s, nn->d, (float)lr, (float)b1, (float)b2, (float)eps, (float)c1, (float)c2);
  }
  NCHK(hipGetLastError());
  if (loss_history) {
    std::vector<double> h(steps);
    NCHK(hipMemcpyAsync(h.data(), nn->d.loss, sizeof(double) * steps, hipMemcpyDeviceToHost, s));
    NCHK(hipStreamSynchronize(s));
    for (int k = 0; k < steps; ++k) loss_history[k] = (float)h[k];
  } else {
    NCHK(hipStreamSynchronize(s));
  }
  return MLC_OK;
}

const char* mlc_nn_last_error(const mlc_nn* nn) { return nn ? nn->err.c_str() : "null network"; }

void mlc_nn_destroy(mlc_nn* nn) { delete nn; }

}  // extern "C"
