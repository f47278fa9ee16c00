// Differentiation with respect to the network parameters and the Adam update.
#include "nep_common.h"

namespace nep {
namespace {

__global__ void k_adam(float* __restrict__ theta, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, int64_t n, double c1, double c2, double lr, double b1,
                       double b2, double eps) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double gk = g[k];
  const double a = b1 * (double)m1[k] + (1.0 - b1) * gk;
  const double b = b2 * (double)m2[k] + (1.0 - b2) * gk * gk;
  m1[k] = (float)a;
  m2[k] = (float)b;
  theta[k] = (float)((double)theta[k] - lr * (a / c1) / (sqrt(b / c2) + eps));
}

}  // namespace

hipError_t launch_adam(float* theta, const float* g, float* m1, float* m2, int64_t n, int64_t t, double lr,
                       double b1, double b2, double eps, hipStream_t st) {
  const double c1 = 1.0 - pow(b1, (double)t);
  const double c2 = 1.0 - pow(b2, (double)t);
  hipLaunchKernelGGL(k_adam, dim3(grid_blocks(n)), dim3(kBlock), 0, st, theta, g, m1, m2, n, c1, c2, lr, b1,
                     b2, eps);
  return hipGetLastError();
}

int train_partial_blocks(int64_t N) { return grid_blocks(N); }

hipError_t launch_train_forward(const ModelDev& m, const float* theta, const EvalBuffers& b,
                                hipStream_t st) {
  ModelDev mt = m;
  const int G = m.H * m.D;
  mt.W0 = theta;
  mt.b0 = theta + G;
  mt.w1 = theta + G + m.H;
  mt.b1 = theta + G + 2 * m.H;
  return launch_eval(mt, 0, b, st);
}

hipError_t launch_train_backward(const ModelDev&, const TrainBuffers&, hipStream_t) {
  return hipErrorNotSupported;
}

}  // namespace nep
