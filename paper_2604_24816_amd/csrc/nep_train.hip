// Differentiation of L = gE * E + sum_i gF_i . F_i with respect to the network
// parameters theta = (W0, b0, w1, b1), and the Adam update.
//
// With F = -dE/dx, sum_i gF_i . F_i = -sum_a dU_a/dq_a . v_a where
// v_a = sum_j dq_a/dr_aj . (gF_j - gF_a) is the descriptor JVP along gF.
// Writing q~ = sigma q, v~ = sigma v, h = W0 q~ - b0, t = tanh h, d = 1 - t^2 and
// z = W0 v~, the per-atom contributions are
//   dL/dW0 = alpha q~^T - beta v~^T,  alpha = gE w1 d + 2 z w1 t d,  beta = w1 d
//   dL/db0 = -alpha,  dL/dw1 = gE t - z d,  dL/db1 = -gE,
// summed over atoms. k_train_backward recomputes the descriptors of each center,
// evaluates the JVP over the same pair lists as the force kernel, and reduces
// the outer products over the 64 centers of a wavefront with FP32 MFMA
// (atoms as the K dimension), then over workgroups in FP64.
#include "nep_kernels.h"

namespace nep {
namespace {

using namespace kern;

constexpr int kGW = 32 * 32;        // gW0 tile, hidden-major, padded
constexpr int kGB0 = kGW;           // 32 sums of alpha
constexpr int kGW1 = kGW + 32;      // 32 sums of gE t - z d
constexpr int kGradStride = kGW + 64 + 1;

template <class S, bool MULTI>
__global__ void __launch_bounds__(kBlock, 1)
k_train_backward(ModelDev m, EvalBuffers b, const float* __restrict__ gF, double gE,
                 double* __restrict__ gpart) {
  __shared__ float tA[kBlock / 64][64 * kLdsStride];
  __shared__ float tB[kBlock / 64][64 * kLdsStride];
  constexpr int NR = S::NR, NA = S::NA, NC = S::NC, D = S::D, H = S::H;
  const int64_t N = b.N;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t i = (int64_t)tile * kBlock + threadIdx.x;
  const bool valid = i < N;
  const double* __restrict__ x = b.x;
  const double Lx = b.box[0], Ly = b.box[1], Lz = b.box[2];
  const float rcR_inv = 1.f / m.rcR, rcA_inv = 1.f / m.rcA;

  float q[D], v[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    q[k] = 0.f;
    v[k] = 0.f;
  }
  if (valid) {
    float s[NA * NC];
#pragma unroll
    for (int k = 0; k < NA * NC; ++k) s[k] = 0.f;
    const int ti = MULTI ? b.type[i] : 0;
    const double xi = x[i], yi = x[N + i], zi = x[2 * N + i];
    int nr = 0, na = 0;
    desc_accumulate<S, MULTI>(m, b, i, ti, xi, yi, zi, Lx, Ly, Lz, q, s, nr, na);
    const double rcR2 = m.rcR64 * m.rcR64, rcA2 = m.rcA64 * m.rcA64;
    desc_finish<S>(s, q);
    if (gF) {
      const float wi0 = gF[i], wi1 = gF[N + i], wi2 = gF[2 * N + i];
      // radial JVP: dq_n/dr_ij . w = g_n'(r) (u . w)
      const int kR = radial_bound(b, i);
      for (int p = 0; p < kR; ++p) {
        const int32_t j = b.nbr[(int64_t)p * N + i];
        float dx, dy, dz;
        if (!pair_inside(x, N, j, xi, yi, zi, Lx, Ly, Lz, rcR2, dx, dy, dz)) continue;
        const float r = sqrtf(dx * dx + dy * dy + dz * dz);
        const float rinv = 1.f / r;
        const int tj = MULTI ? b.type[j] : 0;
        float g[NR], dg[NR];
        radial_g_dg<NR, S::KR>(r, rcR_inv, m.cR + (ti * m.T + tj) * NR * S::KR, g, dg);
        const float uw = ((gF[j] - wi0) * dx + (gF[N + j] - wi1) * dy + (gF[2 * N + j] - wi2) * dz) * rinv;
#pragma unroll
        for (int n = 0; n < NR; ++n) v[n] = fmaf(dg[n], uw, v[n]);
      }
      // angular JVP: dq_nl = sum_m 2 W_lm s_nlm ds_nlm, dq4_n = sum_k (d q4/d s_k) ds_k, with
      // ds_nlm = g_n' (u.w) P_lm + g_n (grad P_lm . w - l P_lm (u.w)) / r
      float d4[S::FB ? NA * 5 : 1];
      if constexpr (S::FB) {
#pragma unroll
        for (int n = 0; n < NA; ++n) fourbody_ds(s + n * NC, d4 + 5 * n);
      }
#pragma unroll
      for (int n = 0; n < NA; ++n)
#pragma unroll
        for (int lm = 0; lm < NC; ++lm) s[n * NC + lm] *= 2.f * kW[lm];
      const int kA = angular_bound(b, i);
      for (int p = 0; p < kA; ++p) {
        const int32_t j = b.nbr[(int64_t)p * N + i];
        float dx, dy, dz;
        if (!pair_inside(x, N, j, xi, yi, zi, Lx, Ly, Lz, rcA2, dx, dy, dz)) continue;
        const float r = sqrtf(dx * dx + dy * dy + dz * dz);
        const float rinv = 1.f / r;
        const int tj = MULTI ? b.type[j] : 0;
        float g[NA], dg[NA];
        radial_g_dg<NA, S::KA>(r, rcA_inv, m.cA + (ti * m.T + tj) * NA * S::KA, g, dg);
        const float w0 = gF[j] - wi0, w1 = gF[N + j] - wi1, w2 = gF[2 * N + j] - wi2;
        const float ux = dx * rinv, uy = dy * rinv, uz = dz * rinv;
        const float uw = ux * w0 + uy * w1 + uz * w2;
        for_each_poly_grad<NC>(ux, uy, uz, [&](int lm, float P, float px, float py, float pz) {
          const int l = comp_l(lm);
          const float a = uw * P;
          const float bb = (px * w0 + py * w1 + pz * w2 - (float)l * P * uw) * rinv;
#pragma unroll
          for (int n = 0; n < NA; ++n) {
            const float t = fmaf(dg[n], a, g[n] * bb);
            v[NR + (l - 1) * NA + n] = fmaf(s[n * NC + lm], t, v[NR + (l - 1) * NA + n]);
            if constexpr (S::FB) {
              if (l == 2) v[NR + S::L3 * NA + n] = fmaf(d4[5 * n + lm - 3], t, v[NR + S::L3 * NA + n]);
            }
          }
        });
      }
    }
  }
  // per-atom gradient terms (VALU); invalid lanes contribute zeros
  float qs[D], vs[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    qs[k] = valid ? q[k] * m.sigma[k] : 0.f;
    vs[k] = valid ? v[k] * m.sigma[k] : 0.f;
  }
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15, lk = lane >> 4;
  float* A = tA[wave];
  float* B = tB[wave];
  float alpha[H], beta[H], gw1c[H];
  const float gEf = (float)gE;
#pragma unroll
  for (int mu = 0; mu < H; ++mu) {
    float h = -m.b0[mu], z = 0.f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      h = fmaf(m.W0[mu * D + k], qs[k], h);
      z = fmaf(m.W0[mu * D + k], vs[k], z);
    }
    const float t = tanhf(h);
    const float d = 1.f - t * t;
    const float w1d = m.w1[mu] * d;
    alpha[mu] = valid ? fmaf(gEf, w1d, 2.f * z * m.w1[mu] * t * d) : 0.f;
    beta[mu] = valid ? w1d : 0.f;
    gw1c[mu] = valid ? fmaf(gEf, t, -z * d) : 0.f;
  }
  floatx4 acc[2][2];
#pragma unroll
  for (int R = 0; R < 2; ++R)
#pragma unroll
    for (int C = 0; C < 2; ++C) acc[R][C] = floatx4{0.f, 0.f, 0.f, 0.f};
  // sum over the wavefront's 64 atoms of alpha q~^T - beta v~^T on MFMA
#pragma unroll
  for (int pass = 0; pass < 2; ++pass) {
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      A[lane * kLdsStride + k] = k < H ? (pass == 0 ? alpha[k] : -beta[k]) : 0.f;
      B[lane * kLdsStride + k] = k < D ? (pass == 0 ? qs[k] : vs[k]) : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kb = 0; kb < 16; ++kb) {
      const int atom = 4 * kb + lk;
      float aop[2], bop[2];
#pragma unroll
      for (int R = 0; R < 2; ++R) aop[R] = A[atom * kLdsStride + 16 * R + lr];
#pragma unroll
      for (int C = 0; C < 2; ++C) bop[C] = B[atom * kLdsStride + 16 * C + lr];
#pragma unroll
      for (int R = 0; R < 2; ++R)
#pragma unroll
        for (int C = 0; C < 2; ++C)
          acc[R][C] = __builtin_amdgcn_mfma_f32_16x16x4f32(aop[R], bop[C], acc[R][C], 0, 0, 0);
    }
  }
  // column sums of alpha and of gE t - z d over the wavefront
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 32; ++k) {
    A[lane * kLdsStride + k] = k < H ? alpha[k] : 0.f;
    B[lane * kLdsStride + k] = k < H ? gw1c[k] : 0.f;
  }
  __syncthreads();
  float ca = 0.f, cb = 0.f;
  if (lane < 32) {
    for (int a = 0; a < 64; ++a) {
      ca += A[a * kLdsStride + lane];
      cb += B[a * kLdsStride + lane];
    }
  }
  __syncthreads();
  // combine the 4 wavefronts in FP64; tA is reused as [4][kGW + 64] floats
  float* red = &tA[0][0];
  constexpr int kW4 = kGW + 64;
#pragma unroll
  for (int R = 0; R < 2; ++R)
#pragma unroll
    for (int C = 0; C < 2; ++C)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[wave * kW4 + (16 * R + 4 * lk + r) * 32 + 16 * C + lr] = acc[R][C][r];
  if (lane < 32) {
    red[wave * kW4 + kGB0 + lane] = ca;
    red[wave * kW4 + kGW1 + lane] = cb;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kW4; e += kBlock) {
    double sum = 0.0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) sum += (double)red[w * kW4 + e];
    gpart[(int64_t)tile * kGradStride + e] = sum;
  }
}

// grad[theta] = sum over workgroups (FP64), in theta's packed order.
__global__ void k_grad_reduce(const double* __restrict__ gpart, int nblocks, int H, int D, double gE, int64_t N,
                              float* __restrict__ grad, int accumulate) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int G = H * D + 2 * H + 1;
  if (e >= G) return;
  double out;
  if (e == G - 1) {
    out = -gE * (double)N;
  } else {
    int src;
    double sign = 1.0;
    if (e < H * D) src = (e / D) * 32 + (e % D);
    else if (e < H * D + H) { src = kGB0 + (e - H * D); sign = -1.0; }
    else src = kGW1 + (e - H * D - H);
    double sum = 0.0;
    for (int blk = 0; blk < nblocks; ++blk) sum += gpart[(int64_t)blk * kGradStride + src];
    out = sign * sum;
  }
  grad[e] = accumulate ? (float)((double)grad[e] + out) : (float)out;
}

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

template <class S>
hipError_t launch_backward_shape(const ModelDev& m, const TrainBuffers& t, hipStream_t st) {
  const int nb = grid_blocks(t.e.N);
  if (m.T > 1)
    hipLaunchKernelGGL((k_train_backward<S, true>), dim3(nb), dim3(kBlock), 0, st, m, t.e, t.gF, t.gE, t.gpart);
  else
    hipLaunchKernelGGL((k_train_backward<S, false>), dim3(nb), dim3(kBlock), 0, st, m, t.e, t.gF, t.gE, t.gpart);
  const int G = m.H * m.D + 2 * m.H + 1;
  hipLaunchKernelGGL(k_grad_reduce, dim3(grid_blocks(G)), dim3(kBlock), 0, st, t.gpart, nb, m.H, m.D, t.gE,
                     t.e.N, t.grad, t.accumulate);
  return hipGetLastError();
}

ModelDev with_theta(const ModelDev& m, const float* theta) {
  ModelDev mt = m;
  const int G = m.H * m.D;
  mt.W0 = theta;
  mt.b0 = theta + G;
  mt.w1 = theta + G + m.H;
  mt.b1 = theta + G + 2 * m.H;
  return mt;
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
int train_grad_stride() { return kGradStride; }

hipError_t launch_train_forward(const ModelDev& m, const float* theta, const EvalBuffers& b, hipStream_t st) {
  return launch_eval(with_theta(m, theta), 0, b, st);
}

hipError_t launch_train_backward(const ModelDev& m, const TrainBuffers& t, hipStream_t st) {
  const ModelDev mt = with_theta(m, t.theta);
  if (is_shape<FullShape>(mt)) return launch_backward_shape<FullShape>(mt, t, st);
  if (is_shape<SurShape>(mt)) return launch_backward_shape<SurShape>(mt, t, st);
  return hipErrorInvalidValue;
}

}  // namespace nep
