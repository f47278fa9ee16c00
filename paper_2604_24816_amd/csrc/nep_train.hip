// Differentiation of L = gE * E + sum_i gF_i . F_i with respect to the network
// parameters theta = (W0, b0, w1, b1), with respect to the expansion coefficients
// and the scaler, and the Adam update.
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
    ZblSeenFor<MULTI> zs;  // the ZBL terms do not depend on the parameters
    desc_accumulate<S, MULTI>(m, b, i, ti, xi, yi, zi, Lx, Ly, Lz, q, s, zs, nr, na);
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

// Sum of v over the wavefront, added by its first lane to an LDS word.
__device__ __forceinline__ void wave_add_lds(float v, float* dst) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) atomicAdd(dst, v);
}

// Adds v for centers of species ti into dst[ti * stride] (one species: dst).
template <bool MULTI>
__device__ __forceinline__ void wave_add_by_type(float v, int ti, int T, float* dst, int stride) {
  if constexpr (MULTI) {
    for (int t = 0; t < T; ++t) wave_add_lds(ti == t ? v : 0.f, dst + t * stride);
  } else {
    wave_add_lds(v, dst);
  }
}

// Gradient of L = gE * E + sum_i gF_i . F_i with respect to the expansion
// coefficients c of the radial functions (Section III.B) and the descriptor
// scaler sigma. Each center contributes L_i = gE U_i - Fp_i . v_i (v_i: the
// descriptor JVP along gF). With alpha and beta as in k_train_backward,
// rho = sigma * (W0^T alpha) is dL_i/dq and -Fp = -sigma * (W0^T beta) is dL_i/dv.
//  * radial: q_n and v_n are linear in c through the basis sums over the neighbours
//    j of each species t, F_k = sum f_k(r_ij) and E_k = sum f'_k(r_ij) (u.w), so
//    dL/dc^{t_i t}_{nk} += rho_n F_k - Fp_n E_k;
//  * angular: with s_nlm, its JVP sd_nlm and the weights W_lm of q_nl,
//      A_nlm = 2 W_lm Fp_nl s_nlm,  C_nlm = 2 W_lm (rho_nl s_nlm - Fp_nl sd_nlm)
//    (plus, for the four-body term, Fp4 dq4/ds in A and rho4 dq4/ds - Fp4 (d^2q4/ds^2) sd
//    in C), and each pair adds f_k (X_n - Z_n) - f'_k (u.w) Y_n to dL/dc_nk, with
//    X_n = sum_lm C_nlm P_lm, Y_n = sum_lm A_nlm P_lm and
//    Z_n = sum_lm A_nlm (grad P_lm . w - l P_lm (u.w)) / r;
//  * scaler: dL/dsigma_k += q_k (W0^T alpha)_k - v_k (W0^T beta)_k.
// Sums over the workgroup run in FP32 (wavefront shuffles, then LDS atomics); each
// workgroup writes its sums as FP64 in the packed order [cR | cA | sigma].
template <class S, bool MULTI>
__global__ void __launch_bounds__(kBlock, 1)
k_train_cgrad(ModelDev m, EvalBuffers b, const float* __restrict__ gF, double gE, double* __restrict__ gpart) {
  constexpr int NR = S::NR, NA = S::NA, NC = S::NC, D = S::D, H = S::H, KR = S::KR, KA = S::KA;
  constexpr int TT = MULTI ? kMaxTypes : 1;
  static_assert(kMaxTypes * kMaxTypes * (NR * KR + NA * KA) + D <= kGradStride, "partial row too short");
  __shared__ float red[kMaxTypes * kMaxTypes * (NR * KR + NA * KA) + D];
  const int T = MULTI ? m.T : 1;
  const int oA = T * T * NR * KR, oS = oA + T * T * NA * KA;
  const int nred = oS + D;
  for (int e = threadIdx.x; e < nred; e += kBlock) red[e] = 0.f;
  __syncthreads();
  const int64_t N = b.N;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t i = (int64_t)tile * kBlock + threadIdx.x;
  const bool valid = i < N;
  const double* __restrict__ x = b.x;
  const double Lx = b.box[0], Ly = b.box[1], Lz = b.box[2];
  const float rcR_inv = 1.f / m.rcR, rcA_inv = 1.f / m.rcA;
  const double rcR2 = m.rcR64 * m.rcR64, rcA2 = m.rcA64 * m.rcA64;

  float q[D], v[D], s[NA * NC], sd[NA * NC], Fk[TT][KR], Ek[TT][KR];
#pragma unroll
  for (int k = 0; k < D; ++k) q[k] = v[k] = 0.f;
#pragma unroll
  for (int k = 0; k < NA * NC; ++k) s[k] = sd[k] = 0.f;
#pragma unroll
  for (int t = 0; t < TT; ++t)
#pragma unroll
    for (int k = 0; k < KR; ++k) Fk[t][k] = Ek[t][k] = 0.f;
  int ti = 0;
  double xi = 0, yi = 0, zi = 0;
  float wi0 = 0.f, wi1 = 0.f, wi2 = 0.f;
  if (valid) {
    ti = MULTI ? b.type[i] : 0;
    xi = x[i];
    yi = x[N + i];
    zi = x[2 * N + i];
    int nr = 0, na = 0;
    ZblSeenFor<MULTI> zs;  // the ZBL terms do not depend on the parameters
    desc_accumulate<S, MULTI>(m, b, i, ti, xi, yi, zi, Lx, Ly, Lz, q, s, zs, nr, na);
    desc_finish<S>(s, q);
    if (gF) {
      wi0 = gF[i];
      wi1 = gF[N + i];
      wi2 = gF[2 * N + i];
    }
    // radial basis sums per neighbour species
    const int kR = radial_bound(b, i);
    for (int p = 0; p < kR; ++p) {
      const int32_t j = b.nbr[(int64_t)p * N + i];
      float dx, dy, dz;
      if (!pair_inside(x, N, j, xi, yi, zi, Lx, Ly, Lz, rcR2, dx, dy, dz)) continue;
      const float r = sqrtf(dx * dx + dy * dy + dz * dz);
      const float rinv = 1.f / r;
      const int tj = MULTI ? b.type[j] : 0;
      float f[KR], e[KR];
      radial_basis<KR>(r, rcR_inv, f);
      float uw = 0.f;
      if (gF) {
        radial_basis_deriv<KR>(r, rcR_inv, e);
        uw = ((gF[j] - wi0) * dx + (gF[N + j] - wi1) * dy + (gF[2 * N + j] - wi2) * dz) * rinv;
      } else {
#pragma unroll
        for (int k = 0; k < KR; ++k) e[k] = 0.f;
      }
#pragma unroll
      for (int t = 0; t < TT; ++t) {
        const bool on = !MULTI || tj == t;
#pragma unroll
        for (int k = 0; k < KR; ++k) {
          Fk[t][k] += on ? f[k] : 0.f;
          Ek[t][k] = fmaf(on ? e[k] : 0.f, uw, Ek[t][k]);
        }
      }
    }
    if (gF) {
      // radial JVP v_n = sum_t sum_k c^{t_i t}_{nk} E_k
#pragma unroll
      for (int t = 0; t < TT; ++t) {
        if (t >= T) break;
        const float* c = m.cR + (ti * T + t) * NR * KR;
#pragma unroll
        for (int n = 0; n < NR; ++n)
#pragma unroll
          for (int k = 0; k < KR; ++k) v[n] = fmaf(c[n * KR + k], Ek[t][k], v[n]);
      }
      // angular JVP sd_nlm = sum_j [g_n' (u.w) P_lm + g_n (grad P_lm . w - l P_lm (u.w)) / r]
      const int kA = angular_bound(b, i);
      for (int p = 0; p < kA; ++p) {
        const int32_t j = b.nbr[(int64_t)p * N + i];
        float dx, dy, dz;
        if (!pair_inside(x, N, j, xi, yi, zi, Lx, Ly, Lz, rcA2, dx, dy, dz)) continue;
        const float r = sqrtf(dx * dx + dy * dy + dz * dz);
        const float rinv = 1.f / r;
        const int tj = MULTI ? b.type[j] : 0;
        float g[NA], dg[NA];
        radial_g_dg<NA, KA>(r, rcA_inv, m.cA + (ti * m.T + tj) * NA * KA, g, dg);
        const float w0 = gF[j] - wi0, w1 = gF[N + j] - wi1, w2 = gF[2 * N + j] - wi2;
        const float ux = dx * rinv, uy = dy * rinv, uz = dz * rinv;
        const float uw = ux * w0 + uy * w1 + uz * w2;
        for_each_poly_grad<NC>(ux, uy, uz, [&](int lm, float P, float px, float py, float pz) {
          const float a = uw * P;
          const float bb = (px * w0 + py * w1 + pz * w2 - (float)comp_l(lm) * P * uw) * rinv;
#pragma unroll
          for (int n = 0; n < NA; ++n) sd[n * NC + lm] = fmaf(dg[n], a, fmaf(g[n], bb, sd[n * NC + lm]));
        });
      }
#pragma unroll
      for (int n = 0; n < NA; ++n)
#pragma unroll
        for (int lm = 0; lm < NC; ++lm) {
          const int k = NR + (comp_l(lm) - 1) * NA + n;
          v[k] = fmaf(2.f * kW[lm] * s[n * NC + lm], sd[n * NC + lm], v[k]);
        }
      if constexpr (S::FB) {
#pragma unroll
        for (int n = 0; n < NA; ++n) {
          float d4[5];
          fourbody_ds(s + n * NC, d4);
#pragma unroll
          for (int c = 0; c < 5; ++c) v[NR + S::L3 * NA + n] = fmaf(d4[c], sd[n * NC + 3 + c], v[NR + S::L3 * NA + n]);
        }
      }
    }
  }
  // network: rho = sigma W0^T alpha, Fp = sigma W0^T beta
  float al[H], be[H];
  const float gEf = (float)gE;
#pragma unroll
  for (int mu = 0; mu < H; ++mu) {
    float h = -m.b0[mu], z = 0.f;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      h = fmaf(m.W0[mu * D + k], q[k] * m.sigma[k], h);
      z = fmaf(m.W0[mu * D + k], v[k] * m.sigma[k], z);
    }
    const float t = tanhf(h);
    const float d = 1.f - t * t;
    be[mu] = m.w1[mu] * d;
    al[mu] = fmaf(gEf, be[mu], 2.f * z * m.w1[mu] * t * d);
  }
  float rho[D], fp[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    float sa = 0.f, sb = 0.f;
#pragma unroll
    for (int mu = 0; mu < H; ++mu) {
      sa = fmaf(m.W0[mu * D + k], al[mu], sa);
      sb = fmaf(m.W0[mu * D + k], be[mu], sb);
    }
    rho[k] = m.sigma[k] * sa;
    fp[k] = m.sigma[k] * sb;
    wave_add_lds(valid ? q[k] * sa - v[k] * sb : 0.f, red + oS + k);
  }
  // radial coefficients
#pragma unroll
  for (int t = 0; t < TT; ++t) {
    if (t >= T) break;
#pragma unroll
    for (int n = 0; n < NR; ++n)
#pragma unroll
      for (int k = 0; k < KR; ++k)
        wave_add_by_type<MULTI>(valid ? rho[n] * Fk[t][k] - fp[n] * Ek[t][k] : 0.f, ti, T,
                                red + (t * NR + n) * KR + k, T * NR * KR);
  }
  // angular coefficients A (in place of s) and C (in place of sd)
  if constexpr (S::FB) {
#pragma unroll
    for (int n = 0; n < NA; ++n) {
      float d4[5], h4[5];
      fourbody_ds(s + n * NC, d4);
      fourbody_ds_dir(s + n * NC, sd + n * NC, h4);
      const int k4 = NR + S::L3 * NA + n;
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        const int lm = 3 + c;
        const int k = NR + NA + n;  // l = 2
        const float a = 2.f * kW[lm] * fp[k] * s[n * NC + lm] + fp[k4] * d4[c];
        const float cc = 2.f * kW[lm] * (rho[k] * s[n * NC + lm] - fp[k] * sd[n * NC + lm]) + rho[k4] * d4[c] -
                         fp[k4] * h4[c];
        s[n * NC + lm] = a;
        sd[n * NC + lm] = cc;
      }
    }
  }
#pragma unroll
  for (int n = 0; n < NA; ++n)
#pragma unroll
    for (int lm = 0; lm < NC; ++lm) {
      if (S::FB && comp_l(lm) == 2) continue;
      const int k = NR + (comp_l(lm) - 1) * NA + n;
      const float a = 2.f * kW[lm] * fp[k] * s[n * NC + lm];
      const float cc = 2.f * kW[lm] * (rho[k] * s[n * NC + lm] - fp[k] * sd[n * NC + lm]);
      s[n * NC + lm] = a;
      sd[n * NC + lm] = cc;
    }
  for (int t = 0; t < TT; ++t) {
    if (t >= T) break;
    float acc[NA * KA];
#pragma unroll
    for (int k = 0; k < NA * KA; ++k) acc[k] = 0.f;
    if (valid) {
      const int kA = angular_bound(b, i);
      for (int p = 0; p < kA; ++p) {
        const int32_t j = b.nbr[(int64_t)p * N + i];
        float dx, dy, dz;
        if (!pair_inside(x, N, j, xi, yi, zi, Lx, Ly, Lz, rcA2, dx, dy, dz)) continue;
        if (MULTI && b.type[j] != t) continue;
        const float r = sqrtf(dx * dx + dy * dy + dz * dz);
        const float rinv = 1.f / r;
        const float ux = dx * rinv, uy = dy * rinv, uz = dz * rinv;
        float w0 = 0.f, w1 = 0.f, w2 = 0.f;
        if (gF) {
          w0 = gF[j] - wi0;
          w1 = gF[N + j] - wi1;
          w2 = gF[2 * N + j] - wi2;
        }
        const float uw = ux * w0 + uy * w1 + uz * w2;
        float X[NA], Y[NA], Z[NA];
#pragma unroll
        for (int n = 0; n < NA; ++n) X[n] = Y[n] = Z[n] = 0.f;
        for_each_poly_grad<NC>(ux, uy, uz, [&](int lm, float P, float px, float py, float pz) {
          const float bb = (px * w0 + py * w1 + pz * w2 - (float)comp_l(lm) * P * uw) * rinv;
#pragma unroll
          for (int n = 0; n < NA; ++n) {
            X[n] = fmaf(sd[n * NC + lm], P, X[n]);
            Y[n] = fmaf(s[n * NC + lm], P, Y[n]);
            Z[n] = fmaf(s[n * NC + lm], bb, Z[n]);
          }
        });
        float f[KA], e[KA];
        radial_basis<KA>(r, rcA_inv, f);
        radial_basis_deriv<KA>(r, rcA_inv, e);
#pragma unroll
        for (int n = 0; n < NA; ++n) {
          const float xz = X[n] - Z[n], yu = Y[n] * uw;
#pragma unroll
          for (int k = 0; k < KA; ++k) acc[n * KA + k] = fmaf(f[k], xz, fmaf(-e[k], yu, acc[n * KA + k]));
        }
      }
    }
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
      for (int k = 0; k < KA; ++k)
        wave_add_by_type<MULTI>(valid ? acc[n * KA + k] : 0.f, ti, T, red + oA + (t * NA + n) * KA + k,
                                T * NA * KA);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nred; e += kBlock) gpart[(int64_t)tile * kGradStride + e] = (double)red[e];
}

// grad[e] for e < n (the [cR | cA | sigma] block) = sum over workgroups (FP64).
__global__ void k_cgrad_reduce(const double* __restrict__ gpart, int nblocks, int n, float* __restrict__ grad,
                               int accumulate) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double sum = 0.0;
  for (int blk = 0; blk < nblocks; ++blk) sum += gpart[(int64_t)blk * kGradStride + e];
  grad[e] = accumulate ? (float)((double)grad[e] + sum) : (float)sum;
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

template <class S>
hipError_t launch_cgrad_shape(const ModelDev& m, const TrainBuffers& t, hipStream_t st) {
  const int nb = grid_blocks(t.e.N);
  if (m.T > 1)
    hipLaunchKernelGGL((k_train_cgrad<S, true>), dim3(nb), dim3(kBlock), 0, st, m, t.e, t.gF, t.gE, t.gpart);
  else
    hipLaunchKernelGGL((k_train_cgrad<S, false>), dim3(nb), dim3(kBlock), 0, st, m, t.e, t.gF, t.gE, t.gpart);
  const int n = m.T * m.T * (m.nR * m.kR + m.nA * m.kA) + m.D;
  hipLaunchKernelGGL(k_cgrad_reduce, dim3(grid_blocks(n)), dim3(kBlock), 0, st, t.gpart, nb, n, t.grad,
                     t.accumulate);
  return hipGetLastError();
}

// The model with every parameter read from a packed FP32 vector
// [cR | cA | sigma | W0 | b0 | w1 | b1].
ModelDev with_params(const ModelDev& m, const float* p) {
  ModelDev mp = m;
  mp.cR = p;
  mp.cA = mp.cR + m.T * m.T * m.nR * m.kR;
  mp.sigma = mp.cA + m.T * m.T * m.nA * m.kA;
  mp.W0 = mp.sigma + m.D;
  mp.b0 = mp.W0 + m.H * m.D;
  mp.w1 = mp.b0 + m.H;
  mp.b1 = mp.w1 + m.H;
  return mp;
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

int param_block_offset(const ModelDev& m) {
  return m.T * m.T * (m.nR * m.kR + m.nA * m.kA) + m.D;
}

hipError_t launch_train_forward_params(const ModelDev& m, const float* params, const EvalBuffers& b,
                                       hipStream_t st) {
  // the evaluation kernels read the radial coefficients through their derived tables:
  // build them from this vector's coefficients
  ModelDev mp = with_params(m, params);
  mp.hR = m.hscratch;
  mp.hA = m.hscratch + (int64_t)m.T * m.T * m.nR * (2 * m.kR - 1);
  hipError_t e = launch_derive_coeffs(m.T, m.nR, m.kR, m.nA, m.kA, mp.cR, mp.cA, m.hscratch,
                                      const_cast<float*>(mp.hA), st);
  if (e != hipSuccess) return e;
  return launch_eval(mp, 0, b, st);
}

hipError_t launch_train_backward_params(const ModelDev& m, const TrainBuffers& t, hipStream_t st) {
  const ModelDev mp = with_params(m, t.theta);
  TrainBuffers tn = t;
  tn.grad = t.grad + param_block_offset(m);
  hipError_t e;
  if (is_shape<FullShape>(mp)) {
    if ((e = launch_backward_shape<FullShape>(mp, tn, st)) != hipSuccess) return e;
    return launch_cgrad_shape<FullShape>(mp, t, st);
  }
  if (is_shape<SurShape>(mp)) {
    if ((e = launch_backward_shape<SurShape>(mp, tn, st)) != hipSuccess) return e;
    return launch_cgrad_shape<SurShape>(mp, t, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_train_backward(const ModelDev& m, const TrainBuffers& t, hipStream_t st) {
  const ModelDev mt = with_theta(m, t.theta);
  if (is_shape<FullShape>(mt)) return launch_backward_shape<FullShape>(mt, t, st);
  if (is_shape<SurShape>(mt)) return launch_backward_shape<SurShape>(mt, t, st);
  return hipErrorInvalidValue;
}

}  // namespace nep
