// NEP energy/force evaluation on gfx950: two kernels per force evaluation.
//
//   k_desc_net  (one thread per center, 256-thread workgroups)
//     0. compaction: the neighbours inside the true cutoffs are picked out of
//        the skin list once per evaluation, so the descriptor and force loops
//        below run over exactly the pairs that contribute;
//     1. radial descriptors q_n = sum_j g_n(r_ij) (Section III.B);
//     2. angular accumulators s_nlm = sum_j g_n(r_ij) P_lm(u_ij) for every
//        channel n in one neighbour pass (Algorithm 1's geometry reuse with the
//        channel tile equal to all n_max+1 channels), and from them
//        q_nl = sum_m W_lm s_nlm^2 and the four-body invariant tr(S_n^3);
//     3. the network U_i = w1 . tanh(W0 q~ - b0) - b1 and its gradient
//        dU/dq~ = W0^T (w1 (1 - tanh^2)) as two 64-row MFMA products per
//        wavefront (Section V.B Optimization 1, Fig. 2c), operands staged
//        through LDS; FP32 MFMA or bfloat16 MFMA with FP32 accumulation;
//     4. per-atom dU/ds_nlm is written for the force kernel.
//   k_force
//     radial pair forces by gather (F_i += sum_j [dU_i/dr_ij - dU_j/dr_ji]
//     with the neighbour's dU/dq_n read from HBM), angular and four-body pair
//     forces from dU/ds by scatter with FP32 atomics into the neighbour
//     (Section V.B Optimization 1: no temporary per-pair force buffer), and the
//     virial W_ab = -sum r_a dU_i/dr_b; energy and virial are reduced per
//     workgroup in FP64.
#include "nep_common.h"
#include "nep_poly.h"

namespace nep {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr float kPiF = 3.14159265358979323846f;

// Round-to-nearest-even conversion of an FP32 value to bfloat16 bits.
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ __bf16 bits_to_bf16(uint16_t b) { return __builtin_bit_cast(__bf16, b); }

// Chebyshev-based radial basis f_k(r) = (T_k(x) + 1) f_c(r) / 2 with
// x = 2 (r/rc - 1)^2 - 1 and f_c = (1 + cos(pi r / rc)) / 2 (published NEP form).
// Returns g_n = sum_k c_nk f_k.
template <int N, int K>
__device__ __forceinline__ void radial_g(float r, float rc_inv, const float* __restrict__ c, float* g) {
  float sn, cs;
  sincospif(r * rc_inv, &sn, &cs);
  const float fc = 0.5f * (1.f + cs);
  const float y = r * rc_inv - 1.f;
  const float x = 2.f * y * y - 1.f;
  float Tm1 = 1.f, T = x;
  float fk[K];
  fk[0] = 1.f;
  fk[1] = 0.5f * (x + 1.f);
#pragma unroll
  for (int k = 2; k < K; ++k) {
    const float Tn = 2.f * x * T - Tm1;
    Tm1 = T;
    T = Tn;
    fk[k] = 0.5f * (Tn + 1.f);
  }
#pragma unroll
  for (int n = 0; n < N; ++n) {
    float a = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) a = fmaf(c[n * K + k], fk[k], a);
    g[n] = a * fc;
  }
}

// g_n and dg_n/dr.
template <int N, int K>
__device__ __forceinline__ void radial_g_dg(float r, float rc_inv, const float* __restrict__ c, float* g,
                                            float* dg) {
  float sn, cs;
  sincospif(r * rc_inv, &sn, &cs);
  const float fc = 0.5f * (1.f + cs);
  const float dfc = -0.5f * kPiF * rc_inv * sn;
  const float y = r * rc_inv - 1.f;
  const float x = 2.f * y * y - 1.f;
  const float dx = 4.f * y * rc_inv;
  float hk[K], dk[K];  // (T_k + 1)/2 and T_k'/2
  float Tm1 = 1.f, T = x, dTm1 = 0.f, dT = 1.f;
  hk[0] = 1.f;
  dk[0] = 0.f;
  hk[1] = 0.5f * (x + 1.f);
  dk[1] = 0.5f;
#pragma unroll
  for (int k = 2; k < K; ++k) {
    const float Tn = 2.f * x * T - Tm1;
    const float dTn = 2.f * T + 2.f * x * dT - dTm1;
    Tm1 = T;
    T = Tn;
    dTm1 = dT;
    dT = dTn;
    hk[k] = 0.5f * (Tn + 1.f);
    dk[k] = 0.5f * dTn;
  }
  const float fcdx = fc * dx;
#pragma unroll
  for (int n = 0; n < N; ++n) {
    float a = 0.f, b = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      a = fmaf(c[n * K + k], hk[k], a);
      b = fmaf(c[n * K + k], dk[k], b);
    }
    g[n] = a * fc;
    dg[n] = fmaf(b, fcdx, a * dfc);
  }
}

// FP64 minimum-image pair vector, rounded to FP32 after the subtraction.
__device__ __forceinline__ void pair_vec(const double* __restrict__ x, int64_t N, int64_t j, double xi,
                                         double yi, double zi, double Lx, double Ly, double Lz, float& dx,
                                         float& dy, float& dz) {
  dx = (float)min_image(x[j] - xi, Lx);
  dy = (float)min_image(x[N + j] - yi, Ly);
  dz = (float)min_image(x[2 * N + j] - zi, Lz);
}

// Deterministic FP64 sum over a 256-thread workgroup (fixed tree order).
__device__ __forceinline__ double block_sum(double v, double* sh) {
  __syncthreads();
  sh[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < (unsigned)off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  return sh[0];
}

template <int NR_, int KR_, int NA_, int KA_, int L3_, bool FB_, int H_>
struct Shape {
  static constexpr int NR = NR_, KR = KR_, NA = NA_, KA = KA_, L3 = L3_, H = H_;
  static constexpr bool FB = FB_;
  static constexpr int NC = L3 * (L3 + 2);
  static constexpr int D = NR + NA * L3 + (FB ? NA : 0);
  static_assert(D <= 32 && H <= 32, "network tiles hold at most 32 descriptors and 32 hidden units");
  static_assert(!FB || L3 >= 2, "the four-body term uses the l = 2 accumulators");
};

using FullShape = Shape<5, 9, 5, 9, 4, true, 30>;
using SurShape = Shape<5, 9, 5, 9, 2, false, 8>;

constexpr int kLdsStride = 33;  // 32 columns + 1 pad word against bank conflicts

// ------------------------------------------------------------------------ network
// One wavefront evaluates the network for its 64 centers. qs[lane][v] holds the
// scaled descriptor of the lane's center on entry; on exit fp[v] = dU/dq~ and the
// return value is U. lds: this wavefront's 64 x 33 float tile.
template <class S, int PREC>
__device__ __forceinline__ float network_wave(const ModelDev& m, const float* qs, float* fp, float* lds,
                                              const float* __restrict__ W0, const float* __restrict__ b0,
                                              const float* __restrict__ w1, float b1) {
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15;   // row / column within a 16-wide tile
  const int lk = lane >> 4;   // k group
  float* row = lds + lane * kLdsStride;
#pragma unroll
  for (int v = 0; v < 32; ++v) row[v] = v < S::D ? qs[v] : 0.f;
  __syncthreads();
  floatx4 acc[4][2];
#pragma unroll
  for (int R = 0; R < 4; ++R)
#pragma unroll
    for (int C = 0; C < 2; ++C) acc[R][C] = floatx4{0.f, 0.f, 0.f, 0.f};
  if constexpr (PREC == 0) {
    // h[center][hidden] = sum_desc q~[center][desc] W0[hidden][desc], K = 32 in 8 steps of 4.
#pragma unroll
    for (int kb = 0; kb < 8; ++kb) {
      const int dcol = 4 * kb + lk;
      float bop[2];
#pragma unroll
      for (int C = 0; C < 2; ++C) {
        const int hid = 16 * C + lr;
        bop[C] = (hid < S::H && dcol < S::D) ? W0[hid * S::D + dcol] : 0.f;
      }
#pragma unroll
      for (int R = 0; R < 4; ++R) {
        const float aop = lds[(16 * R + lr) * kLdsStride + dcol];
#pragma unroll
        for (int C = 0; C < 2; ++C)
          acc[R][C] = __builtin_amdgcn_mfma_f32_16x16x4f32(aop, bop[C], acc[R][C], 0, 0, 0);
      }
    }
  } else {
    bf16x8 bop[2];
#pragma unroll
    for (int C = 0; C < 2; ++C) {
      const int hid = 16 * C + lr;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int dcol = 8 * lk + e;
        bop[C][e] = bits_to_bf16((hid < S::H && dcol < S::D) ? m.W0bf[hid * S::D + dcol] : (uint16_t)0);
      }
    }
#pragma unroll
    for (int R = 0; R < 4; ++R) {
      bf16x8 aop;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        aop[e] = bits_to_bf16(f32_to_bf16_bits(lds[(16 * R + lr) * kLdsStride + 8 * lk + e]));
#pragma unroll
      for (int C = 0; C < 2; ++C)
        acc[R][C] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, bop[C], acc[R][C], 0, 0, 0);
    }
  }
  __syncthreads();
  // D layout: lane holds rows 4*lk + r of column lr.
#pragma unroll
  for (int R = 0; R < 4; ++R)
#pragma unroll
    for (int C = 0; C < 2; ++C)
#pragma unroll
      for (int r = 0; r < 4; ++r) lds[(16 * R + 4 * lk + r) * kLdsStride + 16 * C + lr] = acc[R][C][r];
  __syncthreads();
  float U = -b1;
  float a1[32];
#pragma unroll
  for (int mu = 0; mu < 32; ++mu) {
    if (mu < S::H) {
      const float t = tanhf(row[mu] - b0[mu]);
      U = fmaf(w1[mu], t, U);
      a1[mu] = w1[mu] * (1.f - t * t);
    } else {
      a1[mu] = 0.f;
    }
  }
  __syncthreads();
#pragma unroll
  for (int mu = 0; mu < 32; ++mu) row[mu] = a1[mu];
  __syncthreads();
#pragma unroll
  for (int R = 0; R < 4; ++R)
#pragma unroll
    for (int C = 0; C < 2; ++C) acc[R][C] = floatx4{0.f, 0.f, 0.f, 0.f};
  if constexpr (PREC == 0) {
    // Fp[center][desc] = sum_hidden a[center][hidden] W0[hidden][desc].
#pragma unroll
    for (int kb = 0; kb < 8; ++kb) {
      const int hid = 4 * kb + lk;
      float bop[2];
#pragma unroll
      for (int C = 0; C < 2; ++C) {
        const int dcol = 16 * C + lr;
        bop[C] = (hid < S::H && dcol < S::D) ? W0[hid * S::D + dcol] : 0.f;
      }
#pragma unroll
      for (int R = 0; R < 4; ++R) {
        const float aop = lds[(16 * R + lr) * kLdsStride + hid];
#pragma unroll
        for (int C = 0; C < 2; ++C)
          acc[R][C] = __builtin_amdgcn_mfma_f32_16x16x4f32(aop, bop[C], acc[R][C], 0, 0, 0);
      }
    }
  } else {
    bf16x8 bop[2];
#pragma unroll
    for (int C = 0; C < 2; ++C) {
      const int dcol = 16 * C + lr;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int hid = 8 * lk + e;
        bop[C][e] = bits_to_bf16((hid < S::H && dcol < S::D) ? m.W0bf[hid * S::D + dcol] : (uint16_t)0);
      }
    }
#pragma unroll
    for (int R = 0; R < 4; ++R) {
      bf16x8 aop;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        aop[e] = bits_to_bf16(f32_to_bf16_bits(lds[(16 * R + lr) * kLdsStride + 8 * lk + e]));
#pragma unroll
      for (int C = 0; C < 2; ++C)
        acc[R][C] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, bop[C], acc[R][C], 0, 0, 0);
    }
  }
  __syncthreads();
#pragma unroll
  for (int R = 0; R < 4; ++R)
#pragma unroll
    for (int C = 0; C < 2; ++C)
#pragma unroll
      for (int r = 0; r < 4; ++r) lds[(16 * R + 4 * lk + r) * kLdsStride + 16 * C + lr] = acc[R][C][r];
  __syncthreads();
#pragma unroll
  for (int v = 0; v < S::D; ++v) fp[v] = row[v];
  return U;
}

// ------------------------------------------------------------------------ descriptor + network
template <class S, int PREC, bool MULTI>
__global__ void __launch_bounds__(kBlock, 2) k_desc_net(ModelDev m, EvalBuffers b) {
  __shared__ float lds[kBlock / 64][64 * kLdsStride];
  __shared__ double red[kBlock];
  constexpr int NR = S::NR, NA = S::NA, NC = S::NC, D = S::D;
  const int64_t N = b.N;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t i = (int64_t)tile * kBlock + threadIdx.x;
  const bool valid = i < N;
  const double* __restrict__ x = b.x;
  const double Lx = b.box[0], Ly = b.box[1], Lz = b.box[2];
  const float rcR_inv = 1.f / m.rcR, rcA_inv = 1.f / m.rcA;

  float q[D];
#pragma unroll
  for (int v = 0; v < D; ++v) q[v] = 0.f;
  float s[NA * NC];
#pragma unroll
  for (int k = 0; k < NA * NC; ++k) s[k] = 0.f;
  const int ti = valid ? (MULTI ? b.type[i] : 0) : 0;

  if (valid) {
    const double xi = x[i], yi = x[N + i], zi = x[2 * N + i];
    // 0. compaction of the skin list to the true cutoffs
    const int cnt = b.cntR[i];
    const double rcR2 = m.rcR64 * m.rcR64, rcA2 = m.rcA64 * m.rcA64;
    int nr = 0, na = 0;
    for (int p = 0; p < cnt; ++p) {
      const int32_t j = b.nbrR[(int64_t)p * N + i];
      const double dx = min_image(x[j] - xi, Lx);
      const double dy = min_image(x[N + j] - yi, Ly);
      const double dz = min_image(x[2 * N + j] - zi, Lz);
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (r2 < rcR2) {
        b.actR[(int64_t)nr * N + i] = j;
        ++nr;
        if (r2 < rcA2) {
          b.actA[(int64_t)na * N + i] = j;
          ++na;
        }
      }
    }
    b.nactR[i] = nr;
    b.nactA[i] = na;
    // 1. radial descriptors
    for (int p = 0; p < nr; ++p) {
      const int32_t j = b.actR[(int64_t)p * N + i];
      float dx, dy, dz;
      pair_vec(x, N, j, xi, yi, zi, Lx, Ly, Lz, dx, dy, dz);
      const float r = sqrtf(dx * dx + dy * dy + dz * dz);
      const int tj = MULTI ? b.type[j] : 0;
      float g[NR];
      radial_g<NR, S::KR>(r, rcR_inv, m.cR + (ti * m.T + tj) * NR * S::KR, g);
#pragma unroll
      for (int n = 0; n < NR; ++n) q[n] += g[n];
    }
    // 2. angular accumulators, all channels in one pass over the neighbours
    for (int p = 0; p < na; ++p) {
      const int32_t j = b.actA[(int64_t)p * N + i];
      float dx, dy, dz;
      pair_vec(x, N, j, xi, yi, zi, Lx, Ly, Lz, dx, dy, dz);
      const float r = sqrtf(dx * dx + dy * dy + dz * dz);
      const float rinv = 1.f / r;
      const int tj = MULTI ? b.type[j] : 0;
      float g[NA];
      radial_g<NA, S::KA>(r, rcA_inv, m.cA + (ti * m.T + tj) * NA * S::KA, g);
      for_each_poly<NC>(dx * rinv, dy * rinv, dz * rinv, [&](int lm, float P) {
#pragma unroll
        for (int n = 0; n < NA; ++n) s[n * NC + lm] = fmaf(g[n], P, s[n * NC + lm]);
      });
    }
    // q_nl = sum_m W_lm s_nlm^2
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
      for (int lm = 0; lm < NC; ++lm) {
        const int l = comp_l(lm);
        q[NR + (l - 1) * NA + n] = fmaf(kW[lm], s[n * NC + lm] * s[n * NC + lm], q[NR + (l - 1) * NA + n]);
      }
    // four-body: S_n = sum_j g_n (u u^T - I/3) from the l = 2 sums, q4 = tr(S^3) = 3 det S
    if constexpr (S::FB) {
#pragma unroll
      for (int n = 0; n < NA; ++n) {
        const float* sl = s + n * NC;
        const float Sxy = sl[3], Syz = sl[4], Szz = sl[5] * (1.f / 3.f), Sxz = sl[6], Dxy = sl[7];
        const float Sxx = 0.5f * (Dxy - Szz), Syy = 0.5f * (-Dxy - Szz);
        const float det = Sxx * (Syy * Szz - Syz * Syz) - Sxy * (Sxy * Szz - Syz * Sxz) +
                          Sxz * (Sxy * Syz - Syy * Sxz);
        q[NR + S::L3 * NA + n] = 3.f * det;
      }
    }
  }
  // 3. network (whole wavefronts take part; inactive lanes carry zeros)
  float qs[D], fp[D];
#pragma unroll
  for (int v = 0; v < D; ++v) qs[v] = q[v] * m.sigma[v];
  const float U = network_wave<S, PREC>(m, qs, fp, lds[threadIdx.x >> 6], m.W0, m.b0, m.w1, m.b1[0]);
#pragma unroll
  for (int v = 0; v < D; ++v) fp[v] *= m.sigma[v];  // dU/dq = sigma * dU/dq~

  if (valid) {
    b.U[i] = U;
#pragma unroll
    for (int n = 0; n < NR; ++n) b.FpR[(int64_t)n * N + i] = fp[n];
    // 4. dU/ds_nlm = dU/dq_nl * 2 W_lm s_nlm (+ four-body part for l = 2)
    float Gd[NA * NC];
#pragma unroll
    for (int n = 0; n < NA; ++n)
#pragma unroll
      for (int lm = 0; lm < NC; ++lm) {
        const int l = comp_l(lm);
        Gd[n * NC + lm] = fp[NR + (l - 1) * NA + n] * 2.f * kW[lm] * s[n * NC + lm];
      }
    if constexpr (S::FB) {
#pragma unroll
      for (int n = 0; n < NA; ++n) {
        const float* sl = s + n * NC;
        const float Sxy = sl[3], Syz = sl[4], Szz = sl[5] * (1.f / 3.f), Sxz = sl[6], Dxy = sl[7];
        const float Sxx = 0.5f * (Dxy - Szz), Syy = 0.5f * (-Dxy - Szz);
        // (S^2)_ab
        const float Q_xx = Sxx * Sxx + Sxy * Sxy + Sxz * Sxz;
        const float Q_yy = Sxy * Sxy + Syy * Syy + Syz * Syz;
        const float Q_zz = Sxz * Sxz + Syz * Syz + Szz * Szz;
        const float Q_xy = Sxx * Sxy + Sxy * Syy + Sxz * Syz;
        const float Q_yz = Sxy * Sxz + Syy * Syz + Syz * Szz;
        const float Q_xz = Sxx * Sxz + Sxy * Syz + Sxz * Szz;
        const float f4 = fp[NR + S::L3 * NA + n];
        // d tr(S^3) / d s for s = (xy, yz, 3z^2-r^2, xz, x^2-y^2)
        Gd[n * NC + 3] += f4 * 6.f * Q_xy;
        Gd[n * NC + 4] += f4 * 6.f * Q_yz;
        Gd[n * NC + 5] += f4 * (Q_zz - 0.5f * (Q_xx + Q_yy));
        Gd[n * NC + 6] += f4 * 6.f * Q_xz;
        Gd[n * NC + 7] += f4 * 1.5f * (Q_xx - Q_yy);
      }
    }
#pragma unroll
    for (int k = 0; k < NA * NC; ++k) b.G[(int64_t)k * N + i] = Gd[k];
    b.F[i] = 0.f;
    b.F[N + i] = 0.f;
    b.F[2 * N + i] = 0.f;
  }
  const double e = block_sum(valid ? (double)U : 0.0, red);
  if (threadIdx.x == 0) b.partial[(int64_t)tile * kPartialStride + P_ENERGY] = e;
}

// ------------------------------------------------------------------------ forces
template <class S, bool MULTI>
__global__ void __launch_bounds__(kBlock, 2) k_force(ModelDev m, EvalBuffers b) {
  __shared__ double red[kBlock];
  constexpr int NR = S::NR, NA = S::NA, NC = S::NC;
  const int64_t N = b.N;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t i = (int64_t)tile * kBlock + threadIdx.x;
  const bool valid = i < N;
  const double* __restrict__ x = b.x;
  const double Lx = b.box[0], Ly = b.box[1], Lz = b.box[2];
  const float rcR_inv = 1.f / m.rcR, rcA_inv = 1.f / m.rcA;
  float fx = 0.f, fy = 0.f, fz = 0.f;
  float w[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) w[k] = 0.f;
  if (valid) {
    const double xi = x[i], yi = x[N + i], zi = x[2 * N + i];
    const int ti = MULTI ? b.type[i] : 0;
    float fpi[NR];
#pragma unroll
    for (int n = 0; n < NR; ++n) fpi[n] = b.FpR[(int64_t)n * N + i];
    // radial: gather, F_i += (Fp_i . g'^{ij} + Fp_j . g'^{ji}) u
    const int nr = b.nactR[i];
    for (int p = 0; p < nr; ++p) {
      const int32_t j = b.actR[(int64_t)p * N + i];
      float dx, dy, dz;
      pair_vec(x, N, j, xi, yi, zi, Lx, Ly, Lz, dx, dy, dz);
      const float r = sqrtf(dx * dx + dy * dy + dz * dz);
      const float rinv = 1.f / r;
      const int tj = MULTI ? b.type[j] : 0;
      float g[NR], dg[NR];
      radial_g_dg<NR, S::KR>(r, rcR_inv, m.cR + (ti * m.T + tj) * NR * S::KR, g, dg);
      float si = 0.f, sj = 0.f;
      if constexpr (MULTI) {
        float g2[NR], dg2[NR];
        radial_g_dg<NR, S::KR>(r, rcR_inv, m.cR + (tj * m.T + ti) * NR * S::KR, g2, dg2);
#pragma unroll
        for (int n = 0; n < NR; ++n) {
          si = fmaf(fpi[n], dg[n], si);
          sj = fmaf(b.FpR[(int64_t)n * N + j], dg2[n], sj);
        }
      } else {
#pragma unroll
        for (int n = 0; n < NR; ++n) {
          si = fmaf(fpi[n], dg[n], si);
          sj = fmaf(b.FpR[(int64_t)n * N + j], dg[n], sj);
        }
      }
      const float ux = dx * rinv, uy = dy * rinv, uz = dz * rinv;
      const float st = (si + sj);
      fx = fmaf(st, ux, fx);
      fy = fmaf(st, uy, fy);
      fz = fmaf(st, uz, fz);
      // virial of dU_i/dr_ij = si u
      const float d[3] = {dx, dy, dz};
      const float f[3] = {si * ux, si * uy, si * uz};
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) w[a * 3 + c] = fmaf(-d[a], f[c], w[a * 3 + c]);
    }
    // angular + four-body: scatter
    float G[NA * NC];
#pragma unroll
    for (int k = 0; k < NA * NC; ++k) G[k] = b.G[(int64_t)k * N + i];
    const int na = b.nactA[i];
    for (int p = 0; p < na; ++p) {
      const int32_t j = b.actA[(int64_t)p * N + i];
      float dx, dy, dz;
      pair_vec(x, N, j, xi, yi, zi, Lx, Ly, Lz, dx, dy, dz);
      const float r = sqrtf(dx * dx + dy * dy + dz * dz);
      const float rinv = 1.f / r;
      const int tj = MULTI ? b.type[j] : 0;
      float g[NA], dg[NA];
      radial_g_dg<NA, S::KA>(r, rcA_inv, m.cA + (ti * m.T + tj) * NA * S::KA, g, dg);
      const float ux = dx * rinv, uy = dy * rinv, uz = dz * rinv;
      float sc = 0.f, vx = 0.f, vy = 0.f, vz = 0.f;
      for_each_poly_grad<NC>(ux, uy, uz, [&](int lm, float P, float px, float py, float pz) {
        float A = 0.f, B = 0.f;
#pragma unroll
        for (int n = 0; n < NA; ++n) {
          A = fmaf(G[n * NC + lm], dg[n], A);
          B = fmaf(G[n * NC + lm], g[n], B);
        }
        sc = fmaf(P, A - (float)comp_l(lm) * rinv * B, sc);
        vx = fmaf(B, px, vx);
        vy = fmaf(B, py, vy);
        vz = fmaf(B, pz, vz);
      });
      const float f0 = fmaf(ux, sc, vx * rinv);
      const float f1 = fmaf(uy, sc, vy * rinv);
      const float f2 = fmaf(uz, sc, vz * rinv);
      fx += f0;
      fy += f1;
      fz += f2;
      unsafeAtomicAdd(&b.F[j], -f0);
      unsafeAtomicAdd(&b.F[N + j], -f1);
      unsafeAtomicAdd(&b.F[2 * N + j], -f2);
      const float d[3] = {dx, dy, dz};
      const float f[3] = {f0, f1, f2};
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) w[a * 3 + c] = fmaf(-d[a], f[c], w[a * 3 + c]);
    }
    unsafeAtomicAdd(&b.F[i], fx);
    unsafeAtomicAdd(&b.F[N + i], fy);
    unsafeAtomicAdd(&b.F[2 * N + i], fz);
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const double t = block_sum((double)w[k], red);
    if (threadIdx.x == 0) b.partial[(int64_t)tile * kPartialStride + P_VIR + k] = t;
  }
}

template <class S, int PREC, bool MULTI>
hipError_t launch_pair(const ModelDev& m, const EvalBuffers& b, hipStream_t st, hipEvent_t* ev) {
  const int nb = grid_blocks(b.N);
  if (ev) (void)hipEventRecord(ev[0], st);
  hipLaunchKernelGGL((k_desc_net<S, PREC, MULTI>), dim3(nb), dim3(kBlock), 0, st, m, b);
  if (ev) (void)hipEventRecord(ev[1], st);
  hipLaunchKernelGGL((k_force<S, MULTI>), dim3(nb), dim3(kBlock), 0, st, m, b);
  if (ev) (void)hipEventRecord(ev[2], st);
  return hipGetLastError();
}

template <class S>
hipError_t launch_shape(const ModelDev& m, int precision, const EvalBuffers& b, hipStream_t st,
                        hipEvent_t* ev) {
  const bool multi = m.T > 1;
  if (precision == 0)
    return multi ? launch_pair<S, 0, true>(m, b, st, ev) : launch_pair<S, 0, false>(m, b, st, ev);
  return multi ? launch_pair<S, 1, true>(m, b, st, ev) : launch_pair<S, 1, false>(m, b, st, ev);
}

template <class S>
bool is_shape(const ModelDev& m) {
  return m.nR == S::NR && m.kR == S::KR && m.nA == S::NA && m.kA == S::KA && m.L3 == S::L3 &&
         (m.L4 == 2) == S::FB && m.H == S::H && m.T >= 1 && m.T <= kMaxTypes;
}

}  // namespace

bool eval_supported(const ModelDev& m) { return is_shape<FullShape>(m) || is_shape<SurShape>(m); }

int eval_partial_blocks(int64_t N) { return grid_blocks(N); }

hipError_t launch_eval(const ModelDev& m, int precision, const EvalBuffers& b, hipStream_t st,
                       hipEvent_t* ev) {
  if (is_shape<FullShape>(m)) return launch_shape<FullShape>(m, precision, b, st, ev);
  if (is_shape<SurShape>(m)) return launch_shape<SurShape>(m, precision, b, st, ev);
  return hipErrorInvalidValue;
}

}  // namespace nep
