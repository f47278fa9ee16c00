// Pair arithmetic of the evaluation kernels (k_desc_net, k_force), written for the
// fewest VALU instructions per pair: the cutoff function from short Taylor series on
// the one interval it needs, the Chebyshev basis through the recurrences of both kinds
// with model-derived coefficient tables, the single-species radial force by Clenshaw's
// recurrence, and a neighbour loop whose prefetch buffers rotate without copies.
// The training kernels keep the direct forms of nep_kernels.h.
#pragma once

#include "nep_kernels.h"

namespace nep {
namespace kern {

// ---------------------------------------------------------------- cutoff function
// f_c = (1 + cos(pi t)) / 2 for t = r / r_c in [0, 1) (the cosine cutoff: value and slope
// vanish at r_c). With psi = pi t - pi/2 in [-pi/2, pi/2): cos(pi t) = -sin(psi) and
// sin(pi t) = cos(psi). sin and cos of psi come from their Taylor series through psi^13
// and psi^14; on |psi| <= pi/2 the remainders are below |psi|^15 / 15! < 7e-10 and
// |psi|^16 / 16! < 7e-11, under the FP32 rounding of the result.
constexpr float kHalfPiF = 1.57079632679489661923f;

__device__ __forceinline__ float taylor_sin(float psi, float p2) {
  float a = (float)(1.0 / 6227020800.0);  // 1/13!
  a = fmaf(a, p2, (float)(-1.0 / 39916800.0));
  a = fmaf(a, p2, (float)(1.0 / 362880.0));
  a = fmaf(a, p2, (float)(-1.0 / 5040.0));
  a = fmaf(a, p2, (float)(1.0 / 120.0));
  a = fmaf(a, p2, (float)(-1.0 / 6.0));
  return fmaf(psi * p2, a, psi);
}

__device__ __forceinline__ float taylor_cos(float p2) {
  float a = (float)(-1.0 / 87178291200.0);  // -1/14!
  a = fmaf(a, p2, (float)(1.0 / 479001600.0));
  a = fmaf(a, p2, (float)(-1.0 / 3628800.0));
  a = fmaf(a, p2, (float)(1.0 / 40320.0));
  a = fmaf(a, p2, (float)(-1.0 / 720.0));
  a = fmaf(a, p2, (float)(1.0 / 24.0));
  a = fmaf(a, p2, -0.5f);
  return fmaf(a, p2, 1.f);
}

// Constants of one cutoff radius, uniform over a launch.
struct CutConst {
  float rc_inv;     // 1 / r_c
  float pi_rc_inv;  // pi / r_c (rounded once from FP64)
};
__device__ __forceinline__ CutConst cut_const(float rc) {
  return {1.f / rc, (float)(3.14159265358979323846 / (double)rc)};
}

// Geometry of one pair at distance r < r_c, t = r / r_c: f_c, the Chebyshev argument
// x = 2 (t - 1)^2 - 1 of the radial basis, and for the r-derivatives c = sin(pi t) and
// y = t - 1, with which d f_c / dr = -(pi / 2) c / r_c and d x / dr = 4 y / r_c.
// psi and y are taken from r in one rounding each (r pi / r_c - pi / 2, r / r_c - 1).
struct RadialGeo {
  float fc, x, c, y;
};
template <bool DERIV>
__device__ __forceinline__ RadialGeo radial_geo(float r, const CutConst& k) {
  const float psi = fmaf(r, k.pi_rc_inv, -kHalfPiF);
  const float p2 = psi * psi;
  const float y = fmaf(r, k.rc_inv, -1.f);
  RadialGeo g;
  g.fc = fmaf(-0.5f, taylor_sin(psi, p2), 0.5f);
  g.x = fmaf(y + y, y, -1.f);
  g.y = y;
  g.c = DERIV ? taylor_cos(p2) : 0.f;
  return g;
}

// Derived coefficient table of one (center type, neighbour type) block of N channels
// and K basis functions, [N][2K - 1] floats: h_n0 = (c_n0 + sum_k c_nk) / 2,
// h_nk = c_nk / 2 (k >= 1), then d_n(k-1) = k c_nk / 2 (k >= 1). With them
//   g_n  = f_c (h_n0 + sum_{k>=1} h_nk T_k(x))                       = f_c C_n
//   g_n' = f_c' C_n + f_c x' sum_{k>=1} d_n(k-1) U_{k-1}(x)          = f_c' C_n + f_c x' D_n
// which are sum_k c_nk f_k and its r-derivative for f_k = f_c (T_k + 1) / 2.
template <int N, int K>
constexpr int derived_block() { return N * (2 * K - 1); }

// g_n = f_c C_n. Runs over k outermost with the recurrence rolled along, so that only
// the channel sums and three terms of the recurrence are live.
template <int N, int K, class CP>
__device__ __forceinline__ void radial_g_fast(float fc, float x, CP h, float* g) {
  float a[N];
#pragma unroll
  for (int n = 0; n < N; ++n) a[n] = h[n * K];
  const float x2 = x + x;
  float Tm = 1.f, T = x;  // T_{k-1}, T_k
#pragma unroll
  for (int k = 1; k < K; ++k) {
#pragma unroll
    for (int n = 0; n < N; ++n) a[n] = fmaf(h[n * K + k], T, a[n]);
    const float Tn = fmaf(x2, T, -Tm);
    Tm = T;
    T = Tn;
  }
#pragma unroll
  for (int n = 0; n < N; ++n) g[n] = fc * a[n];
}

// The channel sums C_n and D_n themselves (the caller applies f_c, f_c' and x').
template <int N, int K, class CP>
__device__ __forceinline__ void radial_cd_fast(float x, CP h, float* C, float* D) {
#pragma unroll
  for (int n = 0; n < N; ++n) {
    C[n] = h[n * K];                // k = 0 of C_n
    D[n] = h[N * K + n * (K - 1)];  // k = 1 of D_n (U_0 = 1)
  }
  const float x2 = x + x;
  float Tm = 1.f, T = x;  // T_{k-1}, T_k
  float Um = 1.f, Uc = x2;   // U_{k-2}, U_{k-1} for the D term of index k + 1
#pragma unroll
  for (int k = 1; k < K; ++k) {
#pragma unroll
    for (int n = 0; n < N; ++n) C[n] = fmaf(h[n * K + k], T, C[n]);
    if (k + 1 < K) {
      // D_n term k + 1: d_nk U_k, with U_k in Uc
#pragma unroll
      for (int n = 0; n < N; ++n) D[n] = fmaf(h[N * K + n * (K - 1) + k], Uc, D[n]);
      const float Un = fmaf(x2, Uc, -Um);
      Um = Uc;
      Uc = Un;
    }
    const float Tn = fmaf(x2, T, -Tm);
    Tm = T;
    T = Tn;
  }
}

// Radial pair force of one species. The r-derivative of sum_k W_k f_k(r), for
// f_k = f_c (T_k(x) + 1) / 2, is X = (f_c' (C + sum_k W_k) + f_c x' C'(x)) / 2 with the
// Chebyshev series C(x) = sum_k W_k T_k(x); with f_c' and x' from the pair geometry,
//   X = -(pi / (4 r_c)) Z,   Z = c (C + sum_k W_k) + f_c y S C'(x),   S = -8 / pi.
// C and C' by Clenshaw's recurrence b_k = W_k + 2x b_{k+1} - b_{k+2} (k >= 1) and its
// x-derivative, carried scaled by S: e_k = 2 S b_{k+1} + 2x e_{k+1} - e_{k+2}; then
// C = W_0 + x b_1 - b_2, C + sum_k W_k = V + x b_1 - b_2 and S C' = S b_1 + x e_1 - e_2.
// Takes W_1..W_{K-1} and V = W_0 + sum_k W_k; returns Z. The first three steps, where
// b_K, e_K and e_{K-1} vanish, are written out.
constexpr float kDerivScale = -8.f / kPiF;
template <int K>
__device__ __forceinline__ float radial_series_z(const RadialGeo& g, const float* W, float V) {
  static_assert(K >= 4, "three steps are written out");
  constexpr float S2 = 2.f * kDerivScale;
  const float x2 = g.x + g.x;
  float b2 = W[K - 1];                 // b_{K-1}
  float b1 = fmaf(x2, b2, W[K - 2]);   // b_{K-2}
  float e1 = S2 * b2, e2;              // e_{K-2} (e_{K-1} = 0)
  {
    const float bk = fmaf(x2, b1, W[K - 3] - b2);
    const float ek = fmaf(x2, e1, S2 * b1);
    b2 = b1;
    b1 = bk;
    e2 = e1;
    e1 = ek;
  }
#pragma unroll
  for (int k = K - 4; k >= 1; --k) {
    const float bk = fmaf(x2, b1, W[k] - b2);
    const float ek = fmaf(x2, e1, fmaf(S2, b1, -e2));
    b2 = b1;
    b1 = bk;
    e2 = e1;
    e1 = ek;
  }
  const float Cs = fmaf(g.x, b1, V - b2);
  const float Cp = fmaf(g.x, e1, fmaf(kDerivScale, b1, -e2));
  return fmaf(g.c, Cs, (g.fc * g.y) * Cp);
}

// ---------------------------------------------------------------- activation
// tanh z = 1 - 2 / (e^{2z} + 1), with e^{2z} = 2^{2 z log2(e)} from the hardware base-2
// exponential and the hardware reciprocal (about 1 ulp each): absolute error within a few
// 1e-7 over the whole range, with no branch; for large |z| e^{2z} overflows to infinity or
// underflows to 0 and the result saturates to +1 or -1 exactly.
__device__ __forceinline__ float tanh_fast(float z) {
  const float e = __builtin_amdgcn_exp2f(z * 2.88539008177792681f);  // 2 / ln 2
  return fmaf(-2.f, __builtin_amdgcn_rcpf(e + 1.f), 1.f);
}

// ---------------------------------------------------------------- pair vectors
// Pair vector x_j - x_i of a list neighbour from the 32-bit box fractions (of the position
// array or the records): the two's-complement difference is the minimum image in units of
// the quantum; it is converted to FP64 exactly, scaled by the quantum (h = L / 2^32) and
// rounded once to FP32. Returns r^2 in FP32.
struct QPos {
  uint32_t x, y, z;
};
__device__ __forceinline__ float pair_vec_q(const uint4& wj, const QPos& qi, double hx, double hy, double hz,
                                            float& dx, float& dy, float& dz) {
  dx = (float)((double)(int32_t)(wj.x - qi.x) * hx);
  dy = (float)((double)(int32_t)(wj.y - qi.y) * hy);
  dz = (float)((double)(int32_t)(wj.z - qi.z) * hz);
  return fmaf(dx, dx, fmaf(dy, dy, dz * dz));
}

// r and 1/r from an FP32 r^2 (hardware reciprocal square root, 1 ulp).
__device__ __forceinline__ void r_of_r2(float r2, float& r, float& rinv) {
  rinv = __builtin_amdgcn_rsqf(r2);
  r = r2 * rinv;
}

// ---------------------------------------------------------------- neighbour loops
// Both visit entries [k0, k1) of atom i's slot-major list, calling body(p, j, w) with the
// first W 16-byte words of neighbour j's entry in rec (RS words per atom: the position
// array with RS = 1, the 64-byte records with RS = 4). The records of entries p + 1 .. p + AHEAD
// and the index of entry p + AHEAD + 1 are in flight while the body of entry p runs, so
// their latency overlaps the pair arithmetic; bodies with little arithmetic per pair need
// the deeper queue. The loads run past k1 - 1 by up to AHEAD + 1 rows, into entries that
// are not visited (later bins, stale entries, or the kListPad rows past the capacity),
// which hold indices of atoms of the system, so every address stays inside the list and
// the records; the index loads walk down the column by a pointer step of one row.
//
// for_each_rec_span moves the queue along by register copies; for_each_rec_fast is
// unrolled AHEAD + 1 times so that each record is loaded straight into the buffer the
// body later reads (a rotation by index, not by copies), at the cost of a few more live
// registers.
template <int W, int AHEAD, int RS, class Body>
__device__ __forceinline__ void for_each_rec_span(const int32_t* __restrict__ nbr, const uint4* __restrict__ rec,
                                                  int64_t N, int64_t i, int k0, int k1, Body&& body) {
  static_assert(AHEAD >= 1 && AHEAD + 1 <= kListPad, "prefetch depth within the list's padding");
  if (k1 <= k0) return;
  const uint64_t n64 = (uint64_t)N;
  const int32_t* __restrict__ col = nbr + i + (uint64_t)(uint32_t)k0 * n64;  // entry k0
  auto record = [&](int32_t j, int w) { return rec[(uint64_t)(uint32_t)j * RS + w]; };
  int32_t jq[AHEAD + 1];  // indices of entries p .. p + AHEAD
#pragma unroll
  for (int a = 0; a <= AHEAD; ++a) {
    jq[a] = *col;
    col += n64;
  }
  uint4 rq[AHEAD][W];  // records of entries p .. p + AHEAD - 1
#pragma unroll
  for (int a = 0; a < AHEAD; ++a)
#pragma unroll
    for (int w = 0; w < W; ++w) rq[a][w] = record(jq[a], w);
  for (int p = k0; p < k1; ++p) {
    const int32_t jn = *col;  // entry p + AHEAD + 1
    col += n64;
    uint4 rn[W];
#pragma unroll
    for (int w = 0; w < W; ++w) rn[w] = record(jq[AHEAD], w);
    body(p, jq[0], rq[0]);
#pragma unroll
    for (int a = 0; a < AHEAD; ++a) jq[a] = jq[a + 1];
    jq[AHEAD] = jn;
#pragma unroll
    for (int a = 0; a + 1 < AHEAD; ++a)
#pragma unroll
      for (int w = 0; w < W; ++w) rq[a][w] = rq[a + 1][w];
#pragma unroll
    for (int w = 0; w < W; ++w) rq[AHEAD - 1][w] = rn[w];
  }
}

template <int W, int AHEAD, int RS, class Body>
__device__ __forceinline__ void for_each_rec_fast(const int32_t* __restrict__ nbr, const uint4* __restrict__ rec,
                                                  int64_t N, int64_t i, int k0, int k1, Body&& body) {
  static_assert(AHEAD >= 1 && AHEAD <= 3 && AHEAD + 1 <= kListPad, "prefetch depth within the list's padding");
  constexpr int U = AHEAD + 1;
  if (k1 <= k0) return;
  const uint64_t n64 = (uint64_t)N;
  const int32_t* __restrict__ col = nbr + i + (uint64_t)(uint32_t)k0 * n64;  // entry k0
  auto record = [&](int32_t j, int w) { return rec[(uint64_t)(uint32_t)j * RS + w]; };
  int32_t jq[AHEAD + 1];  // indices of entries p .. p + AHEAD
#pragma unroll
  for (int a = 0; a <= AHEAD; ++a) {
    jq[a] = *col;
    col += n64;
  }
  uint4 rq[U][W];  // record buffers; entry p sits in buffer (p - k0) % U
#pragma unroll
  for (int a = 0; a < AHEAD; ++a)
#pragma unroll
    for (int w = 0; w < W; ++w) rq[a][w] = record(jq[a], w);
  for (int p0 = k0; p0 < k1; p0 += U) {
#pragma unroll
    for (int ph = 0; ph < U; ++ph) {
      const int p = p0 + ph;
      if (p < k1) {
        const int32_t jn = *col;  // entry p + AHEAD + 1
        col += n64;
#pragma unroll
        for (int w = 0; w < W; ++w) rq[(ph + AHEAD) % U][w] = record(jq[AHEAD], w);
        body(p, jq[0], rq[ph]);
#pragma unroll
        for (int a = 0; a < AHEAD; ++a) jq[a] = jq[a + 1];
        jq[AHEAD] = jn;
      }
    }
  }
}

// ---------------------------------------------------------------- structural zeros
// Gradient components of the harmonic polynomials that vanish identically are passed as
// Zero, so that their products drop out at compile time (an FP32 product with a literal
// 0.0 cannot be removed by the compiler, since it must keep NaN and signed-zero results).
__device__ __forceinline__ float fmac(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ float fmac(float, Zero, float c) { return c; }
__device__ __forceinline__ float fmac(Zero, float, float c) { return c; }

}  // namespace kern
}  // namespace nep
