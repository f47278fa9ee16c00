// Device helpers shared by the evaluation and training kernels: radial basis,
// pair vectors, workgroup reductions, model shapes, and the descriptor
// accumulation of one center (radial q_n, angular s_nlm, q_nl, four-body).
#pragma once

#include "nep_common.h"
#include "nep_poly.h"

namespace nep {
namespace kern {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr float kPiF = 3.14159265358979323846f;

// Read-only view of model coefficients in the constant address space: where the
// index is the same for the whole wavefront (one species) the compiler loads the
// block with scalar loads, keeping it out of vector registers.
typedef const __attribute__((address_space(4))) float* cfloat_ptr;
__device__ __forceinline__ cfloat_ptr uniform_coeffs(const float* p) { return (cfloat_ptr)p; }

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
template <int N, int K, class CP>
__device__ __forceinline__ void radial_g(float r, float rc_inv, CP c, float* g) {
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
template <int N, int K, class CP>
__device__ __forceinline__ void radial_g_dg(float r, float rc_inv, CP c, float* g, float* dg) {
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

// The radial basis itself, f_k = f_c (T_k + 1)/2 for k < K. For one species the
// radial descriptors are linear in it, q_n = sum_k c_nk sum_j f_k(r_ij), so a center
// accumulates the K basis sums and contracts with c once.
template <int K>
__device__ __forceinline__ void radial_basis(float r, float rc_inv, float* f) {
  float sn, cs;
  sincospif(r * rc_inv, &sn, &cs);
  const float fc = 0.5f * (1.f + cs);
  const float y = r * rc_inv - 1.f;
  const float x = 2.f * y * y - 1.f;
  const float hf = 0.5f * fc;
  float Tm1 = 1.f, T = x;
  f[0] = fc;
  f[1] = fmaf(hf, x, hf);
#pragma unroll
  for (int k = 2; k < K; ++k) {
    const float Tn = 2.f * x * T - Tm1;
    Tm1 = T;
    T = Tn;
    f[k] = fmaf(hf, Tn, hf);
  }
}

// e_k = d f_k / dr. For one species dU_i/dr_ij = sum_k w_ik e_k(r_ij) with
// w_ik = sum_n (dU_i/dq_n) c_nk formed once per center.
template <int K>
__device__ __forceinline__ void radial_basis_deriv(float r, float rc_inv, float* e) {
  float sn, cs;
  sincospif(r * rc_inv, &sn, &cs);
  const float fc = 0.5f * (1.f + cs);
  const float dfc = -0.5f * kPiF * rc_inv * sn;
  const float y = r * rc_inv - 1.f;
  const float x = 2.f * y * y - 1.f;
  const float hfd = 2.f * y * rc_inv * fc;  // (f_c / 2) dx/dr
  const float hdf = 0.5f * dfc;
  float Tm1 = 1.f, T = x, dTm1 = 0.f, dT = 1.f;
  e[0] = dfc;
  e[1] = fmaf(hdf, x + 1.f, hfd);
#pragma unroll
  for (int k = 2; k < K; ++k) {
    const float Tn = 2.f * x * T - Tm1;
    const float dTn = 2.f * T + 2.f * x * dT - dTm1;
    Tm1 = T;
    T = Tn;
    dTm1 = dT;
    dT = dTn;
    e[k] = fmaf(hdf, Tn + 1.f, hfd * dTn);
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

// Deterministic FP64 sums of K values over a 256-thread workgroup: a butterfly over the
// 64 lanes of each wavefront (cross-lane moves, no barrier), then the four wavefront
// partials in a fixed order, with one barrier for all K. The result is valid in thread 0.
// sh holds at least 4 K doubles.
template <int K>
__device__ __forceinline__ void block_sum_n(const double* v, double* out, double* sh) {
  double t[K];
#pragma unroll
  for (int k = 0; k < K; ++k) t[k] = v[k];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int k = 0; k < K; ++k) t[k] += __shfl_xor(t[k], off, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();  // sh may still be read by an earlier use
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) sh[w * K + k] = t[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = (sh[k] + sh[K + k]) + (sh[2 * K + k] + sh[3 * K + k]);
}


template <int NR_, int KR_, int NA_, int KA_, int L3_, bool FB_, int H_>
struct Shape {
  static constexpr int NR = NR_, KR = KR_, NA = NA_, KA = KA_, L3 = L3_, H = H_;
  static constexpr bool FB = FB_;
  static constexpr int NC = L3 * (L3 + 2);
  static constexpr int D = NR + NA * L3 + (FB ? NA : 0);
  // neighbour positions in flight ahead of the pair the descriptor pass works on: with
  // l <= 2 that pass does too little arithmetic per pair to hide one gather's latency
  // (the force passes gather 64-byte records and stay at one ahead: a deeper queue there
  // loses more to memory contention than it hides)
  static constexpr int DESC_AHEAD = L3 <= 2 ? 2 : 1;
  static_assert(D <= 32 && H <= 32, "network tiles hold at most 32 descriptors and 32 hidden units");
  static_assert(NR <= 10 && KR <= 10, "the neighbour record holds 10 radial coefficients");
  static_assert(!FB || L3 >= 2, "the four-body term uses the l = 2 accumulators");
};

using FullShape = Shape<5, 9, 5, 9, 4, true, 30>;
using SurShape = Shape<5, 9, 5, 9, 2, false, 8>;

constexpr int kLdsStride = 33;  // 32 columns + 1 pad word against bank conflicts


// r and 1/r of an FP32 pair vector (hardware reciprocal square root, 1 ulp).
__device__ __forceinline__ void pair_r(float dx, float dy, float dz, float& r, float& rinv) {
  const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
  rinv = __builtin_amdgcn_rsqf(r2);
  r = r2 * rinv;
}

// Pair test for an entry whose position is already loaded: FP64 minimum-image
// vector, kept when r^2 < cut2; rounded to FP32 after the subtraction.
__device__ __forceinline__ bool inside(double xj, double yj, double zj, double xi, double yi, double zi,
                                       double Lx, double Ly, double Lz, double cut2, float& dx, float& dy,
                                       float& dz) {
  const double ex = min_image(xj - xi, Lx);
  const double ey = min_image(yj - yi, Ly);
  const double ez = min_image(zj - zi, Lz);
  if (!(ex * ex + ey * ey + ez * ez < cut2)) return false;
  dx = (float)ex;
  dy = (float)ey;
  dz = (float)ez;
  return true;
}

// Pair test for one entry of a list with skin: FP64 minimum-image vector, kept when
// r^2 < cut2 (the true cutoff); the vector is rounded to FP32 after the subtraction.
__device__ __forceinline__ bool pair_inside(const double* __restrict__ x, int64_t N, int32_t j, double xi,
                                            double yi, double zi, double Lx, double Ly, double Lz, double cut2,
                                            float& dx, float& dy, float& dz) {
  const double ex = min_image(x[j] - xi, Lx);
  const double ey = min_image(x[N + j] - yi, Ly);
  const double ez = min_image(x[2 * N + j] - zi, Lz);
  if (!(ex * ex + ey * ey + ez * ez < cut2)) return false;
  dx = (float)ex;
  dy = (float)ey;
  dz = (float)ez;
  return true;
}

// Number of list entries of atom i the current evaluation must visit for radial
// (resp. angular) pairs: the entries of the distance bins those pairs can have
// reached since the last build. The angular bound never exceeds the radial one.
__device__ __forceinline__ int radial_bound(const EvalBuffers& b, int64_t i) {
  return b.bp[(int64_t)b.flags[b.flag_r] * b.N + i];
}
__device__ __forceinline__ int angular_bound(const EvalBuffers& b, int64_t i) {
  return b.bp[(int64_t)b.flags[b.flag_a] * b.N + i];
}

// ZBL universal screened Coulomb repulsion of one pair at distance r (the published
// Ziegler-Biersack-Littmark form, added to the Cu and HfO2 models in Section VI.A):
// phi = k_e Z_i Z_j / r * sum_m c_m exp(-d_m r / a) times a switch that is 1 below
// zbl_ri and (1 + cos(pi (r - zbl_ri) / (zbl_ro - zbl_ri))) / 2 up to zbl_ro.
// Returns the switched energy e and de = d e / d r, in FP64: only the rare pairs
// inside the ZBL radius get here, and the repulsion is steep enough there that an
// FP32 distance would cost several FP32 roundings of the atom's energy.
template <bool MULTI>
__device__ __forceinline__ void zbl_pair(const ModelDev& m, int tp, double r, double& e, double& de) {
  double kzz = m.zbl_kzz[0], ainv = m.zbl_ainv[0];
  if constexpr (MULTI) {
#pragma unroll
    for (int k = 1; k < kMaxTypes * kMaxTypes; ++k) {
      kzz = tp == k ? m.zbl_kzz[k] : kzz;
      ainv = tp == k ? m.zbl_ainv[k] : ainv;
    }
  }
  constexpr double c[4] = {0.18175, 0.50986, 0.28022, 0.02817};
  constexpr double d[4] = {3.19980, 0.94229, 0.40290, 0.20162};
  double S = 0.0, dS = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double t = c[k] * exp(-d[k] * ainv * r);
    S += t;
    dS -= d[k] * ainv * t;
  }
  const double rinv = 1.0 / r;
  const double phi = kzz * rinv * S;
  const double dphi = kzz * rinv * (dS - S * rinv);
  double sw = 1.0, dsw = 0.0;
  if (r >= m.zbl_ri) {
    const double w = 3.14159265358979323846 / (m.zbl_ro - m.zbl_ri);
    sw = 0.5 * (1.0 + cos(w * (r - m.zbl_ri)));
    dsw = -0.5 * w * sin(w * (r - m.zbl_ri));
  }
  e = phi * sw;
  de = dphi * sw + phi * dsw;
}

// Minimum image of a list pair's FP64 component as d - L rint(d / L) (one multiply,
// one rounding, one fused multiply-add instead of two compares and selects of 64-bit
// values). L rint(d / L) is 0 or +-L exactly, so the result is the rule's d, d - L or
// d + L rounded once, as the rule gives it, except when |d| is within rounding of L/2;
// there both candidates lie at L/2 >= rc + skin from the center, outside every cutoff.
__device__ __forceinline__ double min_image_list(double d, double L, double inv_L) {
  return fma(-L, rint(d * inv_L), d);
}

// FP64 minimum-image vector of a list pair whose position is loaded and its r^2.
__device__ __forceinline__ double pair_r2_64(double xj, double yj, double zj, double xi, double yi, double zi,
                                             double Lx, double Ly, double Lz, double iLx, double iLy, double iLz,
                                             double& ex, double& ey, double& ez) {
  ex = min_image_list(xj - xi, Lx, iLx);
  ey = min_image_list(yj - yi, Ly, iLy);
  ez = min_image_list(zj - zi, Lz, iLz);
  return ex * ex + ey * ey + ez * ez;
}

// Close pairs (inside the outer ZBL radius) seen by a main loop: their count and
// the list positions of the first CAP of them, 16 bits each (CAP = 0: count only,
// for kernels with no registers to spare).
template <int CAP>
struct ZblSeen {
  static_assert(CAP >= 0 && CAP <= 4, "four 16-bit slots");
  int n = 0;
  uint64_t slots = 0;
  __device__ __forceinline__ void add(int p) {
    if constexpr (CAP > 0) {
      if (n < CAP) slots |= (uint64_t)p << (16 * n);
    }
    ++n;
  }
};
template <bool MULTI>
using ZblSeenFor = ZblSeen<MULTI ? 0 : 4>;

// ZBL terms of center i (the pairs with r^2 < zbl_o2): half of each pair's energy
// into uz, and, when f is given, the force on i (the whole pair derivative, both
// atoms' halves, along u) into f[3] and the virial of dU_i/dr_ij into w[9]. Called
// only for centers that have such pairs, after the main loop: it visits the
// recorded list positions, or the whole radial list when there were more.
template <bool MULTI, int CAP>
__device__ __forceinline__ void zbl_center(const ModelDev& m, const EvalBuffers& b, int64_t i, int ti, double xi,
                                        double yi, double zi, const ZblSeen<CAP>& seen, float* uz, float* f,
                                        float* w) {
  const int64_t N = b.N;
  const double Lx = b.box[0], Ly = b.box[1], Lz = b.box[2];
  const bool all = seen.n > CAP;
  const int kR = all ? radial_bound(b, i) : seen.n;
  for (int q = 0; q < kR; ++q) {
    const int p = all ? q : (int)((seen.slots >> (16 * q)) & 0xffffu);
    const int32_t j = b.nbr[(int64_t)p * N + i];
    const double ex = min_image(b.x[j] - xi, Lx);
    const double ey = min_image(b.x[N + j] - yi, Ly);
    const double ez = min_image(b.x[2 * N + j] - zi, Lz);
    const double r2 = ex * ex + ey * ey + ez * ez;
    if (!(r2 < m.zbl_o2)) continue;
    const double r = sqrt(r2);
    const int tj = MULTI ? b.type[j] : 0;
    double e, de;
    zbl_pair<MULTI>(m, ti * m.T + tj, r, e, de);
    if (uz) *uz += (float)(0.5 * e);
    if (f) {
      const double d[3] = {ex, ey, ez};
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double fa = de * d[a] / r;  // both halves of the pair derivative along u
        f[a] += (float)fa;
#pragma unroll
        for (int c = 0; c < 3; ++c) w[a * 3 + c] += (float)(-d[a] * 0.5 * de * d[c] / r);
      }
    }
  }
}

// Radial descriptors q[0..NR) and angular accumulators s[NA][NC] of center i over
// the pairs inside the true cutoffs, all channels in one pass over the neighbours
// (geometry computed once per pair and reused for every n). Returns the pair counts
// and the pairs inside the ZBL radius (zs).
template <class S, bool MULTI>
__device__ __forceinline__ void desc_accumulate(const ModelDev& m, const EvalBuffers& b, int64_t i, int ti,
                                                double xi, double yi, double zi, double Lx, double Ly,
                                                double Lz, float* q, float* s, ZblSeenFor<MULTI>& zs, int& nr,
                                                int& na) {
  constexpr int NR = S::NR, NA = S::NA, NC = S::NC;
  const int64_t N = b.N;
  const float rcR_inv = 1.f / m.rcR, rcA_inv = 1.f / m.rcA;
  const double rcR2 = m.rcR64 * m.rcR64, rcA2 = m.rcA64 * m.rcA64;
  const double iLx = 1.0 / Lx, iLy = 1.0 / Ly, iLz = 1.0 / Lz;
  nr = 0;
  na = 0;
  const float* cR = m.cR + (MULTI ? 0 : (ti * m.T) * NR * S::KR);
  const float* cA = m.cA + (MULTI ? 0 : (ti * m.T) * NA * S::KA);
  const int kR = radial_bound(b, i), kA = angular_bound(b, i);
  float Qb[S::KR];  // basis sums (one species)
#pragma unroll
  for (int k = 0; k < S::KR; ++k) Qb[k] = 0.f;
  // one pass over the list: radial terms for every pair inside rc_radial, angular
  // terms for the pairs of the angular prefix inside rc_angular; FP64 positions from
  // the position array (these kernels serve training, not the MD step)
  for (int p = 0; p < kR; ++p) {
    const int32_t j = b.nbr[(int64_t)p * N + i];
    double ex, ey, ez;
    const double r2 = pair_r2_64(b.x[j], b.x[N + j], b.x[2 * N + j], xi, yi, zi, Lx, Ly, Lz, iLx, iLy, iLz, ex,
                                 ey, ez);
    if (!(r2 < rcR2)) continue;
    const float dx = (float)ex, dy = (float)ey, dz = (float)ez;
    ++nr;
    float r, rinv;
    pair_r(dx, dy, dz, r, rinv);
    const int tj = MULTI ? b.type[j] : 0;
    if (r2 < m.zbl_o2) zs.add(p);
    if constexpr (MULTI) {
      float g[NR];
      radial_g<NR, S::KR>(r, rcR_inv, m.cR + (ti * m.T + tj) * NR * S::KR, g);
#pragma unroll
      for (int n = 0; n < NR; ++n) q[n] += g[n];
    } else {
      float f[S::KR];
      radial_basis<S::KR>(r, rcR_inv, f);
#pragma unroll
      for (int k = 0; k < S::KR; ++k) Qb[k] += f[k];
    }
    if (p < kA && r2 < rcA2) {
      ++na;
      float g[NA];
      if constexpr (MULTI)
        radial_g<NA, S::KA>(r, rcA_inv, m.cA + (ti * m.T + tj) * NA * S::KA, g);
      else
        radial_g<NA, S::KA>(r, rcA_inv, uniform_coeffs(cA), g);
      for_each_poly<NC>(dx * rinv, dy * rinv, dz * rinv, [&](int lm, float P) {
#pragma unroll
        for (int n = 0; n < NA; ++n) s[n * NC + lm] = fmaf(g[n], P, s[n * NC + lm]);
      });
    }
  }
  if constexpr (!MULTI) {
    const cfloat_ptr c = uniform_coeffs(cR);
#pragma unroll
    for (int n = 0; n < NR; ++n) {
      float a = 0.f;
#pragma unroll
      for (int k = 0; k < S::KR; ++k) a = fmaf(c[n * S::KR + k], Qb[k], a);
      q[n] += a;
    }
  }
}

// The 3x3 traceless matrix S = sum_j g (u u^T - I/3) of one channel from its
// l = 2 accumulators (xy, yz, 3z^2 - r^2, xz, x^2 - y^2).
struct Sym3 {
  float xx, yy, zz, xy, yz, xz;
};
__device__ __forceinline__ Sym3 s_matrix(const float* sl) {
  Sym3 a;
  a.xy = sl[3];
  a.yz = sl[4];
  a.zz = sl[5] * (1.f / 3.f);
  a.xz = sl[6];
  a.xx = 0.5f * (sl[7] - a.zz);
  a.yy = 0.5f * (-sl[7] - a.zz);
  return a;
}

// q_nl = sum_m W_lm s_nlm^2 and the four-body invariant tr(S^3) = 3 det S.
template <class S>
__device__ __forceinline__ void desc_finish(const float* s, float* q) {
  constexpr int NR = S::NR, NA = S::NA, NC = S::NC;
#pragma unroll
  for (int n = 0; n < NA; ++n)
#pragma unroll
    for (int lm = 0; lm < NC; ++lm) {
      const int l = comp_l(lm);
      q[NR + (l - 1) * NA + n] = fmaf(kW[lm], s[n * NC + lm] * s[n * NC + lm], q[NR + (l - 1) * NA + n]);
    }
  if constexpr (S::FB) {
#pragma unroll
    for (int n = 0; n < NA; ++n) {
      const Sym3 a = s_matrix(s + n * NC);
      const float det = a.xx * (a.yy * a.zz - a.yz * a.yz) - a.xy * (a.xy * a.zz - a.yz * a.xz) +
                        a.xz * (a.xy * a.yz - a.yy * a.xz);
      q[NR + S::L3 * NA + n] = 3.f * det;
    }
  }
}

// 3 Q contracted with dS/ds for the l = 2 accumulators (xy, yz, 3z^2 - r^2, xz,
// x^2 - y^2) of one channel, for a symmetric 3x3 matrix Q.
__device__ __forceinline__ void fourbody_contract(const Sym3& Q, float* d5) {
  d5[0] = 6.f * Q.xy;
  d5[1] = 6.f * Q.yz;
  d5[2] = Q.zz - 0.5f * (Q.xx + Q.yy);
  d5[3] = 6.f * Q.xz;
  d5[4] = 1.5f * (Q.xx - Q.yy);
}

// d tr(S^3) / d s: the contraction above with Q = S^2.
__device__ __forceinline__ void fourbody_ds(const float* sl, float* d5) {
  const Sym3 a = s_matrix(sl);
  Sym3 Q;
  Q.xx = a.xx * a.xx + a.xy * a.xy + a.xz * a.xz;
  Q.yy = a.xy * a.xy + a.yy * a.yy + a.yz * a.yz;
  Q.zz = a.xz * a.xz + a.yz * a.yz + a.zz * a.zz;
  Q.xy = a.xx * a.xy + a.xy * a.yy + a.xz * a.yz;
  Q.yz = a.xy * a.xz + a.yy * a.yz + a.yz * a.zz;
  Q.xz = a.xx * a.xz + a.xy * a.yz + a.xz * a.zz;
  fourbody_contract(Q, d5);
}

// Derivative of fourbody_ds along the accumulator direction sdl (the Hessian of
// tr(S^3) times sdl): S^2 is replaced by S Sd + Sd S.
__device__ __forceinline__ void fourbody_ds_dir(const float* sl, const float* sdl, float* d5) {
  const Sym3 a = s_matrix(sl), b = s_matrix(sdl);
  Sym3 Q;
  Q.xx = 2.f * (a.xx * b.xx + a.xy * b.xy + a.xz * b.xz);
  Q.yy = 2.f * (a.xy * b.xy + a.yy * b.yy + a.yz * b.yz);
  Q.zz = 2.f * (a.xz * b.xz + a.yz * b.yz + a.zz * b.zz);
  Q.xy = a.xx * b.xy + a.xy * b.yy + a.xz * b.yz + b.xx * a.xy + b.xy * a.yy + b.xz * a.yz;
  Q.yz = a.xy * b.xz + a.yy * b.yz + a.yz * b.zz + b.xy * a.xz + b.yy * a.yz + b.yz * a.zz;
  Q.xz = a.xx * b.xz + a.xy * b.yz + a.xz * b.zz + b.xx * a.xz + b.xy * a.yz + b.xz * a.zz;
  fourbody_contract(Q, d5);
}

template <class S>
__host__ __device__ inline bool is_shape(const ModelDev& m) {
  return m.nR == S::NR && m.kR == S::KR && m.nA == S::NA && m.kA == S::KA && m.L3 == S::L3 &&
         (m.L4 == 2) == S::FB && m.H == S::H && m.T >= 1 && m.T <= kMaxTypes;
}

}  // namespace kern
}  // namespace nep
