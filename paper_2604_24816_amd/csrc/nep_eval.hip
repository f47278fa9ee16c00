// NEP energy/force evaluation on gfx950: two kernels per force evaluation.
//
//   k_desc_net  (one thread per center, 256-thread workgroups)
//     1. radial descriptors q_n = sum_j g_n(r_ij) (Section III.B) and angular
//        accumulators s_nlm = sum_j g_n(r_ij) P_lm(u_ij) for every channel n in one
//        pass over the center's list with skin, each visited entry tested against
//        the true cutoffs in FP64 (Algorithm 1's geometry reuse with the channel tile
//        equal to all n_max+1 channels); from them q_nl = sum_m W_lm s_nlm^2 and the
//        four-body invariant tr(S_n^3);
//     2. the network U_i = w1 . tanh(W0 q~ - b0) - b1 and its gradient
//        dU/dq~ = W0^T (w1 (1 - tanh^2)) as two 64-row MFMA products per
//        wavefront (Section V.B Optimization 1, Fig. 2c), operands staged
//        through LDS; FP32 MFMA or bfloat16 MFMA with FP32 accumulation;
//     3. per-atom dU/ds_nlm is written for the force kernel, and the atom's whole
//        neighbour record (its position and radial force coefficients).
//     Neighbour positions are gathered from the 16-byte position array.
//   k_force
//     radial pair forces by gather (F_i += sum_j [dU_i/dr_ij - dU_j/dr_ji]
//     with the neighbour's radial coefficients read from its record), angular and
//     four-body pair forces from dU/ds by scatter into the neighbours (Section V.B
//     Optimization 1: no temporary per-pair force buffer; an LDS copy of the tile's
//     halo, or global atomics where it does not fit), and the virial
//     W_ab = -sum r_a dU_i/dr_b; the tile's energy (the U_i the descriptor kernel
//     wrote) and virial are summed per workgroup in FP64.
//   Pair arithmetic in both comes from nep_fast.h.
#include "nep_fast.h"

namespace nep {
namespace {

using namespace kern;

// ------------------------------------------------------------------------ network
// Row stride of the per-wavefront operand tile: 37 words keep a lane's own row (stride
// odd) and the MFMA operand and result patterns (lane (lr, lk) at 37 lr + lk and
// 148 lk + lr) within two passes of the 64 LDS banks.
constexpr int kNetStride = 37;

// The network's operand tiles are private to a wavefront, so its lanes only have to see
// each other's LDS writes (wave_lds_sync), not a workgroup barrier: the wavefronts of a
// workgroup leave their descriptor loops independently.

// One wavefront evaluates the network for its 64 centers. qs[lane][v] holds the
// scaled descriptor of the lane's center on entry; on exit fp[v] = dU/dq~ and the
// return value is U. lds: this wavefront's 64 x kNetStride float tile.
template <class S, int PREC>
__device__ __forceinline__ float network_wave(const ModelDev& m, const float* qs, float* fp, float* lds,
                                              const float* __restrict__ W0, const float* __restrict__ b0,
                                              const float* __restrict__ w1, float b1) {
  const int lane = threadIdx.x & 63;
  const int lr = lane & 15;   // row / column within a 16-wide tile
  const int lk = lane >> 4;   // k group
  float* row = lds + lane * kNetStride;
#pragma unroll
  for (int v = 0; v < 32; ++v) row[v] = v < S::D ? qs[v] : 0.f;
  wave_lds_sync();
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
        const float aop = lds[(16 * R + lr) * kNetStride + dcol];
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
        aop[e] = bits_to_bf16(f32_to_bf16_bits(lds[(16 * R + lr) * kNetStride + 8 * lk + e]));
#pragma unroll
      for (int C = 0; C < 2; ++C)
        acc[R][C] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, bop[C], acc[R][C], 0, 0, 0);
    }
  }
  wave_lds_sync();
  // D layout: lane holds rows 4*lk + r of column lr.
#pragma unroll
  for (int R = 0; R < 4; ++R)
#pragma unroll
    for (int C = 0; C < 2; ++C)
#pragma unroll
      for (int r = 0; r < 4; ++r) lds[(16 * R + 4 * lk + r) * kNetStride + 16 * C + lr] = acc[R][C][r];
  wave_lds_sync();
  float U = -b1;
  float a1[32];
#pragma unroll
  for (int mu = 0; mu < 32; ++mu) {
    if (mu < S::H) {
      const float t = tanh_fast(row[mu] - b0[mu]);
      U = fmaf(w1[mu], t, U);
      a1[mu] = w1[mu] * (1.f - t * t);
    } else {
      a1[mu] = 0.f;
    }
  }
  wave_lds_sync();
#pragma unroll
  for (int mu = 0; mu < 32; ++mu) row[mu] = a1[mu];
  wave_lds_sync();
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
        const float aop = lds[(16 * R + lr) * kNetStride + hid];
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
        aop[e] = bits_to_bf16(f32_to_bf16_bits(lds[(16 * R + lr) * kNetStride + 8 * lk + e]));
#pragma unroll
      for (int C = 0; C < 2; ++C)
        acc[R][C] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop, bop[C], acc[R][C], 0, 0, 0);
    }
  }
  wave_lds_sync();
#pragma unroll
  for (int R = 0; R < 4; ++R)
#pragma unroll
    for (int C = 0; C < 2; ++C)
#pragma unroll
      for (int r = 0; r < 4; ++r) lds[(16 * R + 4 * lk + r) * kNetStride + 16 * C + lr] = acc[R][C][r];
  wave_lds_sync();
#pragma unroll
  for (int v = 0; v < S::D; ++v) fp[v] = row[v];
  return U;
}

// ------------------------------------------------------------------------ descriptors
// The main loops only count the pairs inside the ZBL radius; a center with any visits its
// whole radial list again afterwards (zbl_center), which keeps the loops free of slot
// bookkeeping for the common case of no close pairs.
using EvalZbl = ZblSeen<0>;

// Radial descriptors q[0..NR) and angular accumulators s[NA][NC] of center i over the
// pairs inside the true cutoffs, all channels in one pass over the list with skin
// (geometry computed once per pair and reused for every n). One species: the radial
// descriptors are linear in the basis sums, q_n = sum_k c_nk sum_j f_k(r_ij), with
// sum_j f_k = (sum_j f_c T_k + sum_j f_c) / 2, so a pair adds f_c and f_c T_k (k >= 1).
// Returns the pair counts and the pairs inside the ZBL radius (zs).
template <class S, bool MULTI>
__device__ __forceinline__ void desc_pass(const ModelDev& m, const EvalBuffers& b, int64_t i, int ti, QPos qi,
                                          float* q, float* s, EvalZbl& zs, int& nr, int& na) {
  constexpr int NR = S::NR, NA = S::NA, NC = S::NC, KR = S::KR, KA = S::KA;
  const int64_t N = b.N;
  const float rcR_inv = 1.f / m.rcR, rcA_inv = 1.f / m.rcA;
  const CutConst cutR = cut_const(m.rcR), cutA = cut_const(m.rcA);
  const float rcR2 = (float)(m.rcR64 * m.rcR64), rcA2 = (float)(m.rcA64 * m.rcA64), zbl2 = (float)m.zbl_o2;
  const bool zbl_on = m.zbl_o2 > 0.0;
  const double hx = box_quantum(b.box[0]), hy = box_quantum(b.box[1]), hz = box_quantum(b.box[2]);
  nr = 0;
  na = 0;
  const int kR = radial_bound(b, i), kA = angular_bound(b, i);
  float Qf = 0.f, QT[KR];  // sum_j f_c and sum_j f_c T_k (one species)
#pragma unroll
  for (int k = 0; k < KR; ++k) QT[k] = 0.f;
  // the radial term of a pair inside rc_radial
  auto radial_term = [&](int p, int32_t j, float r2, float r) {
    ++nr;
    zs.n += (zbl_on && r2 < zbl2) ? 1 : 0;
    if constexpr (MULTI) {
      float g[NR];
      radial_g<NR, KR>(r, rcR_inv, m.cR + (ti * m.T + b.type[j]) * NR * KR, g);
#pragma unroll
      for (int n = 0; n < NR; ++n) q[n] += g[n];
    } else {
      // T_k by the recurrence T_{k+1} = 2x T_k - T_{k-1}
      const RadialGeo ra = radial_geo<false>(r, cutR);
      Qf += ra.fc;
      const float x2 = ra.x + ra.x;
      float Tm = 1.f, T = ra.x;
#pragma unroll
      for (int k = 1; k < KR; ++k) {
        QT[k] = fmaf(ra.fc, T, QT[k]);
        const float Tn = fmaf(x2, T, -Tm);
        Tm = T;
        T = Tn;
      }
    }
  };
  // one entry: the radial term, and for the angular candidates inside rc_angular the angular one
  auto pair_both = [&](int p, int32_t j, const uint4* w) {
    float dx, dy, dz;
    const float r2 = pair_vec_q(w[0], qi, hx, hy, hz, dx, dy, dz);
    if (!(r2 < rcR2)) return;
    float r, rinv;
    r_of_r2(r2, r, rinv);
    radial_term(p, j, r2, r);
    if (p < kA && r2 < rcA2) {
      ++na;
      float g[NA];
      if constexpr (MULTI) {
        radial_g<NA, KA>(r, rcA_inv, m.cA + (ti * m.T + b.type[j]) * NA * KA, g);
      } else {
        const RadialGeo ra = radial_geo<false>(r, cutA);
        radial_g_fast<NA, KA>(ra.fc, ra.x, uniform_coeffs(m.hA), g);
      }
      for_each_poly<NC>(dx * rinv, dy * rinv, dz * rinv, [&](int lm, float P) {
#pragma unroll
        for (int n = 0; n < NA; ++n) s[n * NC + lm] = fmaf(g[n], P, s[n * NC + lm]);
      });
    }
  };
  // the angular candidates are the list's prefix [0, kA)
  if constexpr (MULTI)
    for_each_rec_span<1, S::DESC_AHEAD, 1>(b.nbr, b.pos, N, i, 0, kR, pair_both);
  else
    for_each_rec_fast<1, S::DESC_AHEAD, 1>(b.nbr, b.pos, N, i, 0, kR, pair_both);
  if constexpr (!MULTI) {
    const cfloat_ptr c = uniform_coeffs(m.cR);
    float Qb[KR];
    Qb[0] = Qf;
#pragma unroll
    for (int k = 1; k < KR; ++k) Qb[k] = 0.5f * (QT[k] + Qf);
#pragma unroll
    for (int n = 0; n < NR; ++n) {
      float a = 0.f;
#pragma unroll
      for (int k = 0; k < KR; ++k) a = fmaf(c[n * KR + k], Qb[k], a);
      q[n] += a;
    }
  }
}

// dU/ds of one atom as a row (the deterministic form's layout): NA * NC values padded
// to a multiple of four, so that a row is read with 16-byte loads.
template <class S>
constexpr int g_row() {
  static_assert(((S::NA * S::NC + 3) & ~3) <= 5 * 24, "a row must fit the system's dU/ds buffer");
  return (S::NA * S::NC + 3) & ~3;
}
template <class S>
__device__ __forceinline__ void load_g_row(const float* row, float* g) {
  const float4* r4 = reinterpret_cast<const float4*>(row);
#pragma unroll
  for (int k = 0; k < g_row<S>() / 4; ++k) {
    const float4 v = r4[k];
    g[4 * k] = v.x;
    if (4 * k + 1 < S::NA * S::NC) g[4 * k + 1] = v.y;
    if (4 * k + 2 < S::NA * S::NC) g[4 * k + 2] = v.z;
    if (4 * k + 3 < S::NA * S::NC) g[4 * k + 3] = v.w;
  }
}

// ------------------------------------------------------------------------ descriptor + network
template <class S, int PREC, bool MULTI>
__global__ void __launch_bounds__(kBlock, 2) k_desc_net(ModelDev m, EvalBuffers b) {
  __shared__ float lds[kBlock / 64][64 * kNetStride];
  constexpr int NR = S::NR, NA = S::NA, NC = S::NC, D = S::D;
  const int64_t N = b.N;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t i = (int64_t)tile * kBlock + threadIdx.x;
  const bool valid = i < N;

  float q[D];
#pragma unroll
  for (int v = 0; v < D; ++v) q[v] = 0.f;
  float s[NA * NC];
#pragma unroll
  for (int k = 0; k < NA * NC; ++k) s[k] = 0.f;
  const int ti = valid ? (MULTI ? b.type[i] : 0) : 0;
  EvalZbl zs;  // pairs inside the ZBL radius

  if (valid) {
    const uint4 w0 = b.pos[i];
    int nr = 0, na = 0;
    desc_pass<S, MULTI>(m, b, i, ti, QPos{w0.x, w0.y, w0.z}, q, s, zs, nr, na);
    b.nactR[i] = nr;
    b.nactA[i] = na;
    desc_finish<S>(s, q);
  }
  // 3. network (whole wavefronts take part; inactive lanes carry zeros)
  float qs[D], fp[D];
#pragma unroll
  for (int v = 0; v < D; ++v) qs[v] = q[v] * m.sigma[v];
  float U = network_wave<S, PREC>(m, qs, fp, lds[threadIdx.x >> 6], m.W0, m.b0, m.w1, m.b1[0]);
#pragma unroll
  for (int v = 0; v < D; ++v) fp[v] *= m.sigma[v];  // dU/dq = sigma * dU/dq~

  if (valid) {
    {
      // neighbour record words 0.w, 1, 2: for one species v = w_0 + sum_k w_k and w_1..w_8 with
      // w_k = sum_n (dU/dq_n) c_nk (the radial force of a pair is then a Chebyshev series in
      // w_i + w_j), dU/dq_0..dU/dq_4 for several species
      static_assert(S::KR == 9 && S::NR <= 5, "the record holds nine radial coefficients");
      float t[9];
      if constexpr (MULTI) {
#pragma unroll
        for (int k = 0; k < 9; ++k) t[k] = k < NR ? fp[k] : 0.f;
      } else {
        const cfloat_ptr c = uniform_coeffs(m.cR);
        float sum = 0.f;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          float a = 0.f;
#pragma unroll
          for (int n = 0; n < NR; ++n) a = fmaf(fp[n], c[n * S::KR + k], a);
          t[k] = a;
          sum += a;
        }
        t[0] += sum;
      }
      // the whole 64-byte record: position, the nine coefficients, a zero word
      const uint4 own = b.pos[i];
      uint4* r = b.rec + 4 * i;
      r[0] = make_uint4(own.x, own.y, own.z, __float_as_uint(t[0]));
      reinterpret_cast<float4*>(r + 1)[0] = make_float4(t[1], t[2], t[3], t[4]);
      reinterpret_cast<float4*>(r + 2)[0] = make_float4(t[5], t[6], t[7], t[8]);
      r[3] = make_uint4(0u, 0u, 0u, 0u);
    }
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
        float d5[5];
        fourbody_ds(s + n * NC, d5);
        const float f4 = fp[NR + S::L3 * NA + n];
#pragma unroll
        for (int k = 0; k < 5; ++k) Gd[n * NC + 3 + k] = fmaf(f4, d5[k], Gd[n * NC + 3 + k]);
      }
    }
    if (b.deterministic) {
      // atom-major rows for the force kernel's gathers of the neighbours' dU/ds
      float4* g4 = reinterpret_cast<float4*>(b.G + i * g_row<S>());
#pragma unroll
      for (int k = 0; k < g_row<S>() / 4; ++k)
        g4[k] = make_float4(Gd[4 * k], 4 * k + 1 < NA * NC ? Gd[4 * k + 1] : 0.f,
                            4 * k + 2 < NA * NC ? Gd[4 * k + 2] : 0.f, 4 * k + 3 < NA * NC ? Gd[4 * k + 3] : 0.f);
    } else {
#pragma unroll
      for (int k = 0; k < NA * NC; ++k) b.G[(int64_t)k * N + i] = Gd[k];
    }
    b.F[i] = 0.f;
    b.F[N + i] = 0.f;
    b.F[2 * N + i] = 0.f;
    // ZBL energy (half of each close pair), after the descriptors are no longer live
    if (zs.n) zbl_center<MULTI>(m, b, i, ti, b.x[i], b.x[N + i], b.x[2 * N + i], zs, &U, nullptr, nullptr);
    b.U[i] = U;
  }
}

// ------------------------------------------------------------------------ force halo in LDS
// The angular force kernel scatters -dU_i/dr_ij into every neighbour j. A workgroup's
// 256 cell-sorted atoms only reach atoms of the cells next to theirs (the tile's halo,
// tabulated at list build), so the scatter goes into an LDS copy of the halo's forces
// and one coalesced global atomic per halo atom and component flushes it at the end
// (scattered global atomics resolve at the memory side one cache line each).
struct HaloLds {
  float F[3][kHaloMax];
  int start[kHaloCellsMax];
  int off[kHaloCellsMax + 1];
  int ncells, natoms, ok;
};

// Loads the tile's halo table and clears the LDS forces; returns whether the tile
// uses the LDS halo (uniform over the workgroup).
__device__ bool load_halo(const EvalBuffers& b, int tile, HaloLds& h) {
  if (threadIdx.x == 0) {
    h.ncells = b.hinfo[4 * tile + 0];
    h.natoms = b.hinfo[4 * tile + 1];
    h.ok = b.hinfo[4 * tile + 2];
  }
  __syncthreads();
  if (!h.ok) return false;
  const int nc = h.ncells, na = h.natoms;
  for (int k = threadIdx.x; k < nc; k += kBlock) h.start[k] = b.hstart[(int64_t)tile * kHaloCellsMax + k];
  for (int k = threadIdx.x; k <= nc; k += kBlock) h.off[k] = b.hoff[(int64_t)tile * (kHaloCellsMax + 1) + k];
  for (int t = threadIdx.x; t < na; t += kBlock) {
    h.F[0][t] = 0.f;
    h.F[1][t] = 0.f;
    h.F[2][t] = 0.f;
  }
  __syncthreads();
  return true;
}

// Adds the halo forces to F with one global atomic per halo atom and component that
// received a force: 16 lanes to a halo cell, whose atoms are contiguous both in the halo
// and in F.
__device__ void flush_halo(const HaloLds& h, float* __restrict__ F, int64_t N) {
  const int q = threadIdx.x >> 4, u = threadIdx.x & 15;
  for (int c = q; c < h.ncells; c += kBlock / 16) {
    const int o = h.off[c], n = h.off[c + 1] - o;
    const int64_t g0 = h.start[c];
    for (int t = u; t < n; t += 16) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float v = h.F[k][o + t];
        if (v != 0.f) unsafeAtomicAdd(&F[k * N + g0 + t], v);
      }
    }
  }
}

// ------------------------------------------------------------------------ forces
// Waves per SIMD the force kernel is compiled for: the l <= 2 shapes fit three in
// registers and in LDS (the halo takes a third of a CU's LDS); four would spill.
template <class S>
constexpr int force_waves() { return S::L3 <= 2 ? 3 : 2; }

// Constants of the angular pair force (uniform over a launch).
struct AngConst {
  float rcA_inv;
  CutConst cutA;
  float kDA;  // f_c' = kDA c (angular cutoff)
  float kYA;  // x' = kYA y
};
__device__ __forceinline__ AngConst ang_const(const ModelDev& m) {
  AngConst a;
  a.rcA_inv = 1.f / m.rcA;
  a.cutA = cut_const(m.rcA);
  a.kDA = -0.5f * kPiF * a.cutA.rc_inv;
  a.kYA = 4.f * a.cutA.rc_inv;
  return a;
}

// Angular and four-body force of center c on a neighbour k inside rc_angular, n = -dU_c/dr_ck,
// for the unit vector u from c to k at distance r, from the center's dU/ds (Gc(q) returns
// component q < NA * NC, channel-major) and the pair's types (center tc, neighbour tk):
// F_ck = sum_lm [ A_lm P_lm u + B_lm (grad P_lm - l P_lm u) / r ] with A_lm = sum_n G_nlm g'_n
// and B_lm = sum_n G_nlm g_n; the l P B terms are summed per l and scaled once.
template <class S, bool MULTI, class GF>
__device__ __forceinline__ void angular_pair_force(const ModelDev& m, const AngConst& ac, GF&& Gc, int tc, int tk,
                                                   float ux, float uy, float uz, float r, float rinv, float& n0,
                                                   float& n1, float& n2) {
  constexpr int NA = S::NA, NC = S::NC, KA = S::KA;
  float sc, vx = 0.f, vy = 0.f, vz = 0.f, vscale;
  if constexpr (MULTI) {
    float g[NA], dg[NA];
    radial_g_dg<NA, KA>(r, ac.rcA_inv, m.cA + (tc * m.T + tk) * NA * KA, g, dg);
    float sA = 0.f;
    float sB[4] = {0.f, 0.f, 0.f, 0.f};
    for_each_poly_grad<NC>(ux, uy, uz, [&](int lm, float P, auto px, auto py, auto pz) {
      float A = Gc(lm) * dg[0], B = Gc(lm) * g[0];
#pragma unroll
      for (int n = 1; n < NA; ++n) {
        A = fmaf(Gc(n * NC + lm), dg[n], A);
        B = fmaf(Gc(n * NC + lm), g[n], B);
      }
      sA = fmaf(P, A, sA);
      sB[comp_l(lm) - 1] = fmaf(P, B, sB[comp_l(lm) - 1]);
      vx = fmac(B, px, vx);
      vy = fmac(B, py, vy);
      vz = fmac(B, pz, vz);
    });
    const float lPB = fmaf(4.f, sB[3], fmaf(3.f, sB[2], fmaf(2.f, sB[1], sB[0])));
    sc = fmaf(-rinv, lPB, sA);
    vscale = rinv;
  } else {
    // With g_n = f_c C_n and g'_n = f_c' C_n + f_c x' D_n: B_lm = f_c E_lm and
    // A_lm = f_c' E_lm + f_c x' H_lm for E_lm = sum_n G_nlm C_n, H_lm = sum_n G_nlm D_n,
    // so f_c, f_c' and f_c x' are applied once to the sums over lm.
    const RadialGeo rb = radial_geo<true>(r, ac.cutA);
    float Cn[NA], Dn[NA];
    radial_cd_fast<NA, KA>(rb.x, uniform_coeffs(m.hA), Cn, Dn);
    float sH = 0.f;
    float sE[4] = {0.f, 0.f, 0.f, 0.f};
    for_each_poly_grad<NC>(ux, uy, uz, [&](int lm, float P, auto px, auto py, auto pz) {
      float E = Gc(lm) * Cn[0], H = Gc(lm) * Dn[0];
#pragma unroll
      for (int n = 1; n < NA; ++n) {
        E = fmaf(Gc(n * NC + lm), Cn[n], E);
        H = fmaf(Gc(n * NC + lm), Dn[n], H);
      }
      sH = fmaf(P, H, sH);
      sE[comp_l(lm) - 1] = fmaf(P, E, sE[comp_l(lm) - 1]);
      vx = fmac(E, px, vx);
      vy = fmac(E, py, vy);
      vz = fmac(E, pz, vz);
    });
    const float sPE = (sE[0] + sE[1]) + (sE[2] + sE[3]);
    const float lPE = fmaf(4.f, sE[3], fmaf(3.f, sE[2], fmaf(2.f, sE[1], sE[0])));
    const float sA = fmaf(ac.kDA * rb.c, sPE, (rb.fc * (ac.kYA * rb.y)) * sH);
    vscale = rb.fc * rinv;
    sc = fmaf(-vscale, lPE, sA);
  }
  // n = -dU_c/dr_ck (sign folded into the operands)
  n0 = fmaf(-ux, sc, -(vx * vscale));
  n1 = fmaf(-uy, sc, -(vy * vscale));
  n2 = fmaf(-uz, sc, -(vz * vscale));
}

// DET: the deterministic form. Nothing is scattered: each atom adds, after its own pair
// terms, the angular forces of the centers that have it as an angular neighbour, each
// recomputed from that center's dU/ds (atom-major rows) in list order, and stores its
// force. The sets agree: a pair inside rc_angular lies in both atoms' angular prefixes,
// and the box-fraction pair vector of (j, i) is the exact negation of that of (i, j), so
// both sides see the same r^2. The terms are bitwise those the scattering form adds, in
// a fixed order.
template <class S, bool MULTI, bool DET>
__global__ void __launch_bounds__(kBlock, force_waves<S>()) k_force(ModelDev m, EvalBuffers b) {
  __shared__ double red[4 * 10];
  __shared__ HaloLds halo;
  constexpr int NR = S::NR, NA = S::NA, NC = S::NC;
  const int64_t N = b.N;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int64_t i = (int64_t)tile * kBlock + threadIdx.x;
  const bool valid = i < N;
  bool lds = false;
  if constexpr (!DET) lds = load_halo(b, tile, halo);
  const double hx = box_quantum(b.box[0]), hy = box_quantum(b.box[1]), hz = box_quantum(b.box[2]);
  const float rcR_inv = 1.f / m.rcR;
  const CutConst cutR = cut_const(m.rcR);
  const float kXR = -0.25f * kPiF * cutR.rc_inv;  // X = kXR Z for the radial series (one species)
  const AngConst ac = ang_const(m);
  const bool zbl_on = m.zbl_o2 > 0.0;
  float fx = 0.f, fy = 0.f, fz = 0.f;
  float w[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) w[k] = 0.f;
  if (valid) {
    const uint4* ri = b.rec + 4 * i;
    const uint4 r0 = ri[0], r1 = ri[1], r2w = ri[2];
    const QPos qi{r0.x, r0.y, r0.z};
    const int ti = MULTI ? b.type[i] : 0;
    // own radial coefficients (v = w_0 + sum_k w_k and w_1..w_8 for one species, dU/dq_n for
    // several)
    const float wi[9] = {__uint_as_float(r0.w),  __uint_as_float(r1.x),  __uint_as_float(r1.y),
                         __uint_as_float(r1.z),  __uint_as_float(r1.w),  __uint_as_float(r2w.x),
                         __uint_as_float(r2w.y), __uint_as_float(r2w.z), __uint_as_float(r2w.w)};
    constexpr int KR = S::KR;
    float G[NA * NC];
    if constexpr (DET) {
      load_g_row<S>(b.G + i * g_row<S>(), G);
    } else {
#pragma unroll
      for (int k = 0; k < NA * NC; ++k) G[k] = b.G[(int64_t)k * N + i];
    }
    const float rcR2 = (float)(m.rcR64 * m.rcR64), rcA2 = (float)(m.rcA64 * m.rcA64), zbl2 = (float)m.zbl_o2;
    const int kR = radial_bound(b, i), kA = angular_bound(b, i);
    EvalZbl zs;  // pairs inside the ZBL radius
    // One entry: the radial term by gather, F_i += (dU_i/dr_ij + dU_j/dr_ji) along u, with
    // the neighbour's radial coefficients read from its record, the virial taking half of
    // that pair term (the lists are symmetric, so the pair's other half comes from j); and
    // for the angular candidates (the list prefix [0, kA)) inside rc_angular the angular
    // and four-body term dU_i/dr_ij, added to this atom and scattered, negated, into the
    // neighbour.
    auto pair_both = [&](int p, int32_t j, const uint4* rw) {
      float dx, dy, dz;
      const float r2 = pair_vec_q(rw[0], qi, hx, hy, hz, dx, dy, dz);
      if (!(r2 < rcR2)) return;
      const bool ang = p < kA && r2 < rcA2;
      const int lj = (!DET && ang && lds) ? (int)b.nbrl[(int64_t)p * N + i] : 0;
      float r, rinv;
      r_of_r2(r2, r, rinv);
      const int tj = MULTI ? b.type[j] : 0;
      const float wj[9] = {__uint_as_float(rw[0].w), __uint_as_float(rw[1].x), __uint_as_float(rw[1].y),
                           __uint_as_float(rw[1].z), __uint_as_float(rw[1].w), __uint_as_float(rw[2].x),
                           __uint_as_float(rw[2].y), __uint_as_float(rw[2].z), __uint_as_float(rw[2].w)};
      float sr;  // (dU_i/dr_ij + dU_j/dr_ji) / r: the pair force is sr (x_j - x_i)
      if constexpr (MULTI) {
        float g[NR], dg[NR], g2[NR], dg2[NR];
        radial_g_dg<NR, KR>(r, rcR_inv, m.cR + (ti * m.T + tj) * NR * KR, g, dg);
        radial_g_dg<NR, KR>(r, rcR_inv, m.cR + (tj * m.T + ti) * NR * KR, g2, dg2);
        float si = 0.f, sj = 0.f;
#pragma unroll
        for (int n = 0; n < NR; ++n) {
          si = fmaf(wi[n], dg[n], si);
          sj = fmaf(wj[n], dg2[n], sj);
        }
        sr = (si + sj) * rinv;
      } else {
        // one species: sum_k (w_ik + w_jk) f_k'(r)
        const RadialGeo ra = radial_geo<true>(r, cutR);
        float W[KR];
#pragma unroll
        for (int k = 1; k < KR; ++k) W[k] = wi[k] + wj[k];
        sr = radial_series_z<KR>(ra, W, wi[0] + wj[0]) * (kXR * rinv);
      }
      zs.n += (zbl_on && r2 < zbl2) ? 1 : 0;
      fx = fmaf(sr, dx, fx);
      fy = fmaf(sr, dy, fy);
      fz = fmaf(sr, dz, fz);
      {
        // W_ac -= d_a (sr d_c) / 2
        const float vs = -0.5f * sr;
        const float d[3] = {dx, dy, dz};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const float vd = vs * d[a];
#pragma unroll
          for (int c = 0; c < 3; ++c) w[a * 3 + c] = fmaf(vd, d[c], w[a * 3 + c]);
        }
      }
      if (!ang) return;
      const float ux = dx * rinv, uy = dy * rinv, uz = dz * rinv;
      float n0, n1, n2;  // -dU_i/dr_ij, the force on the neighbour
      angular_pair_force<S, MULTI>(m, ac, [&](int q) { return G[q]; }, ti, tj, ux, uy, uz, r, rinv, n0, n1, n2);
      fx -= n0;
      fy -= n1;
      fz -= n2;
      if constexpr (!DET) {
        if (lds) {
          atomicAdd(&halo.F[0][lj], n0);
          atomicAdd(&halo.F[1][lj], n1);
          atomicAdd(&halo.F[2][lj], n2);
        } else {
          unsafeAtomicAdd(&b.F[j], n0);
          unsafeAtomicAdd(&b.F[N + j], n1);
          unsafeAtomicAdd(&b.F[2 * N + j], n2);
        }
      }
      const float d[3] = {dx, dy, dz};
      const float nf[3] = {n0, n1, n2};
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) w[a * 3 + c] = fmaf(d[a], nf[c], w[a * 3 + c]);
    };
    if constexpr (MULTI)
      for_each_rec_span<3, 1, 4>(b.nbr, b.rec, N, i, 0, kR, pair_both);
    else
      for_each_rec_fast<3, 1, 4>(b.nbr, b.rec, N, i, 0, kR, pair_both);
    if (zs.n) {
      float f[3] = {fx, fy, fz};
      zbl_center<MULTI>(m, b, i, ti, b.x[i], b.x[N + i], b.x[2 * N + i], zs, nullptr, f, w);
      fx = f[0];
      fy = f[1];
      fz = f[2];
    }
    if constexpr (DET) {
      // the neighbours' angular terms on this atom, in list order
      const uint64_t n64 = (uint64_t)N;
      for (int p = 0; p < kA; ++p) {
        const int32_t j = b.nbr[(uint64_t)(uint32_t)p * n64 + i];
        float dx, dy, dz;
        const float r2 = pair_vec_q(b.pos[j], qi, hx, hy, hz, dx, dy, dz);
        if (!(r2 < rcR2 && r2 < rcA2)) continue;
        float r, rinv;
        r_of_r2(r2, r, rinv);
        const int tj = MULTI ? b.type[j] : 0;
        float Gj[NA * NC];
        load_g_row<S>(b.G + (int64_t)j * g_row<S>(), Gj);
        float n0, n1, n2;  // -dU_j/dr_ji, the force of center j's angular term on this atom
        angular_pair_force<S, MULTI>(m, ac, [&](int q) { return Gj[q]; }, tj, ti, -(dx * rinv), -(dy * rinv),
                                     -(dz * rinv), r, rinv, n0, n1, n2);
        fx += n0;
        fy += n1;
        fz += n2;
      }
      b.F[i] = fx;
      b.F[N + i] = fy;
      b.F[2 * N + i] = fz;
    } else if (lds) {
      const int li = b.selfl[i];
      atomicAdd(&halo.F[0][li], fx);
      atomicAdd(&halo.F[1][li], fy);
      atomicAdd(&halo.F[2][li], fz);
    } else {
      unsafeAtomicAdd(&b.F[i], fx);
      unsafeAtomicAdd(&b.F[N + i], fy);
      unsafeAtomicAdd(&b.F[2 * N + i], fz);
    }
  }
  if constexpr (!DET) {
    if (lds) {
      __syncthreads();
      flush_halo(halo, b.F, N);
    }
  }
  // the tile's energy (the descriptor kernel's U_i, ZBL included) and virial in FP64
  double wd[10], ws[10];
  wd[0] = valid ? (double)b.U[i] : 0.0;
#pragma unroll
  for (int k = 0; k < 9; ++k) wd[1 + k] = (double)w[k];
  block_sum_n<10>(wd, ws, red);
  if (threadIdx.x == 0) {
    b.partial[(int64_t)tile * kPartialStride + P_ENERGY] = ws[0];
#pragma unroll
    for (int k = 0; k < 9; ++k) b.partial[(int64_t)tile * kPartialStride + P_VIR + k] = ws[1 + k];
  }
}

template <class S, int PREC, bool MULTI>
hipError_t launch_pair(const ModelDev& m, const EvalBuffers& b, hipStream_t st, hipEvent_t* ev) {
  const int nb = grid_blocks(b.N);
  if (ev) (void)hipEventRecord(ev[0], st);
  hipLaunchKernelGGL((k_desc_net<S, PREC, MULTI>), dim3(nb), dim3(kBlock), 0, st, m, b);
  if (ev) (void)hipEventRecord(ev[1], st);
  if (b.deterministic)
    hipLaunchKernelGGL((k_force<S, MULTI, true>), dim3(nb), dim3(kBlock), 0, st, m, b);
  else
    hipLaunchKernelGGL((k_force<S, MULTI, false>), dim3(nb), dim3(kBlock), 0, st, m, b);
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


// Derived radial tables (nep_fast.h) of nblk coefficient blocks [nblk][N][K]: one thread
// per (block, channel) writes h_n0 = (c_n0 + sum_k c_nk) / 2, h_nk = c_nk / 2 and
// d_n(k-1) = k c_nk / 2 into that block's [N][2K - 1] table.
__global__ void k_derive_coeffs(const float* __restrict__ c, int nblk, int N, int K, float* __restrict__ h) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nblk * N) return;
  const int blk = t / N, n = t % N;
  const float* cn = c + ((int64_t)blk * N + n) * K;
  float* hb = h + (int64_t)blk * N * (2 * K - 1);
  float sum = 0.f;
  for (int k = 0; k < K; ++k) sum += cn[k];
  hb[n * K] = 0.5f * (cn[0] + sum);
  for (int k = 1; k < K; ++k) {
    hb[n * K + k] = 0.5f * cn[k];
    hb[N * K + n * (K - 1) + k - 1] = (0.5f * (float)k) * cn[k];
  }
}

}  // namespace

int64_t derived_coeff_floats(int T, int nR, int kR, int nA, int kA) {
  return (int64_t)T * T * (nR * (2 * kR - 1) + nA * (2 * kA - 1));
}

hipError_t launch_derive_coeffs(int T, int nR, int kR, int nA, int kA, const float* cR, const float* cA, float* hR,
                                float* hA, hipStream_t st) {
  hipLaunchKernelGGL(k_derive_coeffs, dim3(1), dim3(64), 0, st, cR, T * T, nR, kR, hR);
  hipLaunchKernelGGL(k_derive_coeffs, dim3(1), dim3(64), 0, st, cA, T * T, nA, kA, hA);
  return hipGetLastError();
}

bool eval_supported(const ModelDev& m) { return is_shape<FullShape>(m) || is_shape<SurShape>(m); }

int eval_partial_blocks(int64_t N) { return grid_blocks(N); }

hipError_t launch_eval(const ModelDev& m, int precision, const EvalBuffers& b, hipStream_t st,
                       hipEvent_t* ev) {
  if (is_shape<FullShape>(m)) return launch_shape<FullShape>(m, precision, b, st, ev);
  if (is_shape<SurShape>(m)) return launch_shape<SurShape>(m, precision, b, st, ev);
  return hipErrorInvalidValue;
}

}  // namespace nep
