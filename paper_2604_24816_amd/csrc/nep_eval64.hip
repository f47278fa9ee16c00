// FP64 evaluation of energy, forces and virial (the NEP_FP64 precision).
//
// Every descriptor, network, force and virial operation runs in FP64, from an FP64
// copy of the model parameters, over the same neighbour lists as the FP32 path.
// It exists for checks -- central differences at h = 1e-5 A, agreement with an FP64
// reference to round-off -- not for speed: one thread per center, the angular
// accumulators recomputed one channel at a time, FP64 global atomics for the angular
// reaction forces, no LDS staging and no neighbour records.
//
// Quantities (Section III.B): radial q_n = sum_j g_n(r_ij), angular s_nlm = sum_j
// g_n(r_ij) P_lm(u_ij) with q_nl = sum_m W_lm s_nlm^2, the four-body tr(S_n^3), the
// network U_i and dU_i/dq; forces F_i = sum_j [dU_i/dr_ij + dU_j/dr_ji] (radial, by
// gather) plus the angular pair forces applied to both atoms; W_ab = -sum r_a (dU_i/dr_ij)_b.
#include "nep_kernels.h"

namespace nep {
namespace {

using namespace kern;

constexpr double kPi64 = 3.14159265358979323846;

// f_k(r) = f_c(r) (T_k(x) + 1) / 2 and df_k/dr for k < K, with x = 2 (r/rc - 1)^2 - 1
// and f_c = (1 + cos(pi r / rc)) / 2.
template <int K>
__device__ void basis64(double r, double rc, double* f, double* df) {
  const double rr = r / rc;
  const double fc = 0.5 * (1.0 + cospi(rr));
  const double dfc = -0.5 * kPi64 / rc * sinpi(rr);
  const double y = rr - 1.0;
  const double x = 2.0 * y * y - 1.0;
  const double dx = 4.0 * y / rc;
  double Tm1 = 1.0, T = x, dTm1 = 0.0, dT = 1.0;
  f[0] = fc;
  df[0] = dfc;
  f[1] = 0.5 * (x + 1.0) * fc;
  df[1] = 0.5 * dx * fc + 0.5 * (x + 1.0) * dfc;
#pragma unroll
  for (int k = 2; k < K; ++k) {
    const double Tn = 2.0 * x * T - Tm1;
    const double dTn = 2.0 * T + 2.0 * x * dT - dTm1;
    Tm1 = T;
    T = Tn;
    dTm1 = dT;
    dT = dTn;
    f[k] = 0.5 * (Tn + 1.0) * fc;
    df[k] = 0.5 * dTn * dx * fc + 0.5 * (Tn + 1.0) * dfc;
  }
}

// g_n and g_n' for n < N from coefficients c[n][K].
template <int N, int K>
__device__ void radial64(double r, double rc, const double* c, double* g, double* dg) {
  double f[K], df[K];
  basis64<K>(r, rc, f, df);
#pragma unroll
  for (int n = 0; n < N; ++n) {
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int k = 0; k < K; ++k) {
      a += c[n * K + k] * f[k];
      b += c[n * K + k] * df[k];
    }
    g[n] = a;
    dg[n] = b;
  }
}

struct Pair64 {
  int32_t j;
  double d[3], r;
};

// Visits the pairs of center i inside rcut (FP64 minimum image over the first kmax
// list entries): fn(p, Pair64).
template <class Fn>
__device__ void for_pairs64(const EvalBuffers& b, int64_t i, int kmax, double rcut2, Fn&& fn) {
  const int64_t N = b.N;
  const double xi = b.x[i], yi = b.x[N + i], zi = b.x[2 * N + i];
  for (int p = 0; p < kmax; ++p) {
    Pair64 q;
    q.j = b.nbr[(int64_t)p * N + i];
    q.d[0] = min_image(b.x[q.j] - xi, b.box[0]);
    q.d[1] = min_image(b.x[N + q.j] - yi, b.box[1]);
    q.d[2] = min_image(b.x[2 * N + q.j] - zi, b.box[2]);
    const double r2 = q.d[0] * q.d[0] + q.d[1] * q.d[1] + q.d[2] * q.d[2];
    if (!(r2 < rcut2)) continue;
    q.r = sqrt(r2);
    fn(p, q);
  }
}

// Accumulators s_n[lm] of one angular channel n.
template <class S, bool MULTI>
__device__ void channel64(const Model64& p, const ModelDev& m, const EvalBuffers& b, int64_t i, int ti, int n,
                          double* sn) {
  constexpr int NA = S::NA, NC = S::NC, KA = S::KA;
#pragma unroll
  for (int lm = 0; lm < NC; ++lm) sn[lm] = 0.0;
  for_pairs64(b, i, angular_bound(b, i), m.rcA64 * m.rcA64, [&](int, const Pair64& q) {
    const int tj = MULTI ? b.type[q.j] : 0;
    double g[NA], dg[NA];
    radial64<NA, KA>(q.r, m.rcA64, p.cA + (ti * m.T + tj) * NA * KA, g, dg);
    for_each_poly<NC>(q.d[0] / q.r, q.d[1] / q.r, q.d[2] / q.r, [&](int lm, double P) { sn[lm] += g[n] * P; });
  });
}

// 3 det S = tr(S^3) of one channel's traceless S, and d tr(S^3) / d s for its five
// l = 2 accumulators (xy, yz, 3z^2 - r^2, xz, x^2 - y^2).
__device__ void fourbody64(const double* s2, double& q4, double* d5) {
  const double xy = s2[0], yz = s2[1], zz = s2[2] / 3.0, xz = s2[3];
  const double xx = 0.5 * (s2[4] - zz), yy = 0.5 * (-s2[4] - zz);
  q4 = 3.0 * (xx * (yy * zz - yz * yz) - xy * (xy * zz - yz * xz) + xz * (xy * yz - yy * xz));
  const double Qxx = xx * xx + xy * xy + xz * xz, Qyy = xy * xy + yy * yy + yz * yz;
  const double Qzz = xz * xz + yz * yz + zz * zz;
  const double Qxy = xx * xy + xy * yy + xz * yz, Qyz = xy * xz + yy * yz + yz * zz;
  const double Qxz = xx * xz + xy * yz + xz * zz;
  d5[0] = 6.0 * Qxy;
  d5[1] = 6.0 * Qyz;
  d5[2] = Qzz - 0.5 * (Qxx + Qyy);
  d5[3] = 6.0 * Qxz;
  d5[4] = 1.5 * (Qxx - Qyy);
}

__device__ double block_sum64(double v, double* sh) {
  __syncthreads();
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < (unsigned)off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  return sh[0];
}

// Descriptors, network, U_i (+ ZBL) and dU_i/dq (FP64): U64[i], Fp64[k][i].
template <class S, bool MULTI>
__global__ void __launch_bounds__(kBlock) k_desc64(ModelDev m, Model64 p, EvalBuffers b, double* __restrict__ U64,
                                                   double* __restrict__ Fp64) {
  __shared__ double sh[kBlock];
  constexpr int NR = S::NR, NA = S::NA, NC = S::NC, KR = S::KR, D = S::D, H = S::H;
  const int64_t N = b.N;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double U = 0.0;
  if (i < N) {
    const int ti = MULTI ? b.type[i] : 0;
    double q[D];
#pragma unroll
    for (int k = 0; k < D; ++k) q[k] = 0.0;
    double uz = 0.0;
    for_pairs64(b, i, radial_bound(b, i), m.rcR64 * m.rcR64, [&](int, const Pair64& pr) {
      const int tj = MULTI ? b.type[pr.j] : 0;
      double g[NR], dg[NR];
      radial64<NR, KR>(pr.r, m.rcR64, p.cR + (ti * m.T + tj) * NR * KR, g, dg);
#pragma unroll
      for (int n = 0; n < NR; ++n) q[n] += g[n];
      if (pr.r * pr.r < m.zbl_o2) {
        double e, de;
        zbl_pair<MULTI>(m, ti * m.T + tj, pr.r, e, de);
        uz += 0.5 * e;
      }
    });
    for (int n = 0; n < NA; ++n) {
      double sn[NC];
      channel64<S, MULTI>(p, m, b, i, ti, n, sn);
#pragma unroll
      for (int lm = 0; lm < NC; ++lm) q[NR + (comp_l(lm) - 1) * NA + n] += (double)kW[lm] * sn[lm] * sn[lm];
      if constexpr (S::FB) {
        double q4, d5[5];
        fourbody64(sn + 3, q4, d5);
        q[NR + S::L3 * NA + n] = q4;
      }
    }
    // network
    double a[H];
    U = -p.b1;
#pragma unroll
    for (int mu = 0; mu < H; ++mu) {
      double h = -p.b0[mu];
#pragma unroll
      for (int k = 0; k < D; ++k) h += p.W0[mu * D + k] * (p.sigma[k] * q[k]);
      const double t = tanh(h);
      U += p.w1[mu] * t;
      a[mu] = p.w1[mu] * (1.0 - t * t);
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
      double v = 0.0;
#pragma unroll
      for (int mu = 0; mu < H; ++mu) v += p.W0[mu * D + k] * a[mu];
      Fp64[(int64_t)k * N + i] = p.sigma[k] * v;
    }
    U += uz;
    U64[i] = U;
  }
  const double e = block_sum64(U, sh);
  if (threadIdx.x == 0) b.partial[(int64_t)blockIdx.x * kPartialStride + P_ENERGY] = e;
}

// Forces (F64 [3][N], zeroed before) and virial partials (FP64).
template <class S, bool MULTI>
__global__ void __launch_bounds__(kBlock) k_force64(ModelDev m, Model64 p, EvalBuffers b,
                                                    const double* __restrict__ Fp64, double* __restrict__ F64) {
  __shared__ double sh[kBlock];
  constexpr int NR = S::NR, NA = S::NA, NC = S::NC, KR = S::KR, KA = S::KA;
  const int64_t N = b.N;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double f[3] = {0.0, 0.0, 0.0}, w[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) w[k] = 0.0;
  auto add_pair = [&](const Pair64& q, const double* fij) {  // dU_i/dr_ij on both atoms + virial
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
      for (int c = 0; c < 3; ++c) w[a * 3 + c] -= q.d[a] * fij[c];
    }
  };
  if (i < N) {
    const int ti = MULTI ? b.type[i] : 0;
    // radial (gather): (dU_i/dr + dU_j/dr) along u; ZBL's pair derivative likewise
    for_pairs64(b, i, radial_bound(b, i), m.rcR64 * m.rcR64, [&](int, const Pair64& q) {
      const int tj = MULTI ? b.type[q.j] : 0;
      double g[NR], dgi[NR], dgj[NR];
      radial64<NR, KR>(q.r, m.rcR64, p.cR + (ti * m.T + tj) * NR * KR, g, dgi);
      radial64<NR, KR>(q.r, m.rcR64, p.cR + (tj * m.T + ti) * NR * KR, g, dgj);
      double si = 0.0, sj = 0.0;
#pragma unroll
      for (int n = 0; n < NR; ++n) {
        si += Fp64[(int64_t)n * N + i] * dgi[n];
        sj += Fp64[(int64_t)n * N + q.j] * dgj[n];
      }
      if (q.r * q.r < m.zbl_o2) {
        double e, de;
        zbl_pair<MULTI>(m, ti * m.T + tj, q.r, e, de);
        si += 0.5 * de;
        sj += 0.5 * de;
      }
      double fij[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        f[c] += (si + sj) * q.d[c] / q.r;
        fij[c] = si * q.d[c] / q.r;
      }
      add_pair(q, fij);
    });
    // angular, one channel at a time: dU_i/ds_nlm, then the pair forces of that channel
    for (int n = 0; n < NA; ++n) {
      double sn[NC], G[NC];
      channel64<S, MULTI>(p, m, b, i, ti, n, sn);
#pragma unroll
      for (int lm = 0; lm < NC; ++lm)
        G[lm] = Fp64[(int64_t)(NR + (comp_l(lm) - 1) * NA + n) * N + i] * 2.0 * (double)kW[lm] * sn[lm];
      if constexpr (S::FB) {
        double q4, d5[5];
        fourbody64(sn + 3, q4, d5);
        const double f4 = Fp64[(int64_t)(NR + S::L3 * NA + n) * N + i];
#pragma unroll
        for (int k = 0; k < 5; ++k) G[3 + k] += f4 * d5[k];
      }
      for_pairs64(b, i, angular_bound(b, i), m.rcA64 * m.rcA64, [&](int, const Pair64& q) {
        const int tj = MULTI ? b.type[q.j] : 0;
        double g[NA], dg[NA];
        radial64<NA, KA>(q.r, m.rcA64, p.cA + (ti * m.T + tj) * NA * KA, g, dg);
        const double u[3] = {q.d[0] / q.r, q.d[1] / q.r, q.d[2] / q.r};
        double fij[3] = {0.0, 0.0, 0.0};
        // d(g P_lm)/dr_j = g' P u + g (grad P - l P u) / r
        for_each_poly_grad<NC>(u[0], u[1], u[2], [&](int lm, double P, double px, double py, double pz) {
          const double l = (double)comp_l(lm);
          const double gp[3] = {px, py, pz};
#pragma unroll
          for (int c = 0; c < 3; ++c) fij[c] += G[lm] * (dg[n] * P * u[c] + g[n] * (gp[c] - l * P * u[c]) / q.r);
        });
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          f[c] += fij[c];
          atomicAdd(&F64[(int64_t)c * N + q.j], -fij[c]);
        }
        add_pair(q, fij);
      });
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) atomicAdd(&F64[(int64_t)c * N + i], f[c]);
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    const double t = block_sum64(w[k], sh);
    if (threadIdx.x == 0) b.partial[(int64_t)blockIdx.x * kPartialStride + P_VIR + k] = t;
  }
}

// ------------------------------------------------------------ FP64 parameter gradient
// Gradient of L = gE E + sum_i gF_i . F_i with respect to every packed parameter
// [cR | cA | sigma | W0 | b0 | w1 | b1], all in FP64 (the check form of the FP32
// training kernels). As there, F = -dE/dx turns the force term into
// -sum_i dU_i/dq_i . v_i with v_i = sum_j dq_i/dr_ij . (gF_j - gF_i) the descriptor JVP,
// so each center contributes L_i = gE U_i - Fp_i . v_i (Fp = dU_i/dq). With
// q~ = sigma q, v~ = sigma v, h = W0 q~ - b0, t = tanh h, d = 1 - t^2, z = W0 v~:
//   dL_i/dW0 = alpha q~^T - beta v~^T, alpha = gE w1 d + 2 z w1 t d, beta = w1 d,
//   dL_i/db0 = -alpha, dL_i/dw1 = gE t - z d, dL_i/db1 = -gE,
//   dL_i/dsigma_k = q_k (W0^T alpha)_k - v_k (W0^T beta)_k,
// and the coefficients through rho = dL_i/dq = sigma W0^T alpha and dL_i/dv = -Fp:
//   radial c^{t_i t}_{nk}: sum over neighbours of species t of rho_n f_k - Fp_n f_k' (u.w);
//   angular c^{t_i t}_{nk}: with C_nlm = dL_i/ds_nlm and A_nlm = dL_i/dsd_nlm (sd the
//   JVP of s), sum over neighbours of f_k (X_n + Z_n) + f_k' (u.w) Y_n for
//   X_n = sum_lm C_nlm P_lm, Y_n = sum_lm A_nlm P_lm, Z_n = sum_lm A_nlm (grad P_lm . w - l P_lm (u.w)) / r.
// One thread per center; the angular channels are recomputed one at a time; sums over
// atoms by wavefront shuffles and one FP64 atomic per wavefront and entry.

// Sum of v over the wavefront, added by its first lane to dst.
__device__ __forceinline__ void wave_atomic64(double v, double* dst) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if ((threadIdx.x & 63) == 0) atomicAdd(dst, v);
}

// The same into dst[t_i * stride] for the centers of species t_i (one species: dst).
template <bool MULTI>
__device__ __forceinline__ void wave_atomic64_by_type(double v, int ti, int T, double* dst, int stride) {
  if constexpr (MULTI) {
    for (int t = 0; t < T; ++t) wave_atomic64(ti == t ? v : 0.0, dst + t * stride);
  } else {
    wave_atomic64(v, dst);
  }
}

// w_j - w_i for the force weights w [3][N] (zero without a force term).
__device__ __forceinline__ void weight_diff(const double* w, int64_t N, int64_t i, int32_t j, double* o) {
#pragma unroll
  for (int c = 0; c < 3; ++c) o[c] = w ? w[c * N + j] - w[c * N + i] : 0.0;
}

// Accumulators s_n[lm] of channel n and their JVP sd_n[lm] = sum_j ds_nlm/dr_ij . (w_j - w_i),
// ds/dr . w = g' (u.w) P + g (grad P . w - l P (u.w)) / r.
template <class S, bool MULTI>
__device__ void channel_jvp64(const Model64& p, const ModelDev& m, const EvalBuffers& b, int64_t i, int ti, int n,
                              const double* w, double* sn, double* sdn) {
  constexpr int NA = S::NA, NC = S::NC, KA = S::KA;
#pragma unroll
  for (int lm = 0; lm < NC; ++lm) sn[lm] = sdn[lm] = 0.0;
  for_pairs64(b, i, angular_bound(b, i), m.rcA64 * m.rcA64, [&](int, const Pair64& q) {
    const int tj = MULTI ? b.type[q.j] : 0;
    double g[NA], dg[NA], wd[3];
    radial64<NA, KA>(q.r, m.rcA64, p.cA + (ti * m.T + tj) * NA * KA, g, dg);
    weight_diff(w, b.N, i, q.j, wd);
    const double u[3] = {q.d[0] / q.r, q.d[1] / q.r, q.d[2] / q.r};
    const double uw = u[0] * wd[0] + u[1] * wd[1] + u[2] * wd[2];
    for_each_poly_grad<NC>(u[0], u[1], u[2], [&](int lm, double P, double px, double py, double pz) {
      sn[lm] += g[n] * P;
      sdn[lm] += dg[n] * uw * P + g[n] * (px * wd[0] + py * wd[1] + pz * wd[2] - comp_l(lm) * P * uw) / q.r;
    });
  });
}

// d5 = d tr(S^3)/ds (fourbody64) and its derivative along sd, h5 = (d d5/ds) sd; d5 is
// quadratic in s, so h5 = (d5(s + sd) - d5(s - sd)) / 2 exactly.
__device__ void fourbody_dir64(const double* s2, const double* sd2, double* d5, double* h5) {
  double q4, a[5], b[5], sp[5], sm[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    sp[c] = s2[c] + sd2[c];
    sm[c] = s2[c] - sd2[c];
  }
  fourbody64(s2, q4, d5);
  fourbody64(sp, q4, a);
  fourbody64(sm, q4, b);
#pragma unroll
  for (int c = 0; c < 5; ++c) h5[c] = 0.5 * (a[c] - b[c]);
}

template <class S, bool MULTI>
__global__ void __launch_bounds__(kBlock) k_grad64(ModelDev m, Model64 p, EvalBuffers b, const double* __restrict__ w,
                                                   double gE, double* __restrict__ grad) {
  constexpr int NR = S::NR, NA = S::NA, NC = S::NC, KR = S::KR, KA = S::KA, D = S::D, H = S::H, L3 = S::L3;
  const int64_t N = b.N;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool valid = i < N;
  const int T = MULTI ? m.T : 1;
  const int oA = T * T * NR * KR, oS = oA + T * T * NA * KA, oW = oS + D, oB0 = oW + H * D, oW1 = oB0 + H,
            oB1 = oW1 + H;
  const int ti = (MULTI && valid) ? b.type[i] : 0;
  const double rcR2 = m.rcR64 * m.rcR64;
  // descriptors q and their JVP v
  double q[D], v[D];
#pragma unroll
  for (int k = 0; k < D; ++k) q[k] = v[k] = 0.0;
  if (valid) {
    for_pairs64(b, i, radial_bound(b, i), rcR2, [&](int, const Pair64& pr) {
      const int tj = MULTI ? b.type[pr.j] : 0;
      double g[NR], dg[NR], wd[3];
      radial64<NR, KR>(pr.r, m.rcR64, p.cR + (ti * m.T + tj) * NR * KR, g, dg);
      weight_diff(w, N, i, pr.j, wd);
      const double uw = (pr.d[0] * wd[0] + pr.d[1] * wd[1] + pr.d[2] * wd[2]) / pr.r;
#pragma unroll
      for (int n = 0; n < NR; ++n) {
        q[n] += g[n];
        v[n] += dg[n] * uw;
      }
    });
    for (int n = 0; n < NA; ++n) {
      double sn[NC], sdn[NC];
      channel_jvp64<S, MULTI>(p, m, b, i, ti, n, w, sn, sdn);
#pragma unroll
      for (int lm = 0; lm < NC; ++lm) {
        const int k = NR + (comp_l(lm) - 1) * NA + n;
        q[k] += (double)kW[lm] * sn[lm] * sn[lm];
        v[k] += 2.0 * (double)kW[lm] * sn[lm] * sdn[lm];
      }
      if constexpr (S::FB) {
        double q4, d5[5];
        fourbody64(sn + 3, q4, d5);
        double v4 = 0.0;
#pragma unroll
        for (int c = 0; c < 5; ++c) v4 += d5[c] * sdn[3 + c];
        q[NR + L3 * NA + n] = q4;
        v[NR + L3 * NA + n] = v4;
      }
    }
  }
  // network terms
  double qs[D], vs[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    qs[k] = p.sigma[k] * q[k];
    vs[k] = p.sigma[k] * v[k];
  }
  double al[H], be[H];
  for (int mu = 0; mu < H; ++mu) {
    double h = -p.b0[mu], z = 0.0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
      h += p.W0[mu * D + k] * qs[k];
      z += p.W0[mu * D + k] * vs[k];
    }
    const double t = tanh(h), d = 1.0 - t * t;
    be[mu] = valid ? p.w1[mu] * d : 0.0;
    al[mu] = valid ? gE * p.w1[mu] * d + 2.0 * z * p.w1[mu] * t * d : 0.0;
    wave_atomic64(valid ? gE * t - z * d : 0.0, grad + oW1 + mu);
    wave_atomic64(-al[mu], grad + oB0 + mu);
    for (int k = 0; k < D; ++k) wave_atomic64(al[mu] * qs[k] - be[mu] * vs[k], grad + oW + mu * D + k);
  }
  wave_atomic64(valid ? -gE : 0.0, grad + oB1);
  double rho[D], fp[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    double sa = 0.0, sb = 0.0;
    for (int mu = 0; mu < H; ++mu) {
      sa += p.W0[mu * D + k] * al[mu];
      sb += p.W0[mu * D + k] * be[mu];
    }
    rho[k] = p.sigma[k] * sa;
    fp[k] = p.sigma[k] * sb;
    wave_atomic64(q[k] * sa - v[k] * sb, grad + oS + k);
  }
  // radial coefficients c^{t_i t}
  for (int t = 0; t < T; ++t) {
    double Fk[KR], Ek[KR];
#pragma unroll
    for (int k = 0; k < KR; ++k) Fk[k] = Ek[k] = 0.0;
    if (valid) {
      for_pairs64(b, i, radial_bound(b, i), rcR2, [&](int, const Pair64& pr) {
        if (MULTI && b.type[pr.j] != t) return;
        double f[KR], df[KR], wd[3];
        basis64<KR>(pr.r, m.rcR64, f, df);
        weight_diff(w, N, i, pr.j, wd);
        const double uw = (pr.d[0] * wd[0] + pr.d[1] * wd[1] + pr.d[2] * wd[2]) / pr.r;
#pragma unroll
        for (int k = 0; k < KR; ++k) {
          Fk[k] += f[k];
          Ek[k] += df[k] * uw;
        }
      });
    }
    for (int n = 0; n < NR; ++n)
#pragma unroll
      for (int k = 0; k < KR; ++k)
        wave_atomic64_by_type<MULTI>(rho[n] * Fk[k] - fp[n] * Ek[k], ti, T, grad + (t * NR + n) * KR + k,
                                     T * NR * KR);
  }
  // angular coefficients c^{t_i t}, one channel at a time
  for (int n = 0; n < NA; ++n) {
    double sn[NC], sdn[NC];
    if (valid) {
      channel_jvp64<S, MULTI>(p, m, b, i, ti, n, w, sn, sdn);
    } else {
#pragma unroll
      for (int lm = 0; lm < NC; ++lm) sn[lm] = sdn[lm] = 0.0;
    }
    double C[NC], A[NC];
#pragma unroll
    for (int lm = 0; lm < NC; ++lm) {
      const int k = NR + (comp_l(lm) - 1) * NA + n;
      C[lm] = 2.0 * (double)kW[lm] * (rho[k] * sn[lm] - fp[k] * sdn[lm]);
      A[lm] = -2.0 * (double)kW[lm] * fp[k] * sn[lm];
    }
    if constexpr (S::FB) {
      double d5[5], h5[5];
      fourbody_dir64(sn + 3, sdn + 3, d5, h5);
      const int k4 = NR + L3 * NA + n;
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        C[3 + c] += rho[k4] * d5[c] - fp[k4] * h5[c];
        A[3 + c] -= fp[k4] * d5[c];
      }
    }
    for (int t = 0; t < T; ++t) {
      double acc[KA];
#pragma unroll
      for (int k = 0; k < KA; ++k) acc[k] = 0.0;
      if (valid) {
        for_pairs64(b, i, angular_bound(b, i), m.rcA64 * m.rcA64, [&](int, const Pair64& pr) {
          if (MULTI && b.type[pr.j] != t) return;
          double wd[3], f[KA], df[KA];
          weight_diff(w, N, i, pr.j, wd);
          const double u[3] = {pr.d[0] / pr.r, pr.d[1] / pr.r, pr.d[2] / pr.r};
          const double uw = u[0] * wd[0] + u[1] * wd[1] + u[2] * wd[2];
          double X = 0.0, Y = 0.0, Z = 0.0;
          for_each_poly_grad<NC>(u[0], u[1], u[2], [&](int lm, double P, double px, double py, double pz) {
            X += C[lm] * P;
            Y += A[lm] * P;
            Z += A[lm] * (px * wd[0] + py * wd[1] + pz * wd[2] - comp_l(lm) * P * uw) / pr.r;
          });
          basis64<KA>(pr.r, m.rcA64, f, df);
#pragma unroll
          for (int k = 0; k < KA; ++k) acc[k] += f[k] * (X + Z) + df[k] * uw * Y;
        });
      }
#pragma unroll
      for (int k = 0; k < KA; ++k)
        wave_atomic64_by_type<MULTI>(acc[k], ti, T, grad + oA + (t * NA + n) * KA + k, T * NA * KA);
    }
  }
}

// soa_sorted[c][i] = aos_orig[perm[i]][c]
__global__ void k_gather_vec64(int64_t N, const int32_t* __restrict__ perm, const double* __restrict__ aos_orig,
                               double* __restrict__ soa_sorted) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int64_t o = perm[i];
#pragma unroll
  for (int c = 0; c < 3; ++c) soa_sorted[c * N + i] = aos_orig[3 * o + c];
}

__global__ void k_zero64(int64_t n, double* __restrict__ a) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) a[k] = 0.0;
}

__global__ void k_scalar_out64(int64_t N, const int32_t* __restrict__ perm, const double* __restrict__ u,
                               double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) out[perm[i]] = u[i];
}

template <class S>
hipError_t launch64_shape(const ModelDev& m, const Model64& p, const EvalBuffers& b, double* U64, double* Fp64,
                          double* F64, hipStream_t st) {
  const int nb = grid_blocks(b.N);
  hipLaunchKernelGGL(k_zero64, dim3(grid_blocks(3 * b.N)), dim3(kBlock), 0, st, 3 * b.N, F64);
  if (m.T > 1) {
    hipLaunchKernelGGL((k_desc64<S, true>), dim3(nb), dim3(kBlock), 0, st, m, p, b, U64, Fp64);
    hipLaunchKernelGGL((k_force64<S, true>), dim3(nb), dim3(kBlock), 0, st, m, p, b, Fp64, F64);
  } else {
    hipLaunchKernelGGL((k_desc64<S, false>), dim3(nb), dim3(kBlock), 0, st, m, p, b, U64, Fp64);
    hipLaunchKernelGGL((k_force64<S, false>), dim3(nb), dim3(kBlock), 0, st, m, p, b, Fp64, F64);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_eval64(const ModelDev& m, const Model64& p, const EvalBuffers& b, double* U64, double* Fp64,
                         double* F64, hipStream_t st) {
  if (is_shape<FullShape>(m)) return launch64_shape<FullShape>(m, p, b, U64, Fp64, F64, st);
  if (is_shape<SurShape>(m)) return launch64_shape<SurShape>(m, p, b, U64, Fp64, F64, st);
  return hipErrorInvalidValue;
}

template <class S>
hipError_t grad64_shape(const ModelDev& m, const Model64& p, const EvalBuffers& b, const double* w, double gE,
                        double* grad, int64_t n_params, hipStream_t st) {
  hipLaunchKernelGGL(k_zero64, dim3(grid_blocks(n_params)), dim3(kBlock), 0, st, n_params, grad);
  const int nb = grid_blocks(b.N);
  if (m.T > 1)
    hipLaunchKernelGGL((k_grad64<S, true>), dim3(nb), dim3(kBlock), 0, st, m, p, b, w, gE, grad);
  else
    hipLaunchKernelGGL((k_grad64<S, false>), dim3(nb), dim3(kBlock), 0, st, m, p, b, w, gE, grad);
  return hipGetLastError();
}

hipError_t launch_grad64(const ModelDev& m, const Model64& p, const EvalBuffers& b, const double* gF_sorted,
                         double gE, double* grad, int64_t n_params, hipStream_t st) {
  if (is_shape<FullShape>(m)) return grad64_shape<FullShape>(m, p, b, gF_sorted, gE, grad, n_params, st);
  if (is_shape<SurShape>(m)) return grad64_shape<SurShape>(m, p, b, gF_sorted, gE, grad, n_params, st);
  return hipErrorInvalidValue;
}

hipError_t launch_gather_vec64(int64_t N, const int32_t* perm, const double* aos_orig, double* soa_sorted,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_gather_vec64, dim3(grid_blocks(N)), dim3(kBlock), 0, st, N, perm, aos_orig, soa_sorted);
  return hipGetLastError();
}

hipError_t launch_scalar_out64(int64_t N, const int32_t* perm, const double* u, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_scalar_out64, dim3(grid_blocks(N)), dim3(kBlock), 0, st, N, perm, u, out);
  return hipGetLastError();
}

}  // namespace nep
