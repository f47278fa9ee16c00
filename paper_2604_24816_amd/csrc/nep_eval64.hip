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

hipError_t launch_scalar_out64(int64_t N, const int32_t* perm, const double* u, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_scalar_out64, dim3(grid_blocks(N)), dim3(kBlock), 0, st, N, perm, u, out);
  return hipGetLastError();
}

}  // namespace nep
