// Velocity-Verlet integration in FP64, the rebuild trigger, FP64 reductions and
// the conversions between the caller's original atom order ([N][3] rows) and
// the cell-sorted structure-of-arrays layout ([3][N]) used on the device.
// Section VI.A: 1 fs steps, neighbour lists refreshed every 10 steps with the
// displacement check enabled.
#include "nep_common.h"

namespace nep {
namespace {

__global__ void k_reduce_partials(const double* __restrict__ partial, int nblocks, int first, int nvals,
                                  double* __restrict__ out) {
  __shared__ double sh[kBlock];
  for (int k = 0; k < nvals; ++k) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kBlock) s += partial[(int64_t)b * kPartialStride + first + k];
    __syncthreads();
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
      if (threadIdx.x < (unsigned)off) sh[threadIdx.x] += sh[threadIdx.x + off];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[k] = sh[0];
  }
}

__device__ __forceinline__ double wrap_coord(double xv, double L) {
  if (xv < 0.0) xv += L;
  else if (xv >= L) xv -= L;
  return xv;
}

// v += dt/2 F/(m xi); x += dt v; wrap; flag a rebuild when |x - x_build| > skin/2.
// Strides over a capped grid (kIntegrateGrid workgroups), so that the per-workgroup maxima
// of the squared displacement that k_select_bin reads are few.
constexpr int kIntegrateGrid = 8192;

__global__ void k_kick_drift(int64_t N, double dt, CellGrid g, const float* __restrict__ F,
                             const int32_t* __restrict__ type, MassTable mt, double* __restrict__ x,
                             double* __restrict__ v, uint4* __restrict__ pos, const double* __restrict__ xb,
                             double half_skin2,
                             int32_t* __restrict__ flags, double* __restrict__ partial) {
  __shared__ double sh[kBlock / 64];
  double d2max = 0.0;
  bool moved = false;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (int64_t)gridDim.x * blockDim.x) {
    const double inv = mt.inv_mxi[type[p]];
    double xn[3];
    double d2 = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double vv = v[c * N + p] + 0.5 * dt * (double)F[c * N + p] * inv;
      const double xx = wrap_coord(x[c * N + p] + dt * vv, g.box[c]);
      v[c * N + p] = vv;
      x[c * N + p] = xx;
      xn[c] = xx;
      const double d = min_image(xx - xb[c * N + p], g.box[c]);
      d2 += d * d;
    }
    pos_put(pos, p, xn[0], xn[1], xn[2], g.box);
    if (!(d2 <= half_skin2)) moved = true;  // also catches NaN
    if (!(d2 == d2)) d2 = 1e300;
    d2max = fmax(d2max, d2);
  }
  if (moved) flags[FLAG_REBUILD] = 1;
  // largest squared displacement since the build, per workgroup
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) d2max = fmax(d2max, __shfl_xor(d2max, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = d2max;
  __syncthreads();
  if (threadIdx.x == 0)
    partial[(int64_t)blockIdx.x * kPartialStride + P_MAXD2] =
        fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

// k = first bin fraction with bin_frac(k) * skin >= 2 * (largest displacement since the
// build); the evaluation visits the bins up to the edges rc_radial + f_k skin and
// rc_angular + f_k skin. A rebuild later in the same step resets them to k = 0.
constexpr int kSelBlock = 1024;  // one workgroup reads every partial: many loads in flight

__global__ void __launch_bounds__(kSelBlock)
k_select_bin(const double* __restrict__ partial, int nblocks, int32_t* flags, double skin, BinEdges be) {
  __shared__ double sh[kSelBlock];
  double m = 0.0;
#pragma unroll 4
  for (int b = threadIdx.x; b < nblocks; b += kSelBlock)
    m = fmax(m, partial[(int64_t)b * kPartialStride + P_MAXD2]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int off = kSelBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < (unsigned)off) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double d = sqrt(sh[0]);
  int k = kFracs - 1;
  for (int j = kFracs - 1; j >= 0; --j)
    if ((double)bin_frac(j) * skin >= 2.0 * d * (1.0 + 1e-12)) k = j;
  int br0 = 0, ba0 = 0, br1 = 0, ba1 = 0;
  for (int j = 0; j < kFracs; ++j)
    if (j == k) {
      br0 = be.idxR[0][j];
      ba0 = be.idxA[0][j];
      br1 = be.idxR[1][j];
      ba1 = be.idxA[1][j];
    }
  flags[FLAG_BIN_R] = br0;
  flags[FLAG_BIN_A] = ba0;
  flags[FLAG_BIN_R1] = br1;
  flags[FLAG_BIN_A1] = ba1;
}

__global__ void k_kick(int64_t N, double dt, const float* __restrict__ F, const int32_t* __restrict__ type,
                       MassTable mt, double* __restrict__ v) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const double inv = mt.inv_mxi[type[p]];
  for (int c = 0; c < 3; ++c) v[c * N + p] += 0.5 * dt * (double)F[c * N + p] * inv;
}

// v += dt (Fa - Fb)/(m xi)
__global__ void k_kick_diff(int64_t N, double dt, const float* __restrict__ Fa, const float* __restrict__ Fb,
                            const int32_t* __restrict__ type, MassTable mt, double* __restrict__ v) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const double inv = mt.inv_mxi[type[p]];
  for (int c = 0; c < 3; ++c)
    v[c * N + p] += dt * ((double)Fa[c * N + p] - (double)Fb[c * N + p]) * inv;
}

__device__ __forceinline__ void block_partial(double val, double* sh, double* out) {
  __syncthreads();
  sh[threadIdx.x] = val;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < (unsigned)off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

__global__ void k_kinetic(int64_t N, const double* __restrict__ v, const int32_t* __restrict__ type,
                          MassTable mt, double* __restrict__ partial) {
  __shared__ double sh[kBlock];
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double ke = 0.0;
  if (p < N) {
    const double m = mt.mass[type[p]];
    for (int c = 0; c < 3; ++c) ke += v[c * N + p] * v[c * N + p];
    ke *= 0.5 * m * 103.642697;
  }
  block_partial(ke, sh, partial + (int64_t)blockIdx.x * kPartialStride + P_KE);
}

__global__ void k_force_error(int64_t N, const float* __restrict__ Fa, const float* __restrict__ Fb,
                              double* __restrict__ partial) {
  __shared__ double sh[kBlock];
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double e2 = 0.0, f2 = 0.0;
  if (p < N) {
    for (int c = 0; c < 3; ++c) {
      const double a = (double)Fa[c * N + p];
      const double d = a - (double)Fb[c * N + p];
      e2 += d * d;
      f2 += a * a;
    }
  }
  block_partial(e2, sh, partial + (int64_t)blockIdx.x * kPartialStride + P_ERR2);
  block_partial(f2, sh, partial + (int64_t)blockIdx.x * kPartialStride + P_F2);
  // maximum |e| over the block
  __syncthreads();
  sh[threadIdx.x] = sqrt(e2);
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < (unsigned)off) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * kPartialStride + P_ERRMAX] = sh[0];
}

// One half step (h = dt/2) of a Nose-Hoover chain in the explicit reversible
// Trotter form of Martyna, Tuckerman, Tobias and Klein (1996), FP64, one thread.
// nhc = {eta[kMaxChain], v_eta[kMaxChain], scale}; ke = the current kinetic energy.
// Chain masses Q_1 = Nf kT tau^2, Q_k = kT tau^2; forces G_1 = (2 KE - Nf kT)/Q_1,
// G_k = (Q_{k-1} v_{k-1}^2 - kT)/Q_k. The outermost velocity takes a quarter-step kick,
// the chain is swept inwards (each v_k damped by exp(-v_{k+1} h/4) around its kick),
// the particle velocities are to be scaled by exp(-v_1 h), the positions advance by
// v_k h, and the chain is swept outwards again with the forces recomputed.
__global__ void k_nhc_half(const double* __restrict__ ke_in, double* __restrict__ nhc, int M, double kT,
                           double Nf, double tau2, double h) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double* eta = nhc;
  double* ve = nhc + kMaxChain;
  double ke = *ke_in;
  const double Q1 = Nf * kT * tau2, Qk = kT * tau2;
  auto force = [&](int k) {
    return k == 0 ? (2.0 * ke - Nf * kT) / Q1 : ((k == 1 ? Q1 : Qk) * ve[k - 1] * ve[k - 1] - kT) / Qk;
  };
  const int L = M - 1;
  ve[L] += 0.5 * h * force(L);
  for (int k = L - 1; k >= 0; --k) {
    const double d = exp(-0.25 * h * ve[k + 1]);
    ve[k] = (ve[k] * d + 0.5 * h * force(k)) * d;
  }
  const double sc = exp(-h * ve[0]);
  ke *= sc * sc;
  for (int k = 0; k < M; ++k) eta[k] += h * ve[k];
  for (int k = 0; k < L; ++k) {
    const double d = exp(-0.25 * h * ve[k + 1]);
    ve[k] = (ve[k] * d + 0.5 * h * force(k)) * d;
  }
  ve[L] += 0.5 * h * force(L);
  nhc[2 * kMaxChain] = sc;
}

// v *= scale (the chain's velocity scaling), all 3N components.
__global__ void k_scale_v(int64_t n3, const double* __restrict__ scale, double* __restrict__ v) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n3) v[k] *= *scale;
}

__global__ void k_max_partials(const double* __restrict__ partial, int nblocks, int slot,
                               double* __restrict__ out) {
  __shared__ double sh[kBlock];
  double m = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kBlock) m = fmax(m, partial[(int64_t)b * kPartialStride + slot]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int off = kBlock / 2; off > 0; off >>= 1) {
    if (threadIdx.x < (unsigned)off) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + off]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

__global__ void k_sum_i32(int64_t N, const int32_t* __restrict__ a, double* __restrict__ partial, int slot) {
  __shared__ double sh[kBlock];
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  block_partial(p < N ? (double)a[p] : 0.0, sh, partial + (int64_t)blockIdx.x * kPartialStride + slot);
}

__global__ void k_set_flag(int32_t* flags, int idx, int value) {
  if (threadIdx.x == 0) flags[idx] = value;
}

__global__ void k_state_in(int64_t N, const double* __restrict__ xa, const double* __restrict__ va,
                           const int32_t* __restrict__ tin, int n_types, CellGrid g, double* __restrict__ x,
                           double* __restrict__ v, int32_t* __restrict__ type, int32_t* __restrict__ perm,
                           uint4* __restrict__ pos, int32_t* __restrict__ flags) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  double xn[3];
  for (int c = 0; c < 3; ++c) {
    double xv = xa[3 * p + c];
    if (!isfinite(xv)) flags[FLAG_NONFINITE] = 1;
    else if (xv < 0.0 || xv >= g.box[c]) {
      xv = xv - g.box[c] * floor(xv / g.box[c]);
      if (xv >= g.box[c]) xv -= g.box[c];
    }
    x[c * N + p] = xv;
    xn[c] = xv;
    const double vv = va ? va[3 * p + c] : 0.0;
    if (!isfinite(vv)) flags[FLAG_NONFINITE] = 1;
    v[c * N + p] = vv;
  }
  pos_put(pos, p, xn[0], xn[1], xn[2], g.box);
  const int t = tin[p];
  if (t < 0 || t >= n_types) flags[FLAG_TYPE] = 1;
  type[p] = (t < 0 || t >= n_types) ? 0 : t;
  perm[p] = (int32_t)p;
}

__global__ void k_state_out(int64_t N, const int32_t* __restrict__ perm, const double* __restrict__ soa,
                            double* __restrict__ aos) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const int64_t o = perm[p];
  for (int c = 0; c < 3; ++c) aos[3 * o + c] = soa[c * N + p];
}

__global__ void k_forces_out(int64_t N, const int32_t* __restrict__ perm, const float* __restrict__ F,
                             double* __restrict__ aos) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const int64_t o = perm[p];
  for (int c = 0; c < 3; ++c) aos[3 * o + c] = (double)F[c * N + p];
}

__global__ void k_scalar_out(int64_t N, const int32_t* __restrict__ perm, const float* __restrict__ U,
                             double* __restrict__ out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  out[perm[p]] = (double)U[p];
}

__global__ void k_gather_vec_f32(int64_t N, const int32_t* __restrict__ perm, const float* __restrict__ a,
                                 float* __restrict__ s) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const int64_t o = perm[p];
  for (int c = 0; c < 3; ++c) s[c * N + p] = a[3 * o + c];
}

__global__ void k_scatter_vec_f32(int64_t N, const int32_t* __restrict__ perm, const float* __restrict__ s,
                                  float* __restrict__ a) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= N) return;
  const int64_t o = perm[p];
  for (int c = 0; c < 3; ++c) a[3 * o + c] = s[c * N + p];
}

}  // namespace

hipError_t launch_reduce_partials(const double* partial, int nblocks, int first, int nvals, double* out,
                                  hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_partials, dim3(1), dim3(kBlock), 0, st, partial, nblocks, first, nvals, out);
  return hipGetLastError();
}

hipError_t launch_max_partials(const double* partial, int nblocks, int slot, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_max_partials, dim3(1), dim3(kBlock), 0, st, partial, nblocks, slot, out);
  return hipGetLastError();
}

int kick_drift_blocks(int64_t N) {
  const int nb = grid_blocks(N);
  return nb < kIntegrateGrid ? nb : kIntegrateGrid;
}

hipError_t launch_kick_drift(int64_t N, double dt, CellGrid g, const float* F, const int32_t* type,
                             MassTable mt, double* x, double* v, uint4* pos, const double* x_build,
                             double half_skin2, int32_t* flags, double* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_kick_drift, dim3(kick_drift_blocks(N)), dim3(kBlock), 0, st, N, dt, g, F, type, mt, x, v,
                     pos, x_build, half_skin2, flags, partial);
  return hipGetLastError();
}

hipError_t launch_select_bin(const double* partial, int nblocks, int32_t* flags, double skin,
                             const BinEdges& be, hipStream_t st) {
  hipLaunchKernelGGL(k_select_bin, dim3(1), dim3(kSelBlock), 0, st, partial, nblocks, flags, skin, be);
  return hipGetLastError();
}

hipError_t launch_nhc_half(int64_t N, const double* ke, double* nhc, int M, double kT, double tau, double h,
                           double* v, hipStream_t st) {
  hipLaunchKernelGGL(k_nhc_half, dim3(1), dim3(64), 0, st, ke, nhc, M, kT, 3.0 * (double)N - 3.0, tau * tau, h);
  hipLaunchKernelGGL(k_scale_v, dim3(grid_blocks(3 * N)), dim3(kBlock), 0, st, 3 * N, nhc + 2 * kMaxChain, v);
  return hipGetLastError();
}

hipError_t launch_kick(int64_t N, double dt, const float* F, const int32_t* type, MassTable mt, double* v,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_kick, dim3(grid_blocks(N)), dim3(kBlock), 0, st, N, dt, F, type, mt, v);
  return hipGetLastError();
}

hipError_t launch_kick_diff(int64_t N, double dt, const float* Fa, const float* Fb, const int32_t* type,
                            MassTable mt, double* v, hipStream_t st) {
  hipLaunchKernelGGL(k_kick_diff, dim3(grid_blocks(N)), dim3(kBlock), 0, st, N, dt, Fa, Fb, type, mt, v);
  return hipGetLastError();
}

hipError_t launch_kinetic(int64_t N, const double* v, const int32_t* type, MassTable mt, double* partial,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_kinetic, dim3(grid_blocks(N)), dim3(kBlock), 0, st, N, v, type, mt, partial);
  return hipGetLastError();
}

hipError_t launch_force_error(int64_t N, const float* Fa, const float* Fb, double* partial,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_force_error, dim3(grid_blocks(N)), dim3(kBlock), 0, st, N, Fa, Fb, partial);
  return hipGetLastError();
}

hipError_t launch_sum_i32(int64_t N, const int32_t* a, double* partial, int slot, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_i32, dim3(grid_blocks(N)), dim3(kBlock), 0, st, N, a, partial, slot);
  return hipGetLastError();
}

hipError_t launch_set_flag(int32_t* flags, int idx, int value, hipStream_t st) {
  hipLaunchKernelGGL(k_set_flag, dim3(1), dim3(64), 0, st, flags, idx, value);
  return hipGetLastError();
}

hipError_t launch_state_in(int64_t N, const double* x_aos, const double* v_aos, const int32_t* type_in,
                           int n_types, CellGrid g, double* x, double* v, int32_t* type, int32_t* perm,
                           uint4* pos, int32_t* flags, hipStream_t st) {
  hipLaunchKernelGGL(k_state_in, dim3(grid_blocks(N)), dim3(kBlock), 0, st, N, x_aos, v_aos, type_in,
                     n_types, g, x, v, type, perm, pos, flags);
  return hipGetLastError();
}

hipError_t launch_state_out(int64_t N, const int32_t* perm, const double* soa, double* aos, hipStream_t st) {
  hipLaunchKernelGGL(k_state_out, dim3(grid_blocks(N)), dim3(kBlock), 0, st, N, perm, soa, aos);
  return hipGetLastError();
}

hipError_t launch_forces_out(int64_t N, const int32_t* perm, const float* F, double* aos, hipStream_t st) {
  hipLaunchKernelGGL(k_forces_out, dim3(grid_blocks(N)), dim3(kBlock), 0, st, N, perm, F, aos);
  return hipGetLastError();
}

hipError_t launch_scalar_out(int64_t N, const int32_t* perm, const float* U, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_scalar_out, dim3(grid_blocks(N)), dim3(kBlock), 0, st, N, perm, U, out);
  return hipGetLastError();
}

hipError_t launch_gather_vec_f32(int64_t N, const int32_t* perm, const float* aos_orig, float* soa_sorted,
                                 hipStream_t st) {
  hipLaunchKernelGGL(k_gather_vec_f32, dim3(grid_blocks(N)), dim3(kBlock), 0, st, N, perm, aos_orig,
                     soa_sorted);
  return hipGetLastError();
}

hipError_t launch_scatter_vec_f32(int64_t N, const int32_t* perm, const float* soa_sorted, float* aos_orig,
                                  hipStream_t st) {
  hipLaunchKernelGGL(k_scatter_vec_f32, dim3(grid_blocks(N)), dim3(kBlock), 0, st, N, perm, soa_sorted,
                     aos_orig);
  return hipGetLastError();
}

}  // namespace nep
