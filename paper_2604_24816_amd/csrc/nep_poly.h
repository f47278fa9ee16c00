// Real solid harmonics up to l = 4 as homogeneous polynomials P_lm of a unit
// vector u = (x, y, z), with their Cartesian gradients, for the angular
// descriptors (Section III.B: radial functions times spherical harmonics,
// contracted over m; Algorithm 1 keeps 24 (l, m) components for l_max = 4).
//
// The orthonormal harmonics are Y_lm = N_lm P_lm(u). Only the rotation
// invariants sum_m Y_lm(a) Y_lm(b) = (2l+1)/(4 pi) P_l(a.b) enter the
// descriptor, so the kernels accumulate unnormalised sums s_lm = sum_j g P_lm
// and fold the normalisation into one weight per component,
//   q_nl = sum_m kW[lm] * s_nlm^2,   kW[lm] = 4 pi N_lm^2 / (2l + 1),
// which reproduces q_nl = (4 pi / (2l+1)) sum_m (sum_j g Y_lm)^2.
// Component order: l = 1: y, z, x; l = 2: xy, yz, 3z^2-r^2, xz, x^2-y^2;
// l = 3 and l = 4 in the usual m = -l..l order of the real harmonics.
#pragma once

namespace nep {

__device__ constexpr float kW[24] = {
    1.f, 1.f, 1.f,                                                // l = 1
    3.f, 3.f, 0.25f, 3.f, 0.75f,                                  // l = 2
    0.625f, 15.f, 0.375f, 0.25f, 0.375f, 3.75f, 0.625f,           // l = 3
    8.75f, 4.375f, 1.25f, 0.625f, 0.015625f, 0.625f, 0.3125f, 4.375f, 0.546875f  // l = 4
};

__host__ __device__ constexpr int comp_l(int lm) {
  return lm < 3 ? 1 : (lm < 8 ? 2 : (lm < 15 ? 3 : 4));
}

// Calls f(lm, P) for every component lm < NC (NC = 3, 8, 15 or 24).
template <int NC, typename Fn>
__device__ __forceinline__ void for_each_poly(float x, float y, float z, Fn&& f) {
  f(0, y);
  f(1, z);
  f(2, x);
  if constexpr (NC > 3) {
    const float x2 = x * x, y2 = y * y, z2 = z * z;
    f(3, x * y);
    f(4, y * z);
    f(5, 2.f * z2 - x2 - y2);
    f(6, x * z);
    f(7, x2 - y2);
    if constexpr (NC > 8) {
      const float t = 4.f * z2 - x2 - y2;
      f(8, y * (3.f * x2 - y2));
      f(9, x * y * z);
      f(10, y * t);
      f(11, z * (2.f * z2 - 3.f * x2 - 3.f * y2));
      f(12, x * t);
      f(13, z * (x2 - y2));
      f(14, x * (x2 - 3.f * y2));
      if constexpr (NC > 15) {
        const float rho2 = x2 + y2;
        const float a = 6.f * z2 - rho2;
        const float b = 4.f * z2 - 3.f * rho2;
        f(15, x * y * (x2 - y2));
        f(16, y * z * (3.f * x2 - y2));
        f(17, x * y * a);
        f(18, y * z * b);
        f(19, 8.f * z2 * z2 - 24.f * z2 * rho2 + 3.f * rho2 * rho2);
        f(20, x * z * b);
        f(21, (x2 - y2) * a);
        f(22, x * z * (x2 - 3.f * y2));
        f(23, x2 * x2 - 6.f * x2 * y2 + y2 * y2);
      }
    }
  }
}

// Calls f(lm, P, dP/dx, dP/dy, dP/dz) with the gradient of the homogeneous
// polynomial evaluated at u.
template <int NC, typename Fn>
__device__ __forceinline__ void for_each_poly_grad(float x, float y, float z, Fn&& f) {
  f(0, y, 0.f, 1.f, 0.f);
  f(1, z, 0.f, 0.f, 1.f);
  f(2, x, 1.f, 0.f, 0.f);
  if constexpr (NC > 3) {
    const float x2 = x * x, y2 = y * y, z2 = z * z;
    f(3, x * y, y, x, 0.f);
    f(4, y * z, 0.f, z, y);
    f(5, 2.f * z2 - x2 - y2, -2.f * x, -2.f * y, 4.f * z);
    f(6, x * z, z, 0.f, x);
    f(7, x2 - y2, 2.f * x, -2.f * y, 0.f);
    if constexpr (NC > 8) {
      const float xy = x * y, xz = x * z, yz = y * z;
      const float t = 4.f * z2 - x2 - y2;
      f(8, y * (3.f * x2 - y2), 6.f * xy, 3.f * (x2 - y2), 0.f);
      f(9, xy * z, yz, xz, xy);
      f(10, y * t, -2.f * xy, 4.f * z2 - x2 - 3.f * y2, 8.f * yz);
      f(11, z * (2.f * z2 - 3.f * x2 - 3.f * y2), -6.f * xz, -6.f * yz, 6.f * z2 - 3.f * x2 - 3.f * y2);
      f(12, x * t, 4.f * z2 - 3.f * x2 - y2, -2.f * xy, 8.f * xz);
      f(13, z * (x2 - y2), 2.f * xz, -2.f * yz, x2 - y2);
      f(14, x * (x2 - 3.f * y2), 3.f * (x2 - y2), -6.f * xy, 0.f);
      if constexpr (NC > 15) {
        const float rho2 = x2 + y2;
        const float a = 6.f * z2 - rho2;
        const float b = 4.f * z2 - 3.f * rho2;
        const float xyz = xy * z;
        f(15, xy * (x2 - y2), 3.f * x2 * y - y2 * y, x2 * x - 3.f * x * y2, 0.f);
        f(16, yz * (3.f * x2 - y2), 6.f * xyz, 3.f * z * (x2 - y2), y * (3.f * x2 - y2));
        f(17, xy * a, y * (6.f * z2 - 3.f * x2 - y2), x * (6.f * z2 - x2 - 3.f * y2), 12.f * xyz);
        f(18, yz * b, -6.f * xyz, z * (4.f * z2 - 3.f * x2 - 9.f * y2), 3.f * y * (4.f * z2 - rho2));
        f(19, 8.f * z2 * z2 - 24.f * z2 * rho2 + 3.f * rho2 * rho2, 12.f * x * (rho2 - 4.f * z2),
          12.f * y * (rho2 - 4.f * z2), 16.f * z * (2.f * z2 - 3.f * rho2));
        f(20, xz * b, z * (4.f * z2 - 9.f * x2 - 3.f * y2), -6.f * xyz, 3.f * x * (4.f * z2 - rho2));
        f(21, (x2 - y2) * a, 4.f * x * (3.f * z2 - x2), 4.f * y * (y2 - 3.f * z2), 12.f * z * (x2 - y2));
        f(22, xz * (x2 - 3.f * y2), 3.f * z * (x2 - y2), -6.f * xyz, x * (x2 - 3.f * y2));
        f(23, x2 * x2 - 6.f * x2 * y2 + y2 * y2, 4.f * x * (x2 - 3.f * y2), 4.f * y * (y2 - 3.f * x2), 0.f);
      }
    }
  }
}

}  // namespace nep
