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

// A gradient component that vanishes identically. It converts to 0 where a caller takes
// plain numbers; callers that overload on it drop the products with it.
struct Zero {
  __host__ __device__ constexpr operator float() const { return 0.f; }
  __host__ __device__ constexpr operator double() const { return 0.0; }
};

__host__ __device__ constexpr int comp_l(int lm) {
  return lm < 3 ? 1 : (lm < 8 ? 2 : (lm < 15 ? 3 : 4));
}

// Calls f(lm, P) for every component lm < NC (NC = 3, 8, 15 or 24).
template <int NC, typename R, typename Fn>
__device__ __forceinline__ void for_each_poly(R x, R y, R z, Fn&& f) {
  f(0, y);
  f(1, z);
  f(2, x);
  if constexpr (NC > 3) {
    const R x2 = x * x, y2 = y * y, z2 = z * z;
    f(3, x * y);
    f(4, y * z);
    f(5, R(2) * z2 - x2 - y2);
    f(6, x * z);
    f(7, x2 - y2);
    if constexpr (NC > 8) {
      const R t = R(4) * z2 - x2 - y2;
      f(8, y * (R(3) * x2 - y2));
      f(9, x * y * z);
      f(10, y * t);
      f(11, z * (R(2) * z2 - R(3) * x2 - R(3) * y2));
      f(12, x * t);
      f(13, z * (x2 - y2));
      f(14, x * (x2 - R(3) * y2));
      if constexpr (NC > 15) {
        const R rho2 = x2 + y2;
        const R a = R(6) * z2 - rho2;
        const R b = R(4) * z2 - R(3) * rho2;
        f(15, x * y * (x2 - y2));
        f(16, y * z * (R(3) * x2 - y2));
        f(17, x * y * a);
        f(18, y * z * b);
        f(19, R(8) * z2 * z2 - R(24) * z2 * rho2 + R(3) * rho2 * rho2);
        f(20, x * z * b);
        f(21, (x2 - y2) * a);
        f(22, x * z * (x2 - R(3) * y2));
        f(23, x2 * x2 - R(6) * x2 * y2 + y2 * y2);
      }
    }
  }
}

// Calls f(lm, P, dP/dx, dP/dy, dP/dz) with the gradient of the homogeneous
// polynomial evaluated at u; components that vanish identically are passed as Zero.
template <int NC, typename R, typename Fn>
__device__ __forceinline__ void for_each_poly_grad(R x, R y, R z, Fn&& f) {
  f(0, y, Zero{}, R(1), Zero{});
  f(1, z, Zero{}, Zero{}, R(1));
  f(2, x, R(1), Zero{}, Zero{});
  if constexpr (NC > 3) {
    const R x2 = x * x, y2 = y * y, z2 = z * z;
    f(3, x * y, y, x, Zero{});
    f(4, y * z, Zero{}, z, y);
    f(5, R(2) * z2 - x2 - y2, -R(2) * x, -R(2) * y, R(4) * z);
    f(6, x * z, z, Zero{}, x);
    f(7, x2 - y2, R(2) * x, -R(2) * y, Zero{});
    if constexpr (NC > 8) {
      const R xy = x * y, xz = x * z, yz = y * z;
      const R t = R(4) * z2 - x2 - y2;
      f(8, y * (R(3) * x2 - y2), R(6) * xy, R(3) * (x2 - y2), Zero{});
      f(9, xy * z, yz, xz, xy);
      f(10, y * t, -R(2) * xy, R(4) * z2 - x2 - R(3) * y2, R(8) * yz);
      f(11, z * (R(2) * z2 - R(3) * x2 - R(3) * y2), -R(6) * xz, -R(6) * yz, R(6) * z2 - R(3) * x2 - R(3) * y2);
      f(12, x * t, R(4) * z2 - R(3) * x2 - y2, -R(2) * xy, R(8) * xz);
      f(13, z * (x2 - y2), R(2) * xz, -R(2) * yz, x2 - y2);
      f(14, x * (x2 - R(3) * y2), R(3) * (x2 - y2), -R(6) * xy, Zero{});
      if constexpr (NC > 15) {
        const R rho2 = x2 + y2;
        const R a = R(6) * z2 - rho2;
        const R b = R(4) * z2 - R(3) * rho2;
        const R xyz = xy * z;
        f(15, xy * (x2 - y2), R(3) * x2 * y - y2 * y, x2 * x - R(3) * x * y2, Zero{});
        f(16, yz * (R(3) * x2 - y2), R(6) * xyz, R(3) * z * (x2 - y2), y * (R(3) * x2 - y2));
        f(17, xy * a, y * (R(6) * z2 - R(3) * x2 - y2), x * (R(6) * z2 - x2 - R(3) * y2), R(12) * xyz);
        f(18, yz * b, -R(6) * xyz, z * (R(4) * z2 - R(3) * x2 - R(9) * y2), R(3) * y * (R(4) * z2 - rho2));
        f(19, R(8) * z2 * z2 - R(24) * z2 * rho2 + R(3) * rho2 * rho2, R(12) * x * (rho2 - R(4) * z2),
          R(12) * y * (rho2 - R(4) * z2), R(16) * z * (R(2) * z2 - R(3) * rho2));
        f(20, xz * b, z * (R(4) * z2 - R(9) * x2 - R(3) * y2), -R(6) * xyz, R(3) * x * (R(4) * z2 - rho2));
        f(21, (x2 - y2) * a, R(4) * x * (R(3) * z2 - x2), R(4) * y * (y2 - R(3) * z2), R(12) * z * (x2 - y2));
        f(22, xz * (x2 - R(3) * y2), R(3) * z * (x2 - y2), -R(6) * xyz, x * (x2 - R(3) * y2));
        f(23, x2 * x2 - R(6) * x2 * y2 + y2 * y2, R(4) * x * (x2 - R(3) * y2), R(4) * y * (y2 - R(3) * x2), Zero{});
      }
    }
  }
}

}  // namespace nep
