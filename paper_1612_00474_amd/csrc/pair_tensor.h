// One ordered pair (target i, source j) of the regularised Rotne-Prager-Blake mobility,
// applied to the source's force and torque.  Written once for float64 and float32.
//
// Geometry (heights already clamped to z~ = max(z, a), paper App. A eq. effMob):
//   r = q~_i - q~_j                                   (direct separation)
//   R = q~_i - (x_j, y_j, -z~_j),  e = R/|R|          (separation from the source image)
//
// Unbounded part (Sec. II.B and Sec. III, the RPY forms to which the wall terms are added):
//   |r| >= 2a:  (1/|r|)[(1 + 2a^2/(3r^2)) I + (1 - 2a^2/r^2) rr/r^2],  rotation: T x r / |r|^3
//   |r| <  2a:  (4/(3a))[(1 - 9|r|/(32a)) I + (3/(32a)) rr/|r|],      rotation: (1 - 3|r|/(8a))/(2a^3) T x r
//   (the |r| = 0 limit is the Stokes self-mobility 4/(3a) I and no rotation coupling).
//
// Wall part: the Faxen operators of eq. mobilityDifferential applied to the image system of
// Blake's Green's function collapse, with A = a/|R|, hh = z~_j/|R| and ez = e_z, to
//   8 pi eta W_tt = (1/|R|)[c1 I + c2 e e^T + c3 e z^T + c4 z e^T + c5 z z^T]
//     c1 = -1 + A^2(2ez^2 - 2/3) + A^4(2/3 - 10/3 ez^2) - 2 ez hh + 2 hh^2
//     c2 = -1 + A^2(2 - 10 ez^2) + A^4(70/3 ez^2 - 10/3) + 6 ez hh - 6 hh^2
//     c3 = hh(2 - 12 ez^2) + 12 ez hh^2 + A^2(20 ez^3 - 4 ez) + A^4(40/3 ez - 140/3 ez^3)
//     c4 = 2 hh - 20/3 A^4 ez
//     c5 = -4 hh^2 - 4 A^2 ez^2 + A^4(20 ez^2 - 8/3)
// and those of eq. mobilityDifferentialTR to
//   8 pi eta W_tr T = (1/|R|^2)[ e x T + d2 (T x z) + (d3 e + d4 z) ((e x z) . T) ]
//     d2 = 2 A^2 ez + 2 hh,  d3 = 10 A^2 ez - 6 ez + 6 hh,  d4 = -2 A^2.
// The same expressions hold at i = j (R = (0, 0, 2 z~_i)), where they reduce to the wall
// self-mobility, so the self term needs no separate branch.
//
// Every value here carries the factor 8 pi eta; the caller divides once per target.
#pragma once

#include <hip/hip_runtime.h>

namespace rpb {

template <typename Real>
struct PairConsts {
  Real a2;          // a^2
  Real four_a2;     // (2a)^2, branch point
  Real near_i;      // 4/(3a)
  Real near_i_r;    // 4/(3a) * 9/(32a)
  Real near_rr;     // 4/(3a) * 3/(32a)
  Real near_t;      // 1/(2a^3)
  Real near_t_r;    // 1/(2a^3) * 3/(8a)
};

template <typename Real>
__host__ __device__ inline PairConsts<Real> make_pair_consts(double a) {
  PairConsts<Real> k;
  k.a2 = Real(a * a);
  k.four_a2 = Real(4.0 * a * a);
  k.near_i = Real(4.0 / (3.0 * a));
  k.near_i_r = Real(4.0 / (3.0 * a) * 9.0 / (32.0 * a));
  k.near_rr = Real(4.0 / (3.0 * a) * 3.0 / (32.0 * a));
  k.near_t = Real(1.0 / (2.0 * a * a * a));
  k.near_t_r = Real(1.0 / (2.0 * a * a * a) * 3.0 / (8.0 * a));
  return k;
}

// 1/sqrt(x) for x > 0.
__device__ __forceinline__ float rsqrt_r(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_r(double x) {
  // hardware estimate, then one third-order Newton step on e = 1 - x y^2:
  // y (1 + e/2 + 3e^2/8) = y (1 - e)^{-1/2} + O(e^3)
  double y = __builtin_amdgcn_rsq(x);
  const double e = __builtin_fma(-x * y, y, 1.0);
  return __builtin_fma(y * e, __builtin_fma(e, 0.375, 0.5), y);
}

// Contribution of source j to the velocity of target i (8 pi eta units).
// dx, dy: horizontal separation x_i - x_j, y_i - y_j; zi, zj: clamped heights.
// f: the source's weighted force; t: its weighted torque (used when TORQUE).
template <typename Real, bool TORQUE>
__device__ __forceinline__ void pair_velocity(Real dx, Real dy, Real zi, Real zj, Real fx, Real fy,
                                              Real fz, Real tx, Real ty, Real tz,
                                              const PairConsts<Real> &k, Real &ox, Real &oy,
                                              Real &oz) {
  const Real dz = zi - zj;
  const Real Rz = zi + zj;
  const Real rho2 = dx * dx + dy * dy;
  const Real r2 = rho2 + dz * dz;
  const Real R2 = rho2 + Rz * Rz;
  const Real invr = r2 > Real(0) ? rsqrt_r(r2) : Real(0);
  const Real invR = rsqrt_r(R2);

  // unbounded RPY coefficients: U = cI F + cRR r (r.F) [+ cT T x r]
  Real cI, cRR, cT;
  if (r2 >= k.four_a2) {
    const Real ir2 = invr * invr;
    const Real s = k.a2 * ir2;
    cI = invr * (Real(1) + Real(2.0 / 3.0) * s);
    cRR = invr * ir2 * (Real(1) - Real(2) * s);
    cT = invr * ir2;
  } else {
    const Real r = r2 * invr;
    cI = k.near_i - k.near_i_r * r;
    cRR = k.near_rr * invr;
    cT = k.near_t - k.near_t_r * r;
  }

  // wall coefficients
  const Real ex = dx * invR, ey = dy * invR, ez = Rz * invR;
  const Real hh = zj * invR;
  const Real A2 = k.a2 * invR * invR;
  const Real A4 = A2 * A2;
  const Real ez2 = ez * ez;
  const Real hh2 = hh * hh;
  const Real ezhh = ez * hh;
  const Real c1 = Real(-1) + A2 * (Real(2) * ez2 - Real(2.0 / 3.0)) +
                  A4 * (Real(2.0 / 3.0) - Real(10.0 / 3.0) * ez2) - Real(2) * ezhh + Real(2) * hh2;
  const Real c2 = Real(-1) + A2 * (Real(2) - Real(10) * ez2) +
                  A4 * (Real(70.0 / 3.0) * ez2 - Real(10.0 / 3.0)) + Real(6) * ezhh - Real(6) * hh2;
  const Real c3 = hh * (Real(2) - Real(12) * ez2) + Real(12) * ezhh * hh +
                  ez * (A2 * (Real(20) * ez2 - Real(4)) + A4 * (Real(40.0 / 3.0) - Real(140.0 / 3.0) * ez2));
  const Real c4 = Real(2) * hh - Real(20.0 / 3.0) * A4 * ez;
  const Real c5 = Real(-4) * hh2 - Real(4) * A2 * ez2 + A4 * (Real(20) * ez2 - Real(8.0 / 3.0));

  const Real rF = dx * fx + dy * fy + dz * fz;
  const Real eF = ex * fx + ey * fy + ez * fz;
  const Real cF = cI + invR * c1;
  const Real ce = invR * (c2 * eF + c3 * fz);
  const Real cz = invR * (c4 * eF + c5 * fz);
  const Real cr = cRR * rF;
  ox = cF * fx + cr * dx + ce * ex;
  oy = cF * fy + cr * dy + ce * ey;
  oz = cF * fz + cr * dz + ce * ez + cz;

  if (TORQUE) {
    // unbounded: cT (T x r)
    ox += cT * (ty * dz - tz * dy);
    oy += cT * (tz * dx - tx * dz);
    oz += cT * (tx * dy - ty * dx);
    // wall: (1/|R|^2)[e x T + d2 (T x z) + (d3 e + d4 z) s],  s = (e x z) . T
    const Real iR2 = invR * invR;
    const Real s = ey * tx - ex * ty;
    const Real d2 = Real(2) * (A2 * ez + hh);
    const Real d3s = (Real(10) * A2 * ez - Real(6) * ez + Real(6) * hh) * s;
    const Real d4s = Real(-2) * A2 * s;
    ox += iR2 * (ey * tz - ez * ty + d2 * ty + d3s * ex);
    oy += iR2 * (ez * tx - ex * tz - d2 * tx + d3s * ey);
    oz += iR2 * (d3s * ez + d4s - s);
  }
}

}  // namespace rpb
