// One ordered pair (target i, source j) of the regularised Rotne-Prager-Blake mobility,
// applied to the source's force and torque and added to the target's running sum.  Written
// once for float64 and float32.
//
// All lengths are in units of the radius a (the formulas below keep a for reference; the code
// takes a = 1, see PairConsts).
//
// Geometry (heights already clamped to z~ = max(z, a), paper App. A eq. effMob):
//   r = q~_i - q~_j = (dx, dy, dz)                    (direct separation)
//   R = q~_i - (x_j, y_j, -z~_j) = (dx, dy, Rz)       (separation from the source image)
//
// Unbounded part (Sec. II.B and Sec. III, the RPY forms to which the wall terms are added):
//   |r| >= 2a:  (1/|r|)[(1 + 2a^2/(3r^2)) I + (1 - 2a^2/r^2) rr/r^2],  rotation: T x r / |r|^3
//   |r| <  2a:  (4/(3a))[(1 - 9|r|/(32a)) I + (3/(32a)) rr/|r|],
//               rotation: (1 - 3|r|/(8a))/(2a^3) T x r
//   (the |r| = 0 limit is the Stokes self-mobility 4/(3a) I and no rotation coupling).
//
// Wall part: the Faxen operators of eq. mobilityDifferential applied to the image system of
// Blake's Green's function collapse, with e = R/|R|, X = a^2/|R|^2, Y = X^2, hh = z~_j/|R|,
// ez = e_z, to
//   8 pi eta W_tt = (1/|R|)[c1 I + c2 e e^T + c3 e z^T + c4 z e^T + c5 z z^T]
//     c1 = -1 + X(2ez^2 - 2/3) + Y(2/3 - 10/3 ez^2) - 2 ez hh + 2 hh^2
//     c2 = -1 + X(2 - 10 ez^2) + Y(70/3 ez^2 - 10/3) + 6 ez hh - 6 hh^2
//     c3 = hh(2 - 12 ez^2) + 12 ez hh^2 + X(20 ez^3 - 4 ez) + Y(40/3 ez - 140/3 ez^3)
//     c4 = 2 hh - 20/3 Y ez
//     c5 = -4 hh^2 - 4 X ez^2 + Y(20 ez^2 - 8/3)
// and those of eq. mobilityDifferentialTR to
//   8 pi eta W_tr T = (1/|R|^2)[ e x T + d2 (T x z) + (d3 e + d4 z) ((e x z) . T) ]
//     d2 = 2 X ez + 2 hh,  d3 = 10 X ez - 6 ez + 6 hh,  d4 = -2 X.
// The same expressions hold at i = j (R = (0, 0, 2 z~_i)), where they reduce to the wall
// self-mobility, so the self term needs no separate branch.
//
// Evaluation order (fewest operations): with t = hh (hh - ez), p = X(2 - 10/3 X) and
// q = 20/3 Y, the coefficients are
//     c1 = -1 + 2t - 2/3 (X - Y) + ez^2 p          c2 = -1 - 6t + p + ez^2 (q - 5p)
//     c3 = 2hh + 12 ez t + ez[(q - 2p) - 2 ez^2 (q - 5p)]
//     c4 = 2hh - ez q                               c5 = -4hh^2 - 4X ez^2 + Y(20 ez^2 - 8/3)
// and since r and R share their horizontal part rho = (dx, dy), unbounded and wall terms
// merge into one coefficient for F, one for rho and a z remainder.
//
// With WALL = false (free space) only the unbounded tensors are applied.
//
// Every value here carries the factor 8 pi eta a (8 pi eta a^2 for the torque coupling); the
// caller divides once per target.
#pragma once

#include <hip/hip_runtime.h>

namespace rpb {

// Lengths are in units of the sphere radius a (the packed geometry is divided by a), so the
// tensors take a = 1: M(r; a) = M(r/a; 1)/a and M_C(r; a) = M_C(r/a; 1)/a^2, and the caller
// applies 1/(8 pi eta a) per target and divides the torques by a.
// The closed forms' non-trivial constants travel with the box lengths: the kernels copy them
// into vector registers once (vgpr_consts), because in an isolated loop a float32 vector
// operation that reads a scalar register issued at about half the rate of one that reads
// vector registers or a literal (measured on gfx950).  In the pair kernels the change was
// within the run-to-run noise.
template <typename Real>
struct PairConsts {
  Real lx, ly;      // pseudo-periodic box in units of a (used by the PERIODIC kernels only)
  Real ilx, ily;    // 1/lx, 1/ly
  Real c2_3, c8_3, c10_3, c20_3, c70_3, c5, c6, c10, c12, c20;   // 2/3, 8/3, ..., 20
};

// Overlap branch (r < 2, units of a): cI = 4/3 - (3/8) r, cRR = (1/8)/r, cT = 1/2 - (3/16) r.
constexpr double kNearI = 4.0 / 3.0;
constexpr double kNearIR = 3.0 / 8.0;
constexpr double kNearRR = 1.0 / 8.0;
constexpr double kNearT = 0.5;
constexpr double kNearTR = 3.0 / 16.0;
constexpr double kFourA2 = 4.0;   // (2a)^2, the branch point

template <typename Real>
__host__ __device__ inline PairConsts<Real> make_pair_consts(double lx = 0.0, double ly = 0.0) {
  PairConsts<Real> k;
  k.lx = Real(lx);
  k.ly = Real(ly);
  k.ilx = lx > 0.0 ? Real(1.0 / lx) : Real(0);
  k.ily = ly > 0.0 ? Real(1.0 / ly) : Real(0);
  k.c2_3 = Real(2.0 / 3.0);
  k.c8_3 = Real(8.0 / 3.0);
  k.c10_3 = Real(10.0 / 3.0);
  k.c20_3 = Real(20.0 / 3.0);
  k.c70_3 = Real(70.0 / 3.0);
  k.c5 = Real(5);
  k.c6 = Real(6);
  k.c10 = Real(10);
  k.c12 = Real(12);
  k.c20 = Real(20);
  return k;
}

// A zero the compiler cannot see through, held in a vector register.
__device__ __forceinline__ float opaque_zero(float) {
  float z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  return z;
}
__device__ __forceinline__ double opaque_zero(double) { return double(opaque_zero(0.0f)); }

// The constants of `k` in vector registers (each plus an opaque zero: the same values, but the
// pair code's multiplications by them then read vector registers only).  Called once per
// kernel, outside the pair loops.
template <typename Real>
__device__ __forceinline__ PairConsts<Real> vgpr_consts(const PairConsts<Real> &k) {
  const Real z = opaque_zero(Real(0));
  PairConsts<Real> v = k;
  v.c2_3 = k.c2_3 + z;
  v.c8_3 = k.c8_3 + z;
  v.c10_3 = k.c10_3 + z;
  v.c20_3 = k.c20_3 + z;
  v.c70_3 = k.c70_3 + z;
  v.c5 = k.c5 + z;
  v.c6 = k.c6 + z;
  v.c10 = k.c10 + z;
  v.c12 = k.c12 + z;
  v.c20 = k.c20 + z;
  return v;
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

// Contribution of source j to the velocity of target i (8 pi eta units), added to
// (ox, oy, oz).  dx, dy: x_i - x_j, y_i - y_j; zi, zj: clamped heights; f: the source's weighted
// force; t: its weighted torque (used when TORQUE).  FAR_ONLY evaluates the |r| >= 2a form
// alone (cheaper; the caller routes pairs with |r|^2 < 4a^2 to FAR_ONLY = false).
template <typename Real, bool TORQUE, bool FAR_ONLY = false, bool WALL = true>
__device__ __forceinline__ void pair_velocity(Real dx, Real dy, Real zi, Real zj, Real fx, Real fy,
                                              Real fz, Real tx, Real ty, Real tz,
                                              const PairConsts<Real> &k, Real &ox, Real &oy,
                                              Real &oz) {
  const Real dz = zi - zj;
  const Real Rz = zi + zj;
  const Real rho2 = dx * dx + dy * dy;
  const Real r2 = rho2 + dz * dz;
  const Real R2 = rho2 + Rz * Rz;
  const Real iR = rsqrt_r(R2);

  // unbounded RPY: cI F + cRR r (r.F) [+ cT T x r]
  Real cI, cRR, cT;
  if (FAR_ONLY) {
    const Real invr = rsqrt_r(r2);
    const Real ir2 = invr * invr;
    const Real s = ir2;
    cI = invr * (Real(1) + k.c2_3 * s);
    cT = invr * ir2;
    cRR = cT * (Real(1) - Real(2) * s);
  } else {
    const Real invr = r2 > Real(0) ? rsqrt_r(r2) : Real(0);
    if (r2 >= Real(kFourA2)) {
      const Real ir2 = invr * invr;
      const Real s = ir2;
      cI = invr * (Real(1) + k.c2_3 * s);
      cT = invr * ir2;
      cRR = cT * (Real(1) - Real(2) * s);
    } else {
      const Real r = r2 * invr;
      cI = Real(kNearI) - Real(kNearIR) * r;
      cRR = Real(kNearRR) * invr;
      cT = Real(kNearT) - Real(kNearTR) * r;
    }
  }

  if (!WALL) {   // free space: the unbounded RPY tensors alone
    const Real cr = cRR * (dx * fx + dy * fy + dz * fz);
    ox += cI * fx;
    ox += cr * dx;
    oy += cI * fy;
    oy += cr * dy;
    oz += cI * fz;
    oz += cr * dz;
    if (TORQUE) {   // cT T x r
      ox += cT * (ty * dz - tz * dy);
      oy += cT * (tz * dx - tx * dz);
      oz += cT * (tx * dy - ty * dx);
    }
    return;
  }

  // wall coefficients
  const Real iR2 = iR * iR;
  const Real X = iR2;
  const Real Y = X * X;
  const Real ez = Rz * iR;
  const Real hh = zj * iR;
  const Real ez2 = ez * ez;
  const Real hme = hh - ez;
  const Real t = hh * hme;
  const Real p = X * (Real(2) - k.c10_3 * X);
  const Real q = k.c20_3 * Y;
  const Real hh2x = Real(2) * hh;
  const Real c1 = ez2 * p + (Real(2) * t + (-k.c2_3 * (X - Y) - Real(1)));
  const Real m1 = ez2 * (q - k.c5 * p);   // shared by c2 and c3 (10p - 2q = -2(q - 5p))
  const Real c2 = m1 + (-k.c6 * t + (p - Real(1)));
  const Real c3 = ez * ((q - Real(2) * p) + Real(-2) * m1) + (k.c12 * (ez * t) + hh2x);
  const Real c4 = hh2x - ez * q;
  const Real c5 = Y * (k.c20 * ez2 - k.c8_3) - Real(4) * (hh * hh + X * ez2);

  // apply to the force
  const Real rhoF = dx * fx + dy * fy;
  const Real rF = rhoF + dz * fz;
  const Real eF = (rhoF + Rz * fz) * iR;
  const Real G = c2 * eF + c3 * fz;              // coefficient of e   (times |R|)
  const Real H = c4 * eF + c5 * fz;              // coefficient of z   (times |R|)
  const Real A = cI + iR * c1;                   // coefficient of F
  const Real cr = cRR * rF;
  const Real B = cr + iR2 * G;                   // coefficient of rho
  ox += A * fx;
  ox += B * dx;
  oy += A * fy;
  oy += B * dy;
  oz += A * fz;
  oz += cr * dz;
  oz += iR * (G * ez + H);

  if (TORQUE) {
    // r x T and R x T share their rho terms: kv = (dy tz, -dx tz, dx ty - dy tx)
    const Real kx = dy * tz, ky = -(dx * tz), kz = dx * ty - dy * tx;
    const Real iR3 = iR * iR2;
    const Real al = iR3 - cT;                        // coefficient of kv
    const Real xez = X * ez;
    const Real d2 = Real(2) * xez + hh2x;
    const Real d3 = k.c10 * xez + k.c6 * hme;
    const Real s = -(kz * iR);                       // (e x z) . T
    const Real be = cT * dz + (iR2 * d2 - iR3 * Rz);  // coefficient of (ty, -tx, 0)
    const Real ga = iR3 * (s * d3);                  // coefficient of rho
    ox += al * kx;
    ox += be * ty;
    ox += ga * dx;
    oy += al * ky;
    oy += ga * dy;
    oy -= be * tx;
    oz += al * kz;
    oz += (iR2 * s) * (d3 * ez - Real(2) * X);
  }
}

// Coefficients of one unordered pair, shared by both directions (and by every source vector
// of a multi-vector product): the mobility matrix is symmetric, M_ji = M_ij^T (reciprocity of
// Blake's tensor; the unbounded part depends on r r^T and |r| only).
template <typename Real>
struct SymCoef {
  Real dx, dy, dz, Rz;   // r = (dx, dy, dz), R_z = z~_i + z~_j
  Real iR, iR2, ez;      // 1/|R|, 1/|R|^2, e_z
  Real cI, cRR, cT;      // unbounded: cI F + cRR r (r.F), rotation cT T x r
  Real A;                // cI + c1/|R| (coefficient of F)
  Real X, hh;            // a^2/|R|^2, z~_j/|R| (torque coupling)
  // The wall tensor applied to F, with s = dx F_x + dy F_y:
  //   u_x,y = A F_x,y + (b1 s + b2 F_z) (dx, dy),   u_z = A F_z + z1 s + z2 F_z,
  // and its transpose swaps b2 and z1.
  Real b1, b2, z1, z2;
};

template <typename Real, bool FAR_ONLY, bool TORQUE, bool WALL>
__device__ __forceinline__ void sym_coefficients(Real dx, Real dy, Real zi, Real zj,
                                                 const PairConsts<Real> &k, SymCoef<Real> &c) {
  const Real dz = zi - zj;
  const Real Rz = zi + zj;
  const Real rho2 = dx * dx + dy * dy;
  const Real r2 = rho2 + dz * dz;
  const Real R2 = rho2 + Rz * Rz;
  const Real iR = rsqrt_r(R2);
  c.dx = dx;
  c.dy = dy;
  c.dz = dz;
  c.Rz = Rz;
  c.iR = iR;

  Real cI, cRR, cT = Real(0);
  if (FAR_ONLY) {
    // valid for r2 >= (2a)^2 only: the caller routes closer pairs to FAR_ONLY = false
    const Real invr = rsqrt_r(r2);
    const Real ir2 = invr * invr;
    const Real s = ir2;
    cI = invr * (Real(1) + k.c2_3 * s);
    if (TORQUE) {
      cT = invr * ir2;
      cRR = cT * (Real(1) - Real(2) * s);
    } else {
      cRR = invr * ir2 * (Real(1) - Real(2) * s);
    }
  } else {
    const Real invr = r2 > Real(0) ? rsqrt_r(r2) : Real(0);
    if (r2 >= Real(kFourA2)) {
      const Real ir2 = invr * invr;
      const Real s = ir2;
      cI = invr * (Real(1) + k.c2_3 * s);
      if (TORQUE) {
        cT = invr * ir2;
        cRR = cT * (Real(1) - Real(2) * s);
      } else {
        cRR = invr * ir2 * (Real(1) - Real(2) * s);
      }
    } else {
      const Real r = r2 * invr;
      cI = Real(kNearI) - Real(kNearIR) * r;
      cRR = Real(kNearRR) * invr;
      if (TORQUE) cT = Real(kNearT) - Real(kNearTR) * r;
    }
  }
  c.cI = cI;
  c.cRR = cRR;
  c.cT = cT;
  if (!WALL) return;

  // Wall tensor in the basis {I, e e^T, e z^T, z e^T, z z^T}, e = R/|R|, with X = a^2/|R|^2,
  // Y = X^2, h = z~_j/|R|, t = h (h - e_z), p = 2X - 10Y/3, q = 20Y/3, m = e_z^2 (q - 5p):
  //   c1 = e_z^2 p + 2t - 2(X - Y)/3 - 1,  c2 = m - 6t + p - 1,
  //   c3 = e_z (q - 2p - 2m) + 12 e_z t + 2h,  c4 = 2h - e_z q,
  //   c5 = Y (20 e_z^2 - 8/3) - 4 (h^2 + X e_z^2).
  // Expanded over (dx, dy, dz) together with the unbounded r r^T term, only these enter:
  //   A = cI + c1/|R|,  b1 = cRR + c2/|R|^3,  b2 = cRR dz + (c2 e_z + c3)/|R|^2,
  //   z1 = cRR dz + (c2 e_z + c4)/|R|^2,  z2 = cRR dz^2 + (c2 e_z^2 + (c3 + c4) e_z + c5)/|R|,
  // and with g = m - 6t + p, u = e_z (g - q):
  //   c2 e_z + c3 = 2h - e_z - u,  c2 e_z + c4 = 2h - e_z + u,
  //   c2 e_z^2 + (c3 + c4) e_z + c5 = e_z^2 (6t - m + 70Y/3 - 6X - 1) - 4t - 8Y/3.
  const Real iR2 = iR * iR;
  const Real X = iR2;
  const Real Y = X * X;
  const Real ez = Rz * iR;
  const Real hh = zj * iR;
  const Real ez2 = ez * ez;
  const Real t = hh * (hh - ez);
  const Real p = X * (Real(2) - k.c10_3 * X);
  const Real q = k.c20_3 * Y;
  const Real m = ez2 * (q - k.c5 * p);
  const Real c1 = ez2 * p + (Real(2) * t + (-k.c2_3 * (X - Y) - Real(1)));
  const Real g = m + (-k.c6 * t + p);
  const Real u = ez * (g - q);
  const Real h2e = Real(2) * hh - ez;
  const Real bx = ez2 * ((k.c6 * t - m) + (k.c70_3 * Y - (k.c6 * X + Real(1)))) -
                  (Real(4) * t + k.c8_3 * Y);
  c.A = cI + iR * c1;
  const Real iR3 = iR * iR2;
  const Real crdz = cRR * dz;
  c.b1 = (g - Real(1)) * iR3 + cRR;
  c.b2 = (h2e - u) * iR2 + crdz;
  c.z1 = (h2e + u) * iR2 + crdz;
  c.z2 = crdz * dz + bx * iR;
  c.iR2 = iR2;
  c.ez = ez;
  c.X = X;
  c.hh = hh;
}

// (o) += M_ij f (velocity of i from source j's force f) and (p) += M_ij^T g (velocity of j from
// target i's force g), 8 pi eta units; M_ij^T swaps the roles of c3 and c4 (e z^T <-> z e^T).
template <typename Real, bool WALL>
__device__ __forceinline__ void sym_apply(const SymCoef<Real> &c, Real fx, Real fy, Real fz,
                                          Real gx, Real gy, Real gz, Real &ox, Real &oy,
                                          Real &oz, Real &px, Real &py, Real &pz) {
  const Real dx = c.dx, dy = c.dy, dz = c.dz;
  if (!WALL) {   // free space: the unbounded RPY tensors alone (r -> -r for j <- i)
    const Real cr = c.cRR * (dx * fx + dy * fy + dz * fz);
    const Real cr2 = c.cRR * (dx * gx + dy * gy + dz * gz);
    ox += c.cI * fx;
    ox += cr * dx;
    oy += c.cI * fy;
    oy += cr * dy;
    oz += c.cI * fz;
    oz += cr * dz;
    px += c.cI * gx;
    px += cr2 * dx;
    py += c.cI * gy;
    py += cr2 * dy;
    pz += c.cI * gz;
    pz += cr2 * dz;
    return;
  }
  // i <- j
  const Real s = dx * fx + dy * fy;
  const Real B = c.b1 * s + c.b2 * fz;
  ox += c.A * fx;
  ox += B * dx;
  oy += c.A * fy;
  oy += B * dy;
  oz += c.A * fz;
  oz += c.z1 * s;
  oz += c.z2 * fz;

  // j <- i (transposed tensor: b2 and z1 swap)
  const Real s2 = dx * gx + dy * gy;
  const Real B2 = c.b1 * s2 + c.z1 * gz;
  px += c.A * gx;
  px += B2 * dx;
  py += c.A * gy;
  py += B2 * dy;
  pz += c.A * gz;
  pz += c.b2 * s2;
  pz += c.z2 * gz;
}

// The coupling terms of both directions, (o) += M^C_ij T_j and (p) += M^C_ji T_i (tq: T_j,
// uq: T_i).  M^C has no symmetry, but M^C_ji is the same expression with r -> -r and the image
// height hh = z~_j/|R| replaced by z~_i/|R|, so everything else (|R|, e_z, X, the unbounded
// coefficient) is shared.
template <typename Real, bool WALL>
__device__ __forceinline__ void sym_apply_torque(const SymCoef<Real> &c, const PairConsts<Real> &k,
                                                 Real zi, const Real *tq, const Real *uq, Real &ox,
                                                 Real &oy, Real &oz, Real &px, Real &py, Real &pz) {
  const Real dx = c.dx, dy = c.dy, dz = c.dz, cT = c.cT;
  if (!WALL) {   // cT T_j x r into o, cT T_i x (-r) into p
    ox += cT * (tq[1] * dz - tq[2] * dy);
    oy += cT * (tq[2] * dx - tq[0] * dz);
    oz += cT * (tq[0] * dy - tq[1] * dx);
    px -= cT * (uq[1] * dz - uq[2] * dy);
    py -= cT * (uq[2] * dx - uq[0] * dz);
    pz -= cT * (uq[0] * dy - uq[1] * dx);
    return;
  }
  const Real iR = c.iR, iR2 = c.iR2, ez = c.ez, X = c.X, Rz = c.Rz;
  const Real iR3 = iR * iR2;
  const Real iR4 = iR2 * iR2;
  const Real al = iR3 - cT;                 // coefficient of k (both directions)
  const Real xez = X * ez;
  const Real be0 = iR2 * (Real(2) * xez) - iR3 * Rz;
  const Real d30 = k.c10 * xez - k.c6 * ez;
  const Real wz = d30 * ez - Real(2) * X;   // with the image-height part added per direction
  const Real iR2x2 = Real(2) * iR2;
  const Real ez6 = k.c6 * ez;
  // Per direction, with k = (r_x, r_y, 0) x T = (r_y T_z, -r_x T_z, K):
  //   u_x,y += al k_x,y + be (T_y, -T_x) + ga (r_x, r_y),   u_z += K (al - (wz + 6 h e_z)/|R|^3),
  //   be = 2h/|R|^2 + be0 + cT r_z,   ga = -K (d30 + 6h)/|R|^4,   h = image height / |R|.
  {  // i <- j: torque T_j, r = (dx, dy, dz), image height z~_j
    const Real hh = c.hh;
    const Real tx = tq[0], ty = tq[1], tz = tq[2];
    const Real K = dx * ty - dy * tx;
    const Real P = al * tz;
    const Real be = iR2x2 * hh + (cT * dz + be0);
    const Real ga = -K * (iR4 * (k.c6 * hh + d30));
    const Real cz = al - iR3 * (hh * ez6 + wz);
    ox += P * dy;
    ox += be * ty;
    ox += ga * dx;
    oy -= P * dx;
    oy += ga * dy;
    oy -= be * tx;
    oz += K * cz;
  }
  {  // j <- i: torque T_i, r -> -r, image height z~_i
    const Real hi = zi * iR;
    const Real tx = uq[0], ty = uq[1], tz = uq[2];
    const Real K = dy * tx - dx * ty;
    const Real P = al * tz;
    const Real be = iR2x2 * hi + (be0 - cT * dz);
    const Real ga = -K * (iR4 * (k.c6 * hi + d30));
    const Real cz = al - iR3 * (hi * ez6 + wz);
    px -= P * dy;
    px += be * ty;
    px -= ga * dx;
    py += P * dx;
    py -= ga * dy;
    py -= be * tx;
    pz += K * cz;
  }
}

// One direction only: (o) += M_ij f.
template <typename Real, bool WALL>
__device__ __forceinline__ void sym_apply_one(const SymCoef<Real> &c, Real fx, Real fy, Real fz,
                                              Real &ox, Real &oy, Real &oz) {
  const Real dx = c.dx, dy = c.dy, dz = c.dz;
  if (!WALL) {
    const Real cr = c.cRR * (dx * fx + dy * fy + dz * fz);
    ox += c.cI * fx;
    ox += cr * dx;
    oy += c.cI * fy;
    oy += cr * dy;
    oz += c.cI * fz;
    oz += cr * dz;
    return;
  }
  const Real s = dx * fx + dy * fy;
  const Real B = c.b1 * s + c.b2 * fz;
  ox += c.A * fx;
  ox += B * dx;
  oy += c.A * fy;
  oy += B * dy;
  oz += c.A * fz;
  oz += c.z1 * s;
  oz += c.z2 * fz;
}

// Both directions of one unordered pair (force and, with TORQUE, torque sources).
template <typename Real, bool FAR_ONLY = false, bool TORQUE = false, bool WALL = true>
__device__ __forceinline__ void pair_velocity_sym(Real dx, Real dy, Real zi, Real zj, Real fx,
                                                  Real fy, Real fz, Real gx, Real gy, Real gz,
                                                  const PairConsts<Real> &k, Real &ox, Real &oy,
                                                  Real &oz, Real &px, Real &py, Real &pz,
                                                  const Real *tq = nullptr,
                                                  const Real *uq = nullptr) {
  SymCoef<Real> c;
  sym_coefficients<Real, FAR_ONLY, TORQUE, WALL>(dx, dy, zi, zj, k, c);
  sym_apply<Real, WALL>(c, fx, fy, fz, gx, gy, gz, ox, oy, oz, px, py, pz);
  if (TORQUE) sym_apply_torque<Real, WALL>(c, k, zi, tq, uq, ox, oy, oz, px, py, pz);
}

__device__ __forceinline__ float round_nearest(float x) { return __builtin_rintf(x); }
__device__ __forceinline__ double round_nearest(double x) { return __builtin_rint(x); }

// Calls f(dx', dy') for the pair separation: once as given, or, with pseudo-periodic
// boundaries (App. B), for the minimum image (|dx|, |dy| <= L/2) and its images in the eight
// neighbour cells.
template <bool PERIODIC, typename Real, typename F>
__device__ __forceinline__ void for_images(Real dx, Real dy, const PairConsts<Real> &k, F &&f) {
  if (!PERIODIC) {
    f(dx, dy);
    return;
  }
  dx -= k.lx * round_nearest(dx * k.ilx);
  dy -= k.ly * round_nearest(dy * k.ily);
  // Kept as a loop: nine inlined copies of the pair code (times the callers' own unrolling)
  // would exhaust the vector registers and leave one wavefront per SIMD.
#pragma unroll 1
  for (int ix = -1; ix <= 1; ++ix)
#pragma unroll 1
    for (int iy = -1; iy <= 1; ++iy) f(dx + Real(ix) * k.lx, dy + Real(iy) * k.ly);
}

}  // namespace rpb
