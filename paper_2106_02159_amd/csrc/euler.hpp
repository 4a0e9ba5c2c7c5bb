// euler.hpp -- device-side pieces of the hyperbolic step: the maximum wave
// speed bound and the pieces of the limiter line search (Sec. 3.1, 3.3).
#pragma once

#include <hip/hip_runtime.h>

namespace ns {

// FP64 reciprocal and square root from the hardware seeds (v_rcp_f64,
// v_rsq_f64) refined by Newton / Goldschmidt iterations: 5 and 10
// instructions instead of the 10-16 of the IEEE-exact sequences, which the
// VALU-bound graph-viscosity sweep spends most of its division and square
// root time in.  For positive normal arguments (the only ones they get:
// densities, pressures, |c_ij|, sums of positive terms) the results agree
// with the correctly rounded ones to within an ulp (on 2^20 samples over
// 2^-20 .. 2^20 both were exact).  fast_sqrt(0) is 0: the seed is taken at
// max(x, 2^-1000), so x * seed stays 0 and every later step keeps it there
// (|c_ii| = 0 on interior rows is an argument it does get).
__device__ __forceinline__ double fast_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

__device__ __forceinline__ double fast_sqrt(double x) {
  const double y = __builtin_amdgcn_rsq(fmax(x, 0x1p-1000));  // ~ x^(-1/2)
  double g = x * y, h = 0.5 * y;             // ~ x^(1/2), x^(-1/2)/2
  double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  return fma(fma(-g, g, x), h, g);           // one residual correction
}

// Exponent (gamma-1)/(2 gamma) of the two-rarefaction pressure and its
// inverse; for gamma = 7/5 the inverse is the integer 7.
struct Gas {
  double gamma;
  double gm1;      // gamma - 1
  double ex;       // (gamma - 1) / (2 gamma)
  double inv_ex;   // 2 gamma / (gamma - 1)
  double cg;       // (gamma + 1) / (2 gamma)
  double lgm1;     // log(gamma - 1)
  int seven;       // 1 when gamma == 7/5
};

// SEV: 1 when gamma == 7/5 is fixed at compile time (integer powers and the
// polynomial entropy test), 0 for a general gamma (pow).  The kernels are
// instantiated for both and the host picks by Gas::seven, so the gamma = 7/5
// kernels carry no pow code at all.
template <int SEV>
__device__ __forceinline__ double pow_inv_ex(const Gas &g, double x) {
  if constexpr (SEV) {
    const double x2 = x * x;
    const double x4 = x2 * x2;
    return x4 * x2 * x;
  }
  return pow(x, g.inv_ex);
}

// Guaranteed upper bound on the largest wave speed of the 1D Riemann problem
// with left state (uL, pL, aL) and right state (uR, pR, aR) along the unit
// direction n (u = v.n).  bL = aL pL^(-ex), bR likewise (precomputed per
// node).  Two-rarefaction bound on the star pressure, valid for
// 1 < gamma <= 5/3, inserted in the extreme shock/rarefaction speeds.
template <int SEV>
__device__ __forceinline__ double lambda_max(const Gas &g, double uL, double pL,
                                             double aL, double bL, double uR,
                                             double pR, double aR, double bR) {
  const double num = aL + aR - 0.5 * g.gm1 * (uR - uL);
  double ptr = 0.0;
  if (num > 0.0) ptr = pow_inv_ex<SEV>(g, num * fast_rcp(bL + bR));
  const double l1 =
      uL - aL * fast_sqrt(1.0 + g.cg * fmax(ptr * fast_rcp(pL) - 1.0, 0.0));
  const double l3 =
      uR + aR * fast_sqrt(1.0 + g.cg * fmax(ptr * fast_rcp(pR) - 1.0, 0.0));
  return fmax(fmax(-l1, 0.0), fmax(l3, 0.0));
}

// ---------------------------------------------------------------------------
// FP32 evaluation of the same bound for gamma = 7/5 (mixed-precision mode
// with FP32 arithmetic).  Approximate reciprocal and square root (1 ulp) are
// enough: the caller inflates the result by 2^-16 relative
// (kLambdaInflate) and uses it only where the rounding error is provably
// below that, i.e. where
//   (a) neither extreme speed u_L - a_L S_L, u_R + a_R S_R cancels by more
//       than a factor 3: max(|u| + a S) over both sides <= 3 lambda, and
//   (b) where a side is in the shock branch (S > 1), the star-pressure
//       numerator a_L + a_R - (gamma-1)/2 (u_R - u_L) cancels by at most a
//       factor 2 against a_L + a_R + (gamma-1)/2 (|u_L| + |u_R|) (its
//       relative error is amplified 7-fold by the power).
// With u = 2^-24 (the inputs rounded to FP32, the normal velocities formed
// in FP32): the numerator carries <= 8u relative, the quotient by b_L + b_R
// <= 12u, the 7th power <= 88u, p*/p <= 91u, each S <= 49u (dS/S <=
// d(p*/p)/2 since 1 - (gamma+1)/(2 gamma) > 0), each a S <= 51u, so each
// extreme speed is off by <= 52u (|u| + a S) <= 156u lambda, and with |c_ij|
// (3u) the product lambda |c_ij| by <= 160u < 2^-16 = 256u.  Elsewhere *ok
// is false and the caller evaluates lambda_max in FP64.
constexpr double kLambdaInflate = 1.0 + 1.0 / 65536.0;

__device__ __forceinline__ float lambda_max_f32(const Gas &g, float uL, float pL, float aL,
                                               float bL, float uR, float pR, float aR,
                                               float bR, bool *ok) {
  const float gm1 = (float)g.gm1, cg = (float)g.cg;
  const float num = aL + aR - 0.5f * gm1 * (uR - uL);
  float ptr = 0.0f;
  if (num > 0.0f) {
    const float x = num * __builtin_amdgcn_rcpf(bL + bR);
    const float x2 = x * x;
    const float x4 = x2 * x2;
    ptr = x4 * x2 * x;  // x^(2 gamma/(gamma-1)) = x^7
  }
  const float rL = ptr * __builtin_amdgcn_rcpf(pL), rR = ptr * __builtin_amdgcn_rcpf(pR);
  const float SL = __builtin_amdgcn_sqrtf(1.0f + cg * fmaxf(rL - 1.0f, 0.0f));
  const float SR = __builtin_amdgcn_sqrtf(1.0f + cg * fmaxf(rR - 1.0f, 0.0f));
  const float eL = aL * SL, eR = aR * SR;
  const float lam = fmaxf(fmaxf(eL - uL, 0.0f), fmaxf(uR + eR, 0.0f));
  const float M = fmaxf(fabsf(uL) + eL, fabsf(uR) + eR);
  const bool shock = rL > 0.999f || rR > 0.999f;
  *ok = M <= 3.0f * lam &&
        (!shock || aL + aR + 0.5f * gm1 * (fabsf(uL) + fabsf(uR)) <= 2.0f * num);
  return lam;
}

// psi(l) = eps(u + l P) - phi_min rho(u + l P)^gamma and its derivative.
template <int DIM>
__device__ __forceinline__ double psi_eval(const Gas &g, const double *u,
                                           const double *P, double l,
                                           double phi_min, double *dpsi) {
  const double r = u[0] + l * P[0];
  double m2 = 0.0, mp = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const double mk = u[1 + k] + l * P[1 + k];
    m2 += mk * mk;
    mp += mk * P[1 + k];
  }
  const double E = u[DIM + 1] + l * P[DIM + 1];
  const double ir = 1.0 / r;
  const double eps = E - 0.5 * m2 * ir;
  const double rg = pow(r, g.gamma);
  if (dpsi) {
    // d eps/dl = P_E - (m.P_m)/rho + |m|^2 P_rho / (2 rho^2)
    const double deps = P[DIM + 1] - mp * ir + 0.5 * m2 * ir * ir * P[0];
    *dpsi = deps - phi_min * g.gamma * rg * ir * P[0];
  }
  return eps - phi_min * rg;
}

// Is u + l P inside the entropy bound Phi >= phi_min?  For gamma = 7/5 the
// test eps >= phi_min rho^(7/5) is taken division- and pow-free as
// (rho eps)^5 >= phi_min^5 rho^12 with rho eps = rho E - |m|^2/2 (both sides
// are non-negative exactly when eps >= 0); pmin5 = phi_min^5.
template <int DIM, int SEV>
__device__ __forceinline__ bool entropy_ok(const Gas &g, const double *u,
                                           const double *P, double l,
                                           double phi_min, double pmin5) {
  // no fused multiply-adds of the compiler's choosing: a pair's two rows
  // evaluate the same test in different kernels and must agree bit for bit
#pragma clang fp contract(off)
  const double r = u[0] + l * P[0];
  double m2 = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const double mk = u[1 + k] + l * P[1 + k];
    m2 += mk * mk;
  }
  const double E = u[DIM + 1] + l * P[DIM + 1];
  if constexpr (SEV) {
    const double A = r * E - 0.5 * m2;
    if (!(A > 0.0)) return false;
    const double A2 = A * A;
    const double r2 = r * r, r4 = r2 * r2, r8 = r4 * r4;
    return A2 * A2 * A >= pmin5 * (r8 * r4);
  }
  else {
    return E - 0.5 * m2 / r - phi_min * pow(r, g.gamma) >= 0.0;
  }
}

// Root of psi in (a, b) with psi(a) >= 0 > psi(b).  psi is concave in l, so
// from the feasible end a the chord's root stays feasible and from the
// infeasible end b the tangent's root stays infeasible: both ends move towards
// the root at once.  Every candidate is checked by evaluating psi, so the
// returned end is feasible even under round-off.  Stops when the bracket is
// below 1e-14 (l is dimensionless, in [0,1]).
template <int DIM>
__device__ __forceinline__ double entropy_root(const Gas &g, const double *u,
                                            const double *P, double b,
                                            double phi_min) {
  double a = 0.0;
  double fa = psi_eval<DIM>(g, u, P, 0.0, phi_min, nullptr);
  double dfb;
  double fb = psi_eval<DIM>(g, u, P, b, phi_min, &dfb);
  if (fa < 0.0) return 0.0;
  if (fb >= 0.0) return b;
  for (int it = 0; it < 24 && b - a > 1e-14; ++it) {
    const double w0 = b - a;
    const double xs = a - fa * (b - a) / (fb - fa);
    if (xs > a && xs < b) {
      const double f = psi_eval<DIM>(g, u, P, xs, phi_min, nullptr);
      if (f >= 0.0) { a = xs; fa = f; }
      else { b = xs; fb = f; dfb = 0.0; }
    }
    if (dfb < 0.0) {
      const double xn = b - fb / dfb;
      if (xn > a && xn < b) {
        double d;
        const double f = psi_eval<DIM>(g, u, P, xn, phi_min, &d);
        if (f < 0.0) { b = xn; fb = f; dfb = d; }
        else { a = xn; fa = f; }
      }
    }
    if (b - a > 0.5 * w0) {
      const double xm = 0.5 * (a + b);
      double d;
      const double f = psi_eval<DIM>(g, u, P, xm, phi_min, &d);
      if (f >= 0.0) { a = xm; fa = f; }
      else { b = xm; fb = f; dfb = d; }
    }
    if (dfb == 0.0 && b - a > 1e-14) psi_eval<DIM>(g, u, P, b, phi_min, &dfb);
  }
  return a;
}

// Root of the entropy bound for gamma = 7/5 on the polynomial form of the
// test: g(l) = A(l)^5 - phi_min^5 rho(l)^12 with rho(l) = rho + l P_rho and
// A(l) = rho(l) E(l) - |m(l)|^2/2 = a0 + a1 l + a2 l^2 (rho(l) eps(l)).  g has
// the sign of psi wherever rho > 0, so its root in (0, b) is psi's.
// Safeguarded Newton inside the bracket [a, b] (g(a) >= 0 > g(b)), falling
// back to bisection when a Newton step leaves the bracket or shrinks it too
// little; stops at a bracket of 1e-14 and returns the feasible end.  No
// divisions by state values and no pow: a handful of FMAs per iteration.
template <int DIM>
__device__ __forceinline__ double entropy_root_seven(const double *u,
                                                    const double *P, double b,
                                                    double pmin5) {
  const double r0 = u[0], pr = P[0];
  double m0p = 0.0, pm2 = 0.0, m02 = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    m0p += u[1 + k] * P[1 + k];
    pm2 += P[1 + k] * P[1 + k];
    m02 += u[1 + k] * u[1 + k];
  }
  const double E0 = u[DIM + 1], pE = P[DIM + 1];
  const double a0 = r0 * E0 - 0.5 * m02;
  const double a1 = r0 * pE + pr * E0 - m0p;
  const double a2 = pr * pE - 0.5 * pm2;
  auto g = [&](double l, double *dg) {
    const double r = r0 + l * pr;
    const double A = a0 + l * (a1 + l * a2);
    const double dA = a1 + 2.0 * l * a2;
    const double A2 = A * A, A4 = A2 * A2;
    const double r2 = r * r, r4 = r2 * r2, r8 = r4 * r4, r11 = r8 * r2 * r;
    *dg = 5.0 * A4 * dA - 12.0 * pmin5 * r11 * pr;
    return A4 * A - pmin5 * (r11 * r);
  };
  double a = 0.0, dga, dgb;
  double ga = g(0.0, &dga);
  double gb = g(b, &dgb);
  if (!(ga >= 0.0)) return 0.0;
  if (gb >= 0.0) return b;
  // start from the chord's root, then Newton; once a Newton step is below
  // round-off the bracket is closed with two probes around it
  double x = a - ga * (b - a) / (gb - ga);
  if (!(x > a && x < b)) x = 0.5 * (a + b);
  for (int it = 0; it < 60 && b - a > 1e-14; ++it) {
    double dgx;
    const double gx = g(x, &dgx);
    if (gx >= 0.0) a = x;
    else b = x;
    if (b - a <= 1e-14) break;
    double xn = x - gx / dgx;
    if (!(xn > a && xn < b)) {
      xn = 0.5 * (a + b);
    } else if (fabs(xn - x) < 2e-15) {
      double d;
      const double lo = fmax(xn - 4e-15, a), hi = fmin(xn + 4e-15, b);
      if (g(lo, &d) >= 0.0) a = lo; else b = lo;
      if (hi > a && hi < b) {
        if (g(hi, &d) >= 0.0) a = hi; else b = hi;
      }
      xn = 0.5 * (a + b);
    }
    x = xn;
  }
  return a;
}

// Root of the entropy bound to the accuracy of psi itself.  For gamma = 7/5
// the polynomial root (whose own rounding can leave it ~1e-12 away) is
// followed by one Newton step on psi: psi is concave, so the tangent root x1
// lies at or beyond the root (within round-off of it from such a close
// start).  A point a below x1 with psi(a) >= 0 is then within x1 - a of the
// root; the rounding of psi blurs its sign change over a band whose width
// grows as psi flattens, so the step back from x1 grows (2e-15, 1.6e-14,
// 1.3e-13, 1e-12) until psi confirms a feasible point.  If none is confirmed
// (x1 was not close), the bracketing search on psi runs.
template <int DIM, int SEV>
__device__ __forceinline__ double entropy_root_fast(const Gas &g, const double *u,
                                                   const double *P, double lr,
                                                   double pmin, double pmin5) {
  if constexpr (SEV) {
    const double x = entropy_root_seven<DIM>(u, P, lr, pmin5);
    double d;
    const double f = psi_eval<DIM>(g, u, P, x, pmin, &d);
    if (d < 0.0) {
      const double x1 = x - f / d;
      if (x1 > 0.0 && x1 <= lr) {
        double h = 2e-15;
        for (int k = 0; k < 4; ++k, h *= 8.0) {
          const double a = fmax(x1 - h, 0.0);
          if (psi_eval<DIM>(g, u, P, a, pmin, nullptr) >= 0.0) return a;
        }
      }
    }
  }
  return entropy_root<DIM>(g, u, P, lr, pmin);
}

}  // namespace ns
