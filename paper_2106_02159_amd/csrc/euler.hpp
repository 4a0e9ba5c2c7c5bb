// euler.hpp -- device-side pieces of the hyperbolic step: the maximum wave
// speed bound and the limiter line search (Sec. 3.1 and 3.3).
#pragma once

#include <hip/hip_runtime.h>

namespace ns {

// Exponent (gamma-1)/(2 gamma) of the two-rarefaction pressure and its
// inverse; for gamma = 7/5 the inverse is the integer 7.
struct Gas {
  double gamma;
  double gm1;      // gamma - 1
  double ex;       // (gamma - 1) / (2 gamma)
  double inv_ex;   // 2 gamma / (gamma - 1)
  double cg;       // (gamma + 1) / (2 gamma)
  int seven;       // 1 when gamma == 7/5
};

__device__ __forceinline__ double pow_inv_ex(const Gas &g, double x) {
  if (g.seven) {
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
__device__ __forceinline__ double lambda_max(const Gas &g, double uL, double pL,
                                             double aL, double bL, double uR,
                                             double pR, double aR, double bR) {
  const double num = aL + aR - 0.5 * g.gm1 * (uR - uL);
  double ptr = 0.0;
  if (num > 0.0) ptr = pow_inv_ex(g, num / (bL + bR));
  const double l1 = uL - aL * sqrt(1.0 + g.cg * fmax(ptr / pL - 1.0, 0.0));
  const double l3 = uR + aR * sqrt(1.0 + g.cg * fmax(ptr / pR - 1.0, 0.0));
  return fmax(fmax(-l1, 0.0), fmax(l3, 0.0));
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

// Largest l in [0,1] keeping rho in [rho_min, rho_max] and Phi >= phi_min.
// Density is affine in l.  psi is concave in l, so from a feasible end a
// (psi >= 0) and an infeasible end b (psi < 0) the chord's root stays
// feasible and the tangent's root at b stays infeasible: both ends move
// towards the root at once.  Every candidate is checked by evaluating psi,
// so the returned end is feasible even under round-off.  Stops when the
// bracket is below 1e-14 (l is dimensionless, in [0,1]).
template <int DIM>
__device__ double line_search(const Gas &g, const double *u, const double *P,
                              double rho_min, double rho_max, double phi_min) {
  double lr;
  if (P[0] > 0.0) lr = (rho_max - u[0]) / P[0];
  else if (P[0] < 0.0) lr = (rho_min - u[0]) / P[0];
  else lr = 1.0;
  lr = fmin(fmax(lr, 0.0), 1.0);
  double db;
  const double pb = psi_eval<DIM>(g, u, P, lr, phi_min, &db);
  if (pb >= 0.0) return lr;
  const double pa0 = psi_eval<DIM>(g, u, P, 0.0, phi_min, nullptr);
  if (pa0 < 0.0) return 0.0;
  double a = 0.0, b = lr, fa = pa0, fb = pb, dfb = db;
  for (int it = 0; it < 24 && b - a > 1e-14; ++it) {
    const double w0 = b - a;
    // chord root (feasible side)
    double xs = a - fa * (b - a) / (fb - fa);
    if (xs > a && xs < b) {
      const double f = psi_eval<DIM>(g, u, P, xs, phi_min, nullptr);
      if (f >= 0.0) { a = xs; fa = f; }
      else { b = xs; fb = f; dfb = 0.0; }
    }
    // tangent root at b (infeasible side)
    if (dfb < 0.0) {
      const double xn = b - fb / dfb;
      if (xn > a && xn < b) {
        double d;
        const double f = psi_eval<DIM>(g, u, P, xn, phi_min, &d);
        if (f < 0.0) { b = xn; fb = f; dfb = d; }
        else { a = xn; fa = f; }
      }
    }
    // safeguard: bisect when the bracket did not halve
    if (b - a > 0.5 * w0) {
      const double xm = 0.5 * (a + b);
      double d;
      const double f = psi_eval<DIM>(g, u, P, xm, phi_min, &d);
      if (f >= 0.0) { a = xm; fa = f; }
      else { b = xm; fb = f; dfb = d; }
    }
    if (dfb == 0.0 && b - a > 1e-14) {
      // refresh the derivative at b for the next tangent step
      psi_eval<DIM>(g, u, P, b, phi_min, &dfb);
    }
  }
  return a;
}

}  // namespace ns
