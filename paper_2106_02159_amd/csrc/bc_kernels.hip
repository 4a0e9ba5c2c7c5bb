// bc_kernels.hip -- non-reflecting boundary post-processing (Sec. 4.3:
// Godunov's method, Sec. 4.3.1; characteristic variables, Sec. 4.3.2):
// one lane per listed boundary node, after each forward-Euler stage.
//
// Characteristic variables (gamma-law, locally isentropic flow): with the
// node state U, the far-field state U^D and the outward unit normal n,
//   lambda_1,2,3 = v_n - a, v_n, v_n + a;  C_1,3 = v_n -+ 2a/(gamma-1);
//   S = p rho^-gamma;  v_perp = v - v_n n.
// Supersonic inflow (lambda_3 < 0) takes U^D, supersonic outflow
// (0 <= lambda_1) keeps U; subsonic flow takes C_1 from U^D and C_3 from U,
// S and v_perp from U^D (inflow, v_n < 0) or U (outflow), and so
//   v_n^P = (C_1 + C_3)/2,  a^P = (gamma-1)/4 (C_3 - C_1),
//   rho^P = ((a^P)^2 / (gamma S))^(1/(gamma-1)),  p^P = S (rho^P)^gamma.
// Godunov: the exact solution at x = 0 of the Riemann problem along n with
// the node state on the left (inside) and U^D on the right (outside); the
// tangential velocity comes from the side of the contact x = 0 lies on.
// The star pressure is the root of f(p) = f_L(p) + f_R(p) + u_R - u_L,
// f increasing and concave, found by Newton from the two-rarefaction
// estimate (a Newton step from either side of the root of an increasing
// concave function lands at or right of it and then decreases
// monotonically), to round-off.  Vacuum data keep U and are flagged.
#include "hyp_kernels.hpp"

namespace ns {
namespace {

struct Prim {
  double rho, vn, vt[3], p, a;
};

template <int DIM>
__device__ __forceinline__ Prim primitives(const Gas &g, const double *U, const double *n) {
  Prim q;
  q.rho = U[0];
  double m2 = 0.0, vn = 0.0, v[DIM];
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    v[k] = U[1 + k] / q.rho;
    m2 += U[1 + k] * U[1 + k];
    vn += v[k] * n[k];
  }
  q.vn = vn;
#pragma unroll
  for (int k = 0; k < DIM; ++k) q.vt[k] = v[k] - vn * n[k];
  q.p = g.gm1 * (U[DIM + 1] - 0.5 * m2 / q.rho);
  q.a = sqrt(g.gamma * q.p / q.rho);
  return q;
}

template <int DIM>
__device__ __forceinline__ void conserved(const Gas &g, double rho, double un,
                                          const double *vt, double p, const double *n,
                                          double *UP) {
  double m2 = 0.0;
  UP[0] = rho;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    UP[1 + k] = rho * (vt[k] + un * n[k]);
    m2 += UP[1 + k] * UP[1 + k];
  }
  UP[DIM + 1] = p / g.gm1 + 0.5 * m2 / rho;
}

// f_K(p) and its derivative: shock branch above p_K, rarefaction below
__device__ __forceinline__ double side_fn(const Gas &g, double p, double rk, double pk,
                                          double ak, double *df) {
  if (p > pk) {
    const double A = 2.0 / ((g.gamma + 1.0) * rk);
    const double B = g.gm1 / (g.gamma + 1.0) * pk;
    const double q = sqrt(A / (p + B));
    *df = q * (1.0 - 0.5 * (p - pk) / (p + B));
    return (p - pk) * q;
  }
  const double r = pow(p / pk, g.ex);
  *df = r / (rk * ak) * (pk / p);
  return 2.0 * ak / g.gm1 * (r - 1.0);
}

// star pressure and velocity; false for vacuum
__device__ bool riemann_star(const Gas &g, double rl, double ul, double pl, double rr,
                             double ur, double pr, double *ps, double *us) {
  const double al = sqrt(g.gamma * pl / rl), ar = sqrt(g.gamma * pr / rr);
  const double du = ur - ul;
  if (2.0 * (al + ar) / g.gm1 <= du) return false;
  // two-rarefaction estimate: exact when both waves are rarefactions
  double p = pow((al + ar - 0.5 * g.gm1 * du) /
                     (al * pow(pl, -g.ex) + ar * pow(pr, -g.ex)),
                 g.inv_ex);
  for (int it = 0; it < 60; ++it) {
    double dl, dr;
    const double f = side_fn(g, p, rl, pl, al, &dl) + side_fn(g, p, rr, pr, ar, &dr) + du;
    double pn = p - f / (dl + dr);
    if (!(pn > 0.0)) pn = 0.5 * p;
    const bool done = fabs(pn - p) <= 4e-16 * pn;
    p = pn;
    if (done) break;
  }
  double dl, dr;
  *ps = p;
  *us = 0.5 * (ul + ur) + 0.5 * (side_fn(g, p, rr, pr, ar, &dr) - side_fn(g, p, rl, pl, al, &dl));
  return true;
}

// solution at x/t = 0; side -1 / +1: left / right of the contact
__device__ bool riemann_at_zero(const Gas &g, double rl, double ul, double pl, double rr,
                                double ur, double pr, double *rho, double *u, double *p,
                                int *side) {
  double ps, us;
  if (!riemann_star(g, rl, ul, pl, rr, ur, pr, &ps, &us)) return false;
  const double gp1 = g.gamma + 1.0, gm = g.gm1 / gp1;
  if (0.0 <= us) {
    *side = -1;
    const double al = sqrt(g.gamma * pl / rl);
    if (ps > pl) {
      const double sl = ul - al * sqrt(gp1 / (2.0 * g.gamma) * ps / pl + g.gm1 / (2.0 * g.gamma));
      if (0.0 <= sl) { *rho = rl; *u = ul; *p = pl; }
      else { *rho = rl * (ps / pl + gm) / (gm * ps / pl + 1.0); *u = us; *p = ps; }
    } else {
      const double head = ul - al;
      const double tail = us - al * pow(ps / pl, g.ex);
      if (0.0 <= head) { *rho = rl; *u = ul; *p = pl; }
      else if (0.0 >= tail) { *rho = rl * pow(ps / pl, 1.0 / g.gamma); *u = us; *p = ps; }
      else {
        const double c = 2.0 / gp1 + g.gm1 / (gp1 * al) * ul;
        *rho = rl * pow(c, 2.0 / g.gm1);
        *u = 2.0 / gp1 * (al + 0.5 * g.gm1 * ul);
        *p = pl * pow(c, 2.0 * g.gamma / g.gm1);
      }
    }
  } else {
    *side = 1;
    const double ar = sqrt(g.gamma * pr / rr);
    if (ps > pr) {
      const double sr = ur + ar * sqrt(gp1 / (2.0 * g.gamma) * ps / pr + g.gm1 / (2.0 * g.gamma));
      if (0.0 >= sr) { *rho = rr; *u = ur; *p = pr; }
      else { *rho = rr * (ps / pr + gm) / (gm * ps / pr + 1.0); *u = us; *p = ps; }
    } else {
      const double head = ur + ar;
      const double tail = us + ar * pow(ps / pr, g.ex);
      if (0.0 >= head) { *rho = rr; *u = ur; *p = pr; }
      else if (0.0 <= tail) { *rho = rr * pow(ps / pr, 1.0 / g.gamma); *u = us; *p = ps; }
      else {
        const double c = 2.0 / gp1 - g.gm1 / (gp1 * ar) * ur;
        *rho = rr * pow(c, 2.0 / g.gm1);
        *u = 2.0 / gp1 * (-ar + 0.5 * g.gm1 * ur);
        *p = pr * pow(c, 2.0 * g.gamma / g.gm1);
      }
    }
  }
  return true;
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_nonreflecting(int n, const int32_t *__restrict__ idx,
                                                          const double *__restrict__ nrm,
                                                          const double *__restrict__ ud,
                                                          int method, Gas g, int64_t N,
                                                          double *__restrict__ U,
                                                          int *__restrict__ flags) {
  constexpr int NC = DIM + 2;
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= n) return;
  const int64_t i = idx[t];
  double u[NC], d[NC], nv[DIM], up[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    u[c] = U[node_at(NC, c, i, N)];
    d[c] = ud[(int64_t)c * n + t];
  }
#pragma unroll
  for (int k = 0; k < DIM; ++k) nv[k] = nrm[(int64_t)k * n + t];
  const Prim q = primitives<DIM>(g, u, nv), f = primitives<DIM>(g, d, nv);
  bool ok = true;
  if (method == 1) {
    double rho, un, p;
    int side;
    ok = riemann_at_zero(g, q.rho, q.vn, q.p, f.rho, f.vn, f.p, &rho, &un, &p, &side);
    if (ok) conserved<DIM>(g, rho, un, side < 0 ? q.vt : f.vt, p, nv, up);
    else
#pragma unroll
      for (int c = 0; c < NC; ++c) up[c] = u[c];
  } else if (q.vn < 0.0 && q.a < fabs(q.vn)) {  // supersonic inflow
#pragma unroll
    for (int c = 0; c < NC; ++c) up[c] = d[c];
  } else if (q.vn >= 0.0 && q.a <= fabs(q.vn)) {  // supersonic outflow
#pragma unroll
    for (int c = 0; c < NC; ++c) up[c] = u[c];
  } else {  // subsonic
    const bool inflow = q.vn < 0.0;
    const double C1 = f.vn - 2.0 * f.a / g.gm1;
    const double C3 = q.vn + 2.0 * q.a / g.gm1;
    const double S = inflow ? f.p * pow(f.rho, -g.gamma) : q.p * pow(q.rho, -g.gamma);
    const double un = 0.5 * (C1 + C3);
    const double aP = 0.25 * g.gm1 * (C3 - C1);
    const double rho = pow(aP * aP / (g.gamma * S), 1.0 / g.gm1);
    const double p = S * pow(rho, g.gamma);
    conserved<DIM>(g, rho, un, inflow ? f.vt : q.vt, p, nv, up);
  }
  double m2 = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) m2 += up[1 + k] * up[1 + k];
  if (!ok || !(up[0] > 0.0) || !(up[NC - 1] - 0.5 * m2 / up[0] > 0.0)) flags[1] = 1;
#pragma unroll
  for (int c = 0; c < NC; ++c) U[node_at(NC, c, i, N)] = up[c];
}

}  // namespace

void launch_nonreflecting(int dim, const Gas &gas, int method, int n, const int32_t *idx,
                          const double *nrm, const double *ud, int64_t N, double *U,
                          int *flags, hipStream_t s) {
  if (n <= 0) return;
  const dim3 grid((unsigned)((n + kBlock - 1) / kBlock)), block(kBlock);
  if (dim == 2)
    hipLaunchKernelGGL(k_nonreflecting<2>, grid, block, 0, s, n, idx, nrm, ud, method, gas,
                       N, U, flags);
  else
    hipLaunchKernelGGL(k_nonreflecting<3>, grid, block, 0, s, n, idx, nrm, ud, method, gas,
                       N, U, flags);
}

}  // namespace ns
