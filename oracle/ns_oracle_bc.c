/*
 * ns_oracle_bc.c -- boundary post-processing of the oracle with slip and
 * non-reflecting faces (Sec. 4.3: eqs. slip_bc, Godunov_bc,
 * Supersonic_inflow, Subsonic_inflow, Subsonic_outflow, Supersonic_outflow,
 * normals of eq. def_ns_nio).
 *
 * TEST INFRASTRUCTURE ONLY (see ns_oracle.h).  The exact Riemann solver
 * finds the star pressure by bisection on the monotone pressure function,
 * so that its result can be trusted without a convergence argument.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "ns_oracle.h"

/* Pressure function of one side of the Riemann problem, gamma-law gas:
 * the Rankine-Hugoniot branch for p above the side's pressure (a shock),
 * the isentropic branch below it (a rarefaction).  Increasing in p. */
static double side_fn(double g, double p, double rk, double pk) {
  if (p > pk) {
    const double A = 2.0 / ((g + 1.0) * rk);
    const double B = (g - 1.0) / (g + 1.0) * pk;
    return (p - pk) * sqrt(A / (p + B));
  }
  const double ak = sqrt(g * pk / rk);
  return 2.0 * ak / (g - 1.0) * (pow(p / pk, (g - 1.0) / (2.0 * g)) - 1.0);
}

int orc_riemann_star(double g, double rl, double ul, double pl, double rr,
                     double ur, double pr, double *pstar, double *ustar) {
  const double du = ur - ul;
  const double al = sqrt(g * pl / rl), ar = sqrt(g * pr / rr);
  /* f(0) = -2 (a_l + a_r) / (gamma - 1) + du: no positive root if >= 0 */
  if (2.0 * (al + ar) / (g - 1.0) <= du) return 1;
  double lo = 0.0, hi = pl > pr ? pl : pr;
  while (side_fn(g, hi, rl, pl) + side_fn(g, hi, rr, pr) + du < 0.0) hi *= 2.0;
  for (int it = 0; it < 2000; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi)) break;
    if (side_fn(g, mid, rl, pl) + side_fn(g, mid, rr, pr) + du < 0.0) lo = mid;
    else hi = mid;
  }
  const double p = 0.5 * (lo + hi);
  *pstar = p;
  *ustar = 0.5 * (ul + ur) + 0.5 * (side_fn(g, p, rr, pr) - side_fn(g, p, rl, pl));
  return 0;
}

int orc_riemann_sample(double g, double rl, double ul, double pl, double rr,
                       double ur, double pr, double xi, double *rho, double *u,
                       double *p, int *side_out) {
  double ps, us;
  if (orc_riemann_star(g, rl, ul, pl, rr, ur, pr, &ps, &us)) return 1;
  const double gm = (g - 1.0) / (g + 1.0);
  if (xi <= us) {  /* left of the contact */
    *side_out = -1;
    const double al = sqrt(g * pl / rl);
    if (ps > pl) {  /* left shock */
      const double sl = ul - al * sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g));
      if (xi <= sl) { *rho = rl; *u = ul; *p = pl; }
      else { *rho = rl * (ps / pl + gm) / (gm * ps / pl + 1.0); *u = us; *p = ps; }
    } else {        /* left rarefaction */
      const double head = ul - al;
      const double tail = us - al * pow(ps / pl, (g - 1.0) / (2.0 * g));
      if (xi <= head) { *rho = rl; *u = ul; *p = pl; }
      else if (xi >= tail) { *rho = rl * pow(ps / pl, 1.0 / g); *u = us; *p = ps; }
      else {
        const double c = 2.0 / (g + 1.0) + (g - 1.0) / ((g + 1.0) * al) * (ul - xi);
        *rho = rl * pow(c, 2.0 / (g - 1.0));
        *u = 2.0 / (g + 1.0) * (al + 0.5 * (g - 1.0) * ul + xi);
        *p = pl * pow(c, 2.0 * g / (g - 1.0));
      }
    }
  } else {         /* right of the contact */
    *side_out = 1;
    const double ar = sqrt(g * pr / rr);
    if (ps > pr) {  /* right shock */
      const double sr = ur + ar * sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g));
      if (xi >= sr) { *rho = rr; *u = ur; *p = pr; }
      else { *rho = rr * (ps / pr + gm) / (gm * ps / pr + 1.0); *u = us; *p = ps; }
    } else {        /* right rarefaction */
      const double head = ur + ar;
      const double tail = us + ar * pow(ps / pr, (g - 1.0) / (2.0 * g));
      if (xi >= head) { *rho = rr; *u = ur; *p = pr; }
      else if (xi <= tail) { *rho = rr * pow(ps / pr, 1.0 / g); *u = us; *p = ps; }
      else {
        const double c = 2.0 / (g + 1.0) - (g - 1.0) / ((g + 1.0) * ar) * (ur - xi);
        *rho = rr * pow(c, 2.0 / (g - 1.0));
        *u = 2.0 / (g + 1.0) * (-ar + 0.5 * (g - 1.0) * ur + xi);
        *p = pr * pow(c, 2.0 * g / (g - 1.0));
      }
    }
  }
  return 0;
}

/* density, velocity, normal velocity, tangential velocity, pressure, sound
 * speed of a conserved state along the unit normal n */
typedef struct prim {
  double rho, v[3], vn, vt[3], p, a;
} prim;

static prim primitives(double g, int dim, const double *U, const double *n) {
  prim q;
  q.rho = U[0];
  double m2 = 0.0;
  q.vn = 0.0;
  for (int k = 0; k < dim; ++k) {
    q.v[k] = U[1 + k] / q.rho;
    m2 += U[1 + k] * U[1 + k];
    q.vn += q.v[k] * n[k];
  }
  for (int k = 0; k < dim; ++k) q.vt[k] = q.v[k] - q.vn * n[k];
  q.p = (g - 1.0) * (U[dim + 1] - 0.5 * m2 / q.rho);
  q.a = sqrt(g * q.p / q.rho);
  return q;
}

/* conserved state from density, normal and tangential velocity, pressure */
static void conserved(double g, int dim, double rho, double un, const double *vt,
                      double p, const double *n, double *UP) {
  double m2 = 0.0;
  UP[0] = rho;
  for (int k = 0; k < dim; ++k) {
    UP[1 + k] = rho * (vt[k] + un * n[k]);
    m2 += UP[1 + k] * UP[1 + k];
  }
  UP[dim + 1] = p / (g - 1.0) + 0.5 * m2 / rho;
}

int orc_nr_state(double g, int dim, int method, const double *U, const double *UD,
                 const double *n, double *UP) {
  const int nc = dim + 2;
  const prim q = primitives(g, dim, U, n), d = primitives(g, dim, UD, n);
  if (method == ORC_NR_GODUNOV) {
    /* Riemann problem along n: the node's state on the left (inside), the
       far-field state on the right; its solution at x = 0 */
    double rho, un, p;
    int side;
    if (orc_riemann_sample(g, q.rho, q.vn, q.p, d.rho, d.vn, d.p, 0.0, &rho, &un, &p,
                           &side)) {
      memcpy(UP, U, sizeof(double) * nc);  /* vacuum: the state is kept, flagged */
      return 1;
    }
    conserved(g, dim, rho, un, side < 0 ? q.vt : d.vt, p, n, UP);
  } else {
    if (q.vn < 0.0 && q.a < fabs(q.vn)) {           /* supersonic inflow */
      memcpy(UP, UD, sizeof(double) * nc);
      return 0;
    }
    if (q.vn >= 0.0 && q.a <= fabs(q.vn)) {         /* supersonic outflow */
      memcpy(UP, U, sizeof(double) * nc);
      return 0;
    }
    /* subsonic: C1 from the far field, C3 from the node; S and the
       tangential velocity from the far field (inflow) or the node (outflow) */
    const int inflow = q.vn < 0.0;
    const double C1 = d.vn - 2.0 * d.a / (g - 1.0);
    const double C3 = q.vn + 2.0 * q.a / (g - 1.0);
    const double S = inflow ? d.p * pow(d.rho, -g) : q.p * pow(q.rho, -g);
    const double un = 0.5 * (C1 + C3);
    const double aP = 0.25 * (g - 1.0) * (C3 - C1);
    const double rho = pow(aP * aP / (g * S), 1.0 / (g - 1.0));
    const double p = S * pow(rho, g);
    conserved(g, dim, rho, un, inflow ? d.vt : q.vt, p, n, UP);
  }
  double m2 = 0.0;
  for (int k = 0; k < dim; ++k) m2 += UP[1 + k] * UP[1 + k];
  return (UP[0] > 0.0 && UP[dim + 1] - 0.5 * m2 / UP[0] > 0.0) ? 0 : 1;
}

/* normal of node i over the faces of one kind (0 if none touches it) */
static double kind_normal(const orc_graph *g, const orc_boundary *b, int kind, long i,
                          double *n, int *first_face) {
  double nn = 0.0;
  *first_face = -1;
  for (int k = 0; k < g->dim; ++k) n[k] = 0.0;
  for (int f = 0; f < 2 * g->dim; ++f) {
    const double w = g->bface[(size_t)f * g->N + i];
    if (b->kind[f] != kind || w == 0.0) continue;
    if (*first_face < 0) *first_face = f;
    n[f / 2] += (f % 2 ? 1.0 : -1.0) * w;
  }
  for (int k = 0; k < g->dim; ++k) nn += n[k] * n[k];
  nn = sqrt(nn);
  if (nn > 0.0)
    for (int k = 0; k < g->dim; ++k) n[k] /= nn;
  return nn;
}

int orc_boundary_bc(const orc_graph *g, const orc_params *p, const orc_boundary *b,
                    double *U) {
  const int dim = g->dim, nc = dim + 2;
  const long N = g->N;
  int bad = 0;
  for (long i = 0; i < N; ++i) {  /* non-reflecting nodes */
    double n[3], u[5], up[5];
    int f;
    if (kind_normal(g, b, ORC_BC_NONREFLECTING, i, n, &f) == 0.0) continue;
    for (int c = 0; c < nc; ++c) u[c] = U[(size_t)c * N + i];
    bad |= orc_nr_state(p->gamma, dim, b->method, u, b->state[f], n, up);
    for (int c = 0; c < nc; ++c) U[(size_t)c * N + i] = up[c];
  }
  for (long i = 0; i < N; ++i) {  /* slip nodes (eq. slip_bc) */
    double n[3], mn = 0.0;
    int f;
    if (kind_normal(g, b, ORC_BC_SLIP, i, n, &f) == 0.0) continue;
    for (int k = 0; k < dim; ++k) mn += U[(size_t)(1 + k) * N + i] * n[k];
    for (int k = 0; k < dim; ++k) U[(size_t)(1 + k) * N + i] -= mn * n[k];
  }
  return bad;
}

int orc_ssprk3_step_bc(const orc_graph *g, const orc_params *p, const orc_boundary *b,
                       const double *U, double tau, double *Uout) {
  const int nc = g->dim + 2;
  const size_t len = (size_t)nc * g->N;
  double *w1 = (double *)malloc(sizeof(double) * len);
  double *w2 = (double *)malloc(sizeof(double) * len);
  double *t = (double *)malloc(sizeof(double) * len);
  int st = 0, bad = 0;
  st |= orc_fe_stage(g, p, U, tau, w1, NULL);
  bad |= orc_boundary_bc(g, p, b, w1);
  st |= orc_fe_stage(g, p, w1, tau, t, NULL);
  for (size_t k = 0; k < len; ++k) w2[k] = 0.75 * U[k] + 0.25 * t[k];
  bad |= orc_boundary_bc(g, p, b, w2);
  st |= orc_fe_stage(g, p, w2, tau, t, NULL);
  for (size_t k = 0; k < len; ++k) Uout[k] = U[k] / 3.0 + 2.0 / 3.0 * t[k];
  bad |= orc_boundary_bc(g, p, b, Uout);
  free(w1); free(w2); free(t);
  return st | (bad << 1);
}

/* admissible: rho > 0 and internal energy > 0 at every node */
static int all_admissible(int dim, long N, const double *U) {
  for (long i = 0; i < N; ++i) {
    double m2 = 0.0;
    for (int k = 0; k < dim; ++k) m2 += U[(size_t)(1 + k) * N + i] * U[(size_t)(1 + k) * N + i];
    const double rho = U[i], e = U[(size_t)(dim + 1) * N + i] - 0.5 * m2 / rho;
    if (!(rho > 0.0) || !(e > 0.0)) return 0;
  }
  return 1;
}

static int post(const orc_graph *g, const orc_params *p, const orc_boundary *b, double *U) {
  if (b) return orc_boundary_bc(g, p, b, U);
  orc_slip_bc(g, U);
  return 0;
}

int orc_ssprk3_step_adaptive(const orc_graph *g, const orc_params *p,
                             const orc_boundary *b, const double *U, double c_start,
                             double *tau_out, double *c_out, double *Uout) {
  const int dim = g->dim, nc = dim + 2;
  const long N = g->N;
  const size_t len = (size_t)nc * N;
  double *w1 = (double *)malloc(sizeof(double) * len);
  double *w2 = (double *)malloc(sizeof(double) * len);
  double *t = (double *)malloc(sizeof(double) * len);
  double *UL = (double *)malloc(sizeof(double) * len);
  orc_debug dbg;
  memset(&dbg, 0, sizeof(dbg));
  dbg.UL = UL;
  int done = 0;
  double c = c_start;
  for (int k = 0; k < 24 && !done; ++k, c *= 0.5) {
    orc_params q = *p;
    q.cfl = c;
    double tau;
    orc_compute_dt(g, &q, U, &tau);
    int ok = 1;
    /* stage 1 */
    orc_fe_stage(g, &q, U, tau, w1, &dbg);
    ok = ok && all_admissible(dim, N, UL) && all_admissible(dim, N, w1);
    ok = ok && !post(g, &q, b, w1);
    /* stage 2 */
    if (ok) {
      orc_fe_stage(g, &q, w1, tau, t, &dbg);
      for (size_t e = 0; e < len; ++e) w2[e] = 0.75 * U[e] + 0.25 * t[e];
      ok = all_admissible(dim, N, UL) && all_admissible(dim, N, w2) && !post(g, &q, b, w2);
    }
    /* stage 3 */
    if (ok) {
      orc_fe_stage(g, &q, w2, tau, t, &dbg);
      for (size_t e = 0; e < len; ++e) Uout[e] = U[e] / 3.0 + 2.0 / 3.0 * t[e];
      ok = all_admissible(dim, N, UL) && all_admissible(dim, N, Uout) &&
           !post(g, &q, b, Uout);
    }
    if (ok) {
      *tau_out = tau;
      *c_out = c;
      done = 1;
    }
  }
  free(w1); free(w2); free(t); free(UL);
  return done ? 0 : 1;
}
