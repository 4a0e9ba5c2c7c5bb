/*
 * ns_oracle_parabolic.c -- plain CPU oracle for the parabolic (viscous)
 * sub-step and the Strang composition of arXiv:2106.02159 (Sec. 5 and
 * the parabolic-step algorithm of the appendix).
 *
 * TEST INFRASTRUCTURE ONLY (see ns_oracle.h).
 *
 * Operators are applied matrix-free, cell by cell, by tensor Gauss
 * quadrature with two points per direction on each box cell (exact for
 * every integrand below on a uniform Q1 mesh):
 *   a(v, w) = int sigma(v) : eps(w),  sigma(v) = 2 mu eps(v)
 *             + (lambda - 2/3 mu) div(v) I,  eps(v) = (grad v + grad v^T)/2
 *   b(e, w) = (kappa / c_v) int grad e . grad w
 *   K_i     = (1/m_i) int sigma(v) : eps(v) phi_i
 * The linear systems are solved by conjugate gradients preconditioned with
 * the diagonal of the operator, from the previous values, until
 * ||r||_2 <= rtol ||b||_2 (unpreconditioned residual).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "ns_oracle.h"

/* ------------------------------------------------------------------------ */
/* cells of the box mesh                                                     */
/* ------------------------------------------------------------------------ */
static const double GP[2] = {0.21132486540518711775, 0.78867513459481288225};

static void cell_counts(const orc_graph *g, long *ncell) {
  for (int d = 0; d < 3; ++d)
    ncell[d] = d < g->dim ? (g->periodic[d] ? g->n[d] : g->n[d] - 1) : 1;
}

/* global indices of the 2^dim nodes of cell kc (local node a: bit d of a
 * is the offset in direction d) */
static void cell_nodes(const orc_graph *g, const long *kc, long *gl) {
  const int nloc = 1 << g->dim;
  for (int a = 0; a < nloc; ++a) {
    long k[3] = {0, 0, 0};
    for (int d = 0; d < g->dim; ++d) k[d] = (kc[d] + ((a >> d) & 1)) % g->n[d];
    gl[a] = k[0] + g->n[0] * (k[1] + g->n[1] * k[2]);
  }
}

/* values and gradients of the 2^dim local shape functions at reference
 * point xi in [0,1]^dim of a cell with sizes h */
static void shape(int dim, const double *h, const double *xi, double *phi,
                  double grad[8][3]) {
  const int nloc = 1 << dim;
  for (int a = 0; a < nloc; ++a) {
    phi[a] = 1.0;
    for (int d = 0; d < dim; ++d) {
      const int s = (a >> d) & 1;
      phi[a] *= s ? xi[d] : 1.0 - xi[d];
    }
    for (int e = 0; e < dim; ++e) {
      double gv = (((a >> e) & 1) ? 1.0 : -1.0) / h[e];
      for (int d = 0; d < dim; ++d) {
        if (d == e) continue;
        const int s = (a >> d) & 1;
        gv *= s ? xi[d] : 1.0 - xi[d];
      }
      grad[a][e] = gv;
    }
  }
}

typedef void (*cell_fn)(const orc_graph *g, const long *gl, const double *phi,
                        double grad[8][3], double w, void *ctx);

/* calls f at every quadrature point of every cell, cells in lexicographic
 * order (serial: the callbacks scatter into node arrays) */
static void for_each_qp(const orc_graph *g, cell_fn f, void *ctx) {
  const int dim = g->dim, nloc = 1 << dim;
  long nc[3], kc[3];
  cell_counts(g, nc);
  double vol = 1.0;
  for (int d = 0; d < dim; ++d) vol *= g->h[d];
  const double w = vol / nloc;
  for (kc[2] = 0; kc[2] < nc[2]; ++kc[2])
    for (kc[1] = 0; kc[1] < nc[1]; ++kc[1])
      for (kc[0] = 0; kc[0] < nc[0]; ++kc[0]) {
        long gl[8];
        cell_nodes(g, kc, gl);
        for (int q = 0; q < nloc; ++q) {
          double xi[3], phi[8], grad[8][3];
          for (int d = 0; d < dim; ++d) xi[d] = GP[(q >> d) & 1];
          shape(dim, g->h, xi, phi, grad);
          f(g, gl, phi, grad, w, ctx);
        }
      }
}

/* sigma(v) from the velocity gradient G[k][p] = d_p v_k */
static void stress(int dim, const orc_visc *vp, double G[3][3], double S[3][3]) {
  double tr = 0.0;
  for (int k = 0; k < dim; ++k) tr += G[k][k];
  for (int k = 0; k < dim; ++k)
    for (int p = 0; p < dim; ++p) {
      const double eps = 0.5 * (G[k][p] + G[p][k]);
      S[k][p] = 2.0 * vp->mu * eps + (k == p ? (vp->lambda - 2.0 / 3.0 * vp->mu) * tr : 0.0);
    }
}

/* ------------------------------------------------------------------------ */
/* operators                                                                 */
/* ------------------------------------------------------------------------ */
struct stress_ctx {
  const orc_visc *vp;
  const double *V;
  double *Y;
};

static void stress_qp(const orc_graph *g, const long *gl, const double *phi,
                      double grad[8][3], double w, void *vctx) {
  (void)phi;
  struct stress_ctx *c = (struct stress_ctx *)vctx;
  const int dim = g->dim, nloc = 1 << dim;
  const long N = g->N;
  double G[3][3] = {{0}}, S[3][3];
  for (int a = 0; a < nloc; ++a)
    for (int k = 0; k < dim; ++k)
      for (int p = 0; p < dim; ++p) G[k][p] += c->V[(size_t)k * N + gl[a]] * grad[a][p];
  stress(dim, c->vp, G, S);
  /* a(v, phi_a e_k) = int sigma : eps(phi_a e_k) = int sum_p sigma_kp d_p phi_a */
  for (int a = 0; a < nloc; ++a)
    for (int k = 0; k < dim; ++k) {
      double s = 0.0;
      for (int p = 0; p < dim; ++p) s += S[k][p] * grad[a][p];
      c->Y[(size_t)k * N + gl[a]] += w * s;
    }
}

void orc_stress_apply(const orc_graph *g, const orc_visc *vp, const double *V,
                      double *Y) {
  memset(Y, 0, sizeof(double) * g->dim * g->N);
  struct stress_ctx c = {vp, V, Y};
  for_each_qp(g, stress_qp, &c);
}

struct heat_ctx {
  double coef;
  const double *e;
  double *Y;
};

static void heat_qp(const orc_graph *g, const long *gl, const double *phi,
                    double grad[8][3], double w, void *vctx) {
  (void)phi;
  struct heat_ctx *c = (struct heat_ctx *)vctx;
  const int dim = g->dim, nloc = 1 << dim;
  double ge[3] = {0, 0, 0};
  for (int a = 0; a < nloc; ++a)
    for (int p = 0; p < dim; ++p) ge[p] += c->e[gl[a]] * grad[a][p];
  for (int a = 0; a < nloc; ++a) {
    double s = 0.0;
    for (int p = 0; p < dim; ++p) s += ge[p] * grad[a][p];
    c->Y[gl[a]] += w * c->coef * s;
  }
}

void orc_heat_apply(const orc_graph *g, const orc_visc *vp, const double *e,
                    double *Y) {
  memset(Y, 0, sizeof(double) * g->N);
  struct heat_ctx c = {vp->kappa / vp->cv, e, Y};
  for_each_qp(g, heat_qp, &c);
}

struct diss_ctx {
  const orc_visc *vp;
  const double *V;
  double *K;
};

static void diss_qp(const orc_graph *g, const long *gl, const double *phi,
                    double grad[8][3], double w, void *vctx) {
  struct diss_ctx *c = (struct diss_ctx *)vctx;
  const int dim = g->dim, nloc = 1 << dim;
  const long N = g->N;
  double G[3][3] = {{0}}, S[3][3];
  for (int a = 0; a < nloc; ++a)
    for (int k = 0; k < dim; ++k)
      for (int p = 0; p < dim; ++p) G[k][p] += c->V[(size_t)k * N + gl[a]] * grad[a][p];
  stress(dim, c->vp, G, S);
  double se = 0.0;
  for (int k = 0; k < dim; ++k)
    for (int p = 0; p < dim; ++p) se += S[k][p] * 0.5 * (G[k][p] + G[p][k]);
  for (int a = 0; a < nloc; ++a) c->K[gl[a]] += w * se * phi[a];
}

/* K_i = (1/m_i) int sigma(v) : eps(v) phi_i (def_Ki_nplusone) */
void orc_dissipation(const orc_graph *g, const orc_visc *vp, const double *V,
                     double *K) {
  memset(K, 0, sizeof(double) * g->N);
  struct diss_ctx c = {vp, V, K};
  for_each_qp(g, diss_qp, &c);
  for (long i = 0; i < g->N; ++i) K[i] /= g->mi[i];
}

/* diagonals: a(phi_i e_k, phi_i e_k) and b(phi_i, phi_i) */
struct diag_ctx {
  const orc_visc *vp;
  double *Ad, *Bd;
};

static void diag_qp(const orc_graph *g, const long *gl, const double *phi,
                    double grad[8][3], double w, void *vctx) {
  (void)phi;
  struct diag_ctx *c = (struct diag_ctx *)vctx;
  const int dim = g->dim, nloc = 1 << dim;
  const long N = g->N;
  for (int a = 0; a < nloc; ++a) {
    double gg = 0.0;
    for (int p = 0; p < dim; ++p) gg += grad[a][p] * grad[a][p];
    c->Bd[gl[a]] += w * c->vp->kappa / c->vp->cv * gg;
    for (int k = 0; k < dim; ++k) {
      double G[3][3] = {{0}}, S[3][3];
      for (int p = 0; p < dim; ++p) G[k][p] = grad[a][p];  /* grad(phi_a e_k) */
      stress(dim, c->vp, G, S);
      double se = 0.0;
      for (int r = 0; r < dim; ++r)
        for (int p = 0; p < dim; ++p) se += S[r][p] * 0.5 * (G[r][p] + G[p][r]);
      c->Ad[(size_t)k * N + gl[a]] += w * se;
    }
  }
}

/* heat matrix entries b(phi_j, phi_i) on the graph's CSR pattern */
struct bmat_ctx {
  double coef;
  double *B;
};

static long entry(const orc_graph *g, long i, long j) {
  long lo = g->row_ptr[i], hi = g->row_ptr[i + 1] - 1;
  while (lo <= hi) {
    const long m = (lo + hi) / 2;
    if (g->col[m] == j) return m;
    if (g->col[m] < j) lo = m + 1; else hi = m - 1;
  }
  return -1;
}

static void bmat_qp(const orc_graph *g, const long *gl, const double *phi,
                    double grad[8][3], double w, void *vctx) {
  (void)phi;
  struct bmat_ctx *c = (struct bmat_ctx *)vctx;
  const int dim = g->dim, nloc = 1 << dim;
  for (int a = 0; a < nloc; ++a)
    for (int b = 0; b < nloc; ++b) {
      double s = 0.0;
      for (int p = 0; p < dim; ++p) s += grad[a][p] * grad[b][p];
      c->B[entry(g, gl[a], gl[b])] += w * c->coef * s;
    }
}

void orc_heat_matrix(const orc_graph *g, const orc_visc *vp, double *B) {
  memset(B, 0, sizeof(double) * g->nnz);
  struct bmat_ctx c = {vp->kappa / vp->cv, B};
  for_each_qp(g, bmat_qp, &c);
}

/* ------------------------------------------------------------------------ */
/* conjugate gradients with the diagonal preconditioner                      */
/* ------------------------------------------------------------------------ */
typedef void (*op_fn)(void *ctx, const double *x, double *y);

static double dot(const double *a, const double *b, long n) {
  double s = 0.0;
  for (long i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/* returns the iteration count, or -1 without convergence in maxit */
static int pcg(op_fn A, void *ctx, const double *diag, const double *b,
               double *x, long n, double rtol, int maxit) {
  double *r = (double *)malloc(sizeof(double) * n);
  double *z = (double *)malloc(sizeof(double) * n);
  double *p = (double *)malloc(sizeof(double) * n);
  double *q = (double *)malloc(sizeof(double) * n);
  const double bb = dot(b, b, n);
  if (bb == 0.0) {  /* the solution is zero */
    memset(x, 0, sizeof(double) * n);
    free(r); free(z); free(p); free(q);
    return 0;
  }
  A(ctx, x, q);
  for (long i = 0; i < n; ++i) r[i] = b[i] - q[i];
  int it = 0, ok = 0;
  double rr = dot(r, r, n);
  if (rr <= rtol * rtol * bb) ok = 1;
  for (long i = 0; i < n; ++i) z[i] = r[i] / diag[i];
  memcpy(p, z, sizeof(double) * n);
  double rz = dot(r, z, n);
  while (!ok && it < maxit) {
    A(ctx, p, q);
    const double alpha = rz / dot(p, q, n);
    for (long i = 0; i < n; ++i) {
      x[i] += alpha * p[i];
      r[i] -= alpha * q[i];
    }
    ++it;
    rr = dot(r, r, n);
    if (rr <= rtol * rtol * bb) { ok = 1; break; }
    for (long i = 0; i < n; ++i) z[i] = r[i] / diag[i];
    const double rz1 = dot(r, z, n);
    const double beta = rz1 / rz;
    rz = rz1;
    for (long i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
  }
  free(r); free(z); free(p); free(q);
  return ok ? it : -1;
}

/* velocity system: (rho_i m_i) V + dt/2 a(V, .) on free rows, identity on
 * the no-slip rows (eliminated columns: V is zero there) */
struct vel_sys {
  const orc_graph *g;
  const orc_visc *vp;
  const double *rm;        /* N: rho_i m_i */
  const unsigned char *fixed;
  double half_dt;
  double *xm, *y;          /* scratch dim*N */
};

static void vel_op(void *vctx, const double *x, double *out) {
  struct vel_sys *s = (struct vel_sys *)vctx;
  const long N = s->g->N;
  const int dim = s->g->dim;
  for (int k = 0; k < dim; ++k)
    for (long i = 0; i < N; ++i)
      s->xm[(size_t)k * N + i] = s->fixed[i] ? 0.0 : x[(size_t)k * N + i];
  orc_stress_apply(s->g, s->vp, s->xm, s->y);
  for (int k = 0; k < dim; ++k)
    for (long i = 0; i < N; ++i) {
      const size_t t = (size_t)k * N + i;
      out[t] = s->fixed[i] ? x[t] : s->rm[i] * x[t] + s->half_dt * s->y[t];
    }
}

/* energy system: (rho_i m_i) e + c dt b(e, .) (homogeneous Neumann) */
struct ene_sys {
  const orc_graph *g;
  const orc_visc *vp;
  const double *rm;
  double cdt;
  double *y;
};

static void ene_op(void *vctx, const double *x, double *out) {
  struct ene_sys *s = (struct ene_sys *)vctx;
  orc_heat_apply(s->g, s->vp, x, s->y);
  for (long i = 0; i < s->g->N; ++i) out[i] = s->rm[i] * x[i] + s->cdt * s->y[i];
}

/* ------------------------------------------------------------------------ */
/* the parabolic step (Sec. 5; parabolic-step algorithm of the appendix)     */
/* ------------------------------------------------------------------------ */
int orc_parabolic_step(const orc_graph *g, const orc_visc *vp, const double *U,
                       double dt, double *Uout, orc_par_info *info) {
  const int dim = g->dim, nc = dim + 2;
  const long N = g->N;
  const size_t dN = (size_t)dim * N;
  orc_par_info loc;
  if (!info) info = &loc;
  memset(info, 0, sizeof(*info));
  const double *rho = U;
  double *Vn = (double *)malloc(sizeof(double) * dN);
  double *Vh = (double *)malloc(sizeof(double) * dN);
  double *bv = (double *)malloc(sizeof(double) * dN);
  double *dv = (double *)malloc(sizeof(double) * dN);
  double *Ad = (double *)calloc(dN, sizeof(double));
  double *Bd = (double *)calloc(N, sizeof(double));
  double *rm = (double *)malloc(sizeof(double) * N);
  double *K = (double *)malloc(sizeof(double) * N);
  double *en = (double *)malloc(sizeof(double) * N);
  double *eh = (double *)malloc(sizeof(double) * N);
  double *eH = (double *)malloc(sizeof(double) * N);
  double *be = (double *)malloc(sizeof(double) * N);
  double *de = (double *)malloc(sizeof(double) * N);
  double *scr1 = (double *)malloc(sizeof(double) * dN);
  double *scr2 = (double *)malloc(sizeof(double) * dN);
  unsigned char *fixed = (unsigned char *)malloc(N);
  int status = 0;

  for (long i = 0; i < N; ++i) {
    rm[i] = rho[i] * g->mi[i];
    fixed[i] = (unsigned char)(g->on_wall[i] != 0);  /* no-slip walls */
  }
  for (int k = 0; k < dim; ++k)
    for (long i = 0; i < N; ++i) Vn[(size_t)k * N + i] = U[(size_t)(1 + k) * N + i] / rho[i];
  {
    struct diag_ctx c = {vp, Ad, Bd};
    for_each_qp(g, diag_qp, &c);
  }

  /* Step 1: velocity, eq. mt_parabolic_discrete with f = 0:
   * rho_i m_i V^{1/2} + dt/2 a(V^{1/2}, phi_i e_k) = m_i M^n */
  for (int k = 0; k < dim; ++k)
    for (long i = 0; i < N; ++i) {
      const size_t t = (size_t)k * N + i;
      bv[t] = fixed[i] ? 0.0 : g->mi[i] * U[(size_t)(1 + k) * N + i];
      Vh[t] = fixed[i] ? 0.0 : Vn[t];
      dv[t] = fixed[i] ? 1.0 : rm[i] + 0.5 * dt * Ad[t];
    }
  {
    struct vel_sys s = {g, vp, rm, fixed, 0.5 * dt, scr1, scr2};
    info->it_v = pcg(vel_op, &s, dv, bv, Vh, (long)dN, vp->cg_rtol, vp->cg_maxit);
    if (info->it_v < 0) status = -1;
  }
  /* eq. vel_parabolic_discrete; at no-slip nodes the prescribed value 0 */
  double *Vnew = bv;  /* reuse */
  for (int k = 0; k < dim; ++k)
    for (long i = 0; i < N; ++i) {
      const size_t t = (size_t)k * N + i;
      Vnew[t] = fixed[i] ? 0.0 : 2.0 * Vh[t] - Vn[t];
    }

  /* Step 2: K_i (def_Ki_nplusone), e^n, eq. high_int_energy_CN */
  orc_dissipation(g, vp, Vh, K);
  for (long i = 0; i < N; ++i) {
    double v2 = 0.0;
    for (int k = 0; k < dim; ++k) v2 += Vn[(size_t)k * N + i] * Vn[(size_t)k * N + i];
    en[i] = U[(size_t)(dim + 1) * N + i] / rho[i] - 0.5 * v2;
    be[i] = rm[i] * en[i] + 0.5 * dt * g->mi[i] * K[i];
    de[i] = rm[i] + 0.5 * dt * Bd[i];
    eh[i] = en[i];
  }
  {
    struct ene_sys s = {g, vp, rm, 0.5 * dt, scr1};
    info->it_e = pcg(ene_op, &s, de, be, eh, N, vp->cg_rtol, vp->cg_maxit);
    if (info->it_e < 0) status = -1;
  }
  double emin = INFINITY;
  for (long i = 0; i < N; ++i) {
    eH[i] = 2.0 * eh[i] - en[i];
    if (eH[i] < emin) emin = eH[i];
  }
  info->min_eH = emin;

  /* Step 3: limiting when the high-order internal energy is not positive
   * (or when forced): low-order backward-Euler update, eq.
   * low_order_update_internal_energy with the source dt m_i K_i, then FCT of
   * A_ij (eq. Aij_for_internal_energy) towards the local bounds
   * [min_j e^L_j, max_j e^L_j], j in I(i) */
  double *enew = eh;  /* reuse after eH is formed */
  if (vp->fct == 1 || !(emin > 0.0)) {
    info->fct = 1;
    double *eL = (double *)malloc(sizeof(double) * N);
    double *B = (double *)malloc(sizeof(double) * g->nnz);
    for (long i = 0; i < N; ++i) {
      be[i] = rm[i] * en[i] + dt * g->mi[i] * K[i];
      de[i] = rm[i] + dt * Bd[i];
      eL[i] = en[i];
    }
    struct ene_sys s = {g, vp, rm, dt, scr1};
    info->it_l = pcg(ene_op, &s, de, be, eL, N, vp->cg_rtol, vp->cg_maxit);
    if (info->it_l < 0) status = -1;
    orc_heat_matrix(g, vp, B);
    double *w = scr2;  /* w = e^H + e^n - 2 e^L */
    for (long i = 0; i < N; ++i) w[i] = eH[i] + en[i] - 2.0 * eL[i];
    double *Rp = (double *)malloc(sizeof(double) * N);
    double *Rm = (double *)malloc(sizeof(double) * N);
    for (long i = 0; i < N; ++i) {
      double Pp = 0.0, Pm = 0.0, lo = eL[i], hi = eL[i];
      for (long e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) {
        const long j = g->col[e];
        if (eL[j] < lo) lo = eL[j];
        if (eL[j] > hi) hi = eL[j];
        if (j == i) continue;
        const double A = -0.5 * dt * B[e] * (w[j] - w[i]);
        if (A > 0.0) Pp += A; else Pm += A;
      }
      const double Qp = rm[i] * (hi - eL[i]), Qm = rm[i] * (lo - eL[i]);
      Rp[i] = Pp > 0.0 ? fmin(1.0, Qp / Pp) : 1.0;
      Rm[i] = Pm < 0.0 ? fmin(1.0, Qm / Pm) : 1.0;
    }
    for (long i = 0; i < N; ++i) {
      double s = 0.0;
      for (long e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) {
        const long j = g->col[e];
        if (j == i) continue;
        const double A = -0.5 * dt * B[e] * (w[j] - w[i]);
        const double l = A > 0.0 ? fmin(Rp[i], Rm[j]) : fmin(Rm[i], Rp[j]);
        s += l * A;
      }
      enew[i] = eL[i] + s / rm[i];
    }
    free(Rp); free(Rm); free(eL); free(B);
  } else {
    memcpy(enew, eH, sizeof(double) * N);
  }

  /* eq. energy_parabolic_discrete */
  double mine = INFINITY;
  for (long i = 0; i < N; ++i) {
    double v2 = 0.0;
    Uout[i] = rho[i];
    for (int k = 0; k < dim; ++k) {
      const double v = Vnew[(size_t)k * N + i];
      Uout[(size_t)(1 + k) * N + i] = rho[i] * v;
      v2 += v * v;
    }
    Uout[(size_t)(nc - 1) * N + i] = rho[i] * enew[i] + 0.5 * rho[i] * v2;
    if (enew[i] < mine) mine = enew[i];
  }
  info->min_e = mine;
  free(Vn); free(Vh); free(bv); free(dv); free(Ad); free(Bd); free(rm);
  free(K); free(en); free(eh); free(eH); free(be); free(de); free(scr1);
  free(scr2); free(fixed);
  return status;
}

/* Strang composition (continuous_Strang): hyperbolic step with tau, parabolic
 * step with 2 tau, hyperbolic step with tau; the time advances by 2 tau. */
int orc_strang_step(const orc_graph *g, const orc_params *p, const orc_visc *vp,
                    const double *U, double tau, double *Uout,
                    orc_par_info *info) {
  const size_t len = (size_t)(g->dim + 2) * g->N;
  double *w1 = (double *)malloc(sizeof(double) * len);
  double *w2 = (double *)malloc(sizeof(double) * len);
  int st = 0;
  if (orc_ssprk3_step(g, p, U, tau, w1) != 0) st |= 1;
  if (orc_parabolic_step(g, vp, w1, 2.0 * tau, w2, info) != 0) st |= 2;
  if (orc_ssprk3_step(g, p, w2, tau, Uout) != 0) st |= 1;
  free(w1); free(w2);
  return st;
}
