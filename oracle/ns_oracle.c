/*
 * ns_oracle.c -- plain, slow CPU oracle for the explicit hyperbolic (Euler)
 * forward-Euler stage, SSPRK(3,3) and slip post-processing of
 * Guermond, Kronbichler, Maier, Popov, Tomas, arXiv:2106.02159.
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product path.
 *
 * Every function follows the paper's statement step by step, in its order
 * and notation, with no blocking, fusion or reordering:
 *   - graph quantities m_i, m_ij, c_ij           (Sec. 2.2, eq. for m_i..n_ij)
 *   - max wave speed, graph viscosity d^L_ij      (Sec. 3.1)
 *   - time step                                   (Sec. 3.1, eq. dtCfl)
 *   - bar states, low-order update, local bounds  (Sec. 3.1, eqs. bar_state,
 *                                                  loworder_bis)
 *   - high-order flux and P_ij                    (Sec. 3.2-3.3, eqs.
 *                                                  highorder, LambdaArrangement)
 *   - convex limiting, two passes                 (Sec. 3.3)
 *   - SSPRK(3,3) and slip post-processing         (Sec. 4.1-4.2, eqs. SPPRK33,
 *                                                  slip_bc)
 * Readings of points the paper leaves open (the wave-speed bound, the
 * indicator alpha_i, the line search, symmetrisation in every pass, the
 * relaxation of the limiter bounds) are restated where they are used.
 *
 * Pins (tests/test_oracle_*.py): closed-form Q1 graph values and the
 * identities of Sec. 2.2; the wave-speed bound against Toro's exact Riemann
 * solver; the closed-form time step on a periodic state at rest; Lemma 3.1's
 * balance; mass conservation by limiting; local bounds; the l = 0 and l = 1
 * special cases; the slip and global-conservation lemmas; convergence on the
 * isentropic vortex and on exact 1D Riemann problems.
 * parity unpinned: the exact value of the indicator alpha_i (a chosen
 * formula; only alpha in [0,1], alpha = 0 on constant states and alpha -> 0
 * on smooth solutions are pinned).
 *
 * Graph assembly is by 2-point-per-direction Gauss quadrature over the cells,
 * which integrates every Q1 product used here exactly.
 */
#include "ns_oracle.h"

#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Mesh and graph (Sec. 2.2)                                                 */
/* ------------------------------------------------------------------------ */

static long nidx(const orc_graph *g, const long *k) {
  return k[0] + g->n[0] * (k[1] + g->n[1] * k[2]);
}

static long find_entry(const orc_graph *g, long i, long j) {
  for (long e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e)
    if (g->col[e] == j) return e;
  return -1;
}

static int cmp_long(const void *a, const void *b) {
  long x = *(const long *)a, y = *(const long *)b;
  return (x > y) - (x < y);
}

/* value of the 1D hat factor (a = 0: 1 - xi, a = 1: xi) */
static double hat(int a, double xi) { return a ? xi : 1.0 - xi; }

/* Planes [p0, p1) along a direction of n nodes owned by the calling
   thread of an OpenMP team (all of them outside a parallel region). */
static void own_planes(long n, long *p0, long *p1) {
#ifdef _OPENMP
  const long t = omp_get_thread_num(), T = omp_get_num_threads();
#else
  const long t = 0, T = 1;
#endif
  *p0 = t * n / T;
  *p1 = (t + 1) * n / T;
}

/* Does cell layer L (nodes on planes L and L+1, wrapped) touch a plane in
   [p0, p1)? */
static int layer_touches(long L, long n, long p0, long p1) {
  const long a = L, b = (L + 1) % n;
  return (a >= p0 && a < p1) || (b >= p0 && b < p1);
}

int orc_graph_build(int dim, const long *n, const double *lo, const double *hi,
                    const int *periodic, orc_graph **out) {
  if (dim != 2 && dim != 3) return -1;
  orc_graph *g = (orc_graph *)calloc(1, sizeof(orc_graph));
  g->dim = dim;
  for (int d = 0; d < 3; ++d) {
    if (d < dim) {
      g->n[d] = n[d];
      g->periodic[d] = periodic[d];
      g->lo[d] = lo[d];
      g->hi[d] = hi[d];
      if (g->periodic[d] ? n[d] < 3 : n[d] < 2) { free(g); return -1; }
      g->h[d] = (hi[d] - lo[d]) / (double)(periodic[d] ? n[d] : n[d] - 1);
    } else {
      g->n[d] = 1; g->periodic[d] = 0; g->lo[d] = 0; g->hi[d] = 0; g->h[d] = 1;
    }
  }
  const long N = g->n[0] * g->n[1] * g->n[2];
  g->N = N;
  const int nloc = 1 << dim;
  long ncell[3];
  for (int d = 0; d < 3; ++d)
    ncell[d] = d < dim ? (g->periodic[d] ? g->n[d] : g->n[d] - 1) : 1;

  /* Every loop over cells below is split by rows: a thread owns the
     nodes of a range of planes along the last direction D and visits, in
     the order of the serial loop, only the cell layers touching them,
     writing only to its own rows.  Each row therefore receives its
     contributions in exactly the serial order (bit-identical sums). */
  const int D = dim - 1;

  /* --- sparsity: j in I(i) iff phi_i and phi_j share a cell --- */
  const int maxrow = dim == 2 ? 9 : 27;
  long *nb = (long *)malloc(sizeof(long) * N * maxrow);
  int *cnt = (int *)calloc(N, sizeof(int));
#pragma omp parallel
  {
    long p0, p1;
    own_planes(g->n[D], &p0, &p1);
    long kc[3], ka[3];
    for (kc[2] = 0; kc[2] < ncell[2]; ++kc[2])
      for (kc[1] = 0; kc[1] < ncell[1]; ++kc[1]) {
        if (!layer_touches(kc[D], g->n[D], p0, p1)) continue;
        for (kc[0] = 0; kc[0] < ncell[0]; ++kc[0]) {
          long gl[8];
          int own[8];
          for (int a = 0; a < nloc; ++a) {
            for (int d = 0; d < 3; ++d)
              ka[d] = d < dim ? (kc[d] + ((a >> d) & 1)) % g->n[d] : 0;
            gl[a] = nidx(g, ka);
            own[a] = ka[D] >= p0 && ka[D] < p1;
          }
          for (int a = 0; a < nloc; ++a) {
            if (!own[a]) continue;
            for (int b = 0; b < nloc; ++b) {
              long i = gl[a], j = gl[b];
              int found = 0;
              for (int t = 0; t < cnt[i]; ++t)
                if (nb[i * maxrow + t] == j) found = 1;
              if (!found) nb[i * maxrow + cnt[i]++] = j;
            }
          }
        }
      }
  }
  g->row_ptr = (long *)malloc(sizeof(long) * (N + 1));
  g->row_ptr[0] = 0;
  for (long i = 0; i < N; ++i) g->row_ptr[i + 1] = g->row_ptr[i] + cnt[i];
  const long nnz = g->row_ptr[N];
  g->nnz = nnz;
  g->col = (long *)malloc(sizeof(long) * nnz);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) {
    qsort(nb + i * maxrow, cnt[i], sizeof(long), cmp_long);
    memcpy(g->col + g->row_ptr[i], nb + i * maxrow, sizeof(long) * cnt[i]);
  }
  free(nb);
  free(cnt);
  g->tr = (long *)malloc(sizeof(long) * nnz);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i)
    for (long e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e)
      g->tr[e] = find_entry(g, g->col[e], i);

  g->mij = (double *)calloc(nnz, sizeof(double));
  g->cij = (double *)calloc((size_t)dim * nnz, sizeof(double));
  g->bpair = (double *)calloc((size_t)dim * nnz, sizeof(double));
  g->mi = (double *)calloc(N, sizeof(double));
  g->bnd = (double *)calloc((size_t)dim * N, sizeof(double));
  g->bface = (double *)calloc((size_t)6 * N, sizeof(double));
  g->on_wall = (int *)calloc(N, sizeof(int));

  /* --- cell integrals by tensor Gauss quadrature (2 points / direction) --- */
  const double gp[2] = {0.5 - 0.5 / sqrt(3.0), 0.5 + 0.5 / sqrt(3.0)};
  double vol = 1.0;
  for (int d = 0; d < dim; ++d) vol *= g->h[d];
  const double wq = vol / nloc; /* each of the 2^dim points */
#pragma omp parallel
  {
    long p0, p1;
    own_planes(g->n[D], &p0, &p1);
    long kc[3], ka[3];
    for (kc[2] = 0; kc[2] < ncell[2]; ++kc[2])
      for (kc[1] = 0; kc[1] < ncell[1]; ++kc[1]) {
        if (!layer_touches(kc[D], g->n[D], p0, p1)) continue;
        for (kc[0] = 0; kc[0] < ncell[0]; ++kc[0]) {
          long gl[8];
          int own[8];
          for (int a = 0; a < nloc; ++a) {
            for (int d = 0; d < 3; ++d)
              ka[d] = d < dim ? (kc[d] + ((a >> d) & 1)) % g->n[d] : 0;
            gl[a] = nidx(g, ka);
            own[a] = ka[D] >= p0 && ka[D] < p1;
          }
          /* entry of (gl[a], gl[b]) for the rows owned here, looked up once
             per cell; every sum below still runs over the quadrature points
             in order */
          long ent[8][8];
          for (int a = 0; a < nloc; ++a)
            for (int b = 0; b < nloc; ++b)
              ent[a][b] = own[a] ? find_entry(g, gl[a], gl[b]) : -1;
          for (int q = 0; q < nloc; ++q) {
            double xi[3];
            for (int d = 0; d < dim; ++d) xi[d] = gp[(q >> d) & 1];
            double phi[8], grad[8][3];
            for (int a = 0; a < nloc; ++a) {
              phi[a] = 1.0;
              for (int d = 0; d < dim; ++d) phi[a] *= hat((a >> d) & 1, xi[d]);
              for (int e = 0; e < dim; ++e) {
                double gv = (((a >> e) & 1) ? 1.0 : -1.0) / g->h[e];
                for (int d = 0; d < dim; ++d)
                  if (d != e) gv *= hat((a >> d) & 1, xi[d]);
                grad[a][e] = gv;
              }
            }
            for (int a = 0; a < nloc; ++a) {
              if (!own[a]) continue;
              g->mi[gl[a]] += wq * phi[a];
              for (int b = 0; b < nloc; ++b) {
                const long e = ent[a][b];
                g->mij[e] += wq * (phi[a] * phi[b]);
                for (int k = 0; k < dim; ++k)
                  g->cij[(size_t)k * nnz + e] += wq * phi[a] * grad[b][k];
              }
            }
          }
          /* --- boundary faces on non-periodic walls --- */
          for (int fdir = 0; fdir < dim; ++fdir) {
            if (g->periodic[fdir]) continue;
            for (int side = 0; side < 2; ++side) {
              if (side == 0 && kc[fdir] != 0) continue;
              if (side == 1 && kc[fdir] != ncell[fdir] - 1) continue;
              const double nrm = side ? 1.0 : -1.0;
              double farea = 1.0;
              for (int d = 0; d < dim; ++d)
                if (d != fdir) farea *= g->h[d];
              const int nfq = 1 << (dim - 1);
              const double wf = farea / nfq;
              for (int q = 0; q < nfq; ++q) {
                double xi[3];
                int t = 0;
                for (int d = 0; d < dim; ++d) {
                  if (d == fdir) xi[d] = (double)side;
                  else xi[d] = gp[(q >> (t++)) & 1];
                }
                double phi[8];
                for (int a = 0; a < nloc; ++a) {
                  phi[a] = 1.0;
                  for (int d = 0; d < dim; ++d) phi[a] *= hat((a >> d) & 1, xi[d]);
                }
                for (int a = 0; a < nloc; ++a) {
                  if (!own[a]) continue;
                  g->bnd[(size_t)fdir * N + gl[a]] += wf * phi[a] * nrm;
                  g->bface[(size_t)(2 * fdir + side) * N + gl[a]] += wf * phi[a];
                  for (int b = 0; b < nloc; ++b) {
                    const long e = ent[a][b];
                    g->bpair[(size_t)fdir * nnz + e] += wf * (phi[a] * phi[b]) * nrm;
                  }
                }
              }
            }
          }
        }
      }
  }
  /* wall nodes: on a face of a non-periodic direction */
  long k[3];
  for (k[2] = 0; k[2] < g->n[2]; ++k[2])
    for (k[1] = 0; k[1] < g->n[1]; ++k[1])
      for (k[0] = 0; k[0] < g->n[0]; ++k[0]) {
        int w = 0;
        for (int d = 0; d < dim; ++d)
          if (!g->periodic[d] && (k[d] == 0 || k[d] == g->n[d] - 1)) w = 1;
        g->on_wall[nidx(g, k)] = w;
      }
  *out = g;
  return 0;
}

void orc_graph_free(orc_graph *g) {
  if (!g) return;
  free(g->row_ptr); free(g->col); free(g->tr); free(g->mij); free(g->cij);
  free(g->bpair); free(g->mi); free(g->bnd); free(g->bface); free(g->on_wall); free(g);
}

long orc_graph_N(const orc_graph *g) { return g->N; }

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the following parallel loops (timing the oracle on n cores). */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
long orc_graph_nnz(const orc_graph *g) { return g->nnz; }

void orc_graph_export(const orc_graph *g, long *row_ptr, long *col, long *tr,
                      double *mij, double *cij, double *bpair, double *mi,
                      double *bnd, int *on_wall) {
  const long N = g->N, nnz = g->nnz;
  const int dim = g->dim;
  if (row_ptr) memcpy(row_ptr, g->row_ptr, sizeof(long) * (N + 1));
  if (col) memcpy(col, g->col, sizeof(long) * nnz);
  if (tr) memcpy(tr, g->tr, sizeof(long) * nnz);
  if (mij) memcpy(mij, g->mij, sizeof(double) * nnz);
  if (cij) memcpy(cij, g->cij, sizeof(double) * dim * nnz);
  if (bpair) memcpy(bpair, g->bpair, sizeof(double) * dim * nnz);
  if (mi) memcpy(mi, g->mi, sizeof(double) * N);
  if (bnd) memcpy(bnd, g->bnd, sizeof(double) * dim * N);
  if (on_wall) memcpy(on_wall, g->on_wall, sizeof(int) * N);
}

/* ------------------------------------------------------------------------ */
/* Euler model (Sec. 2.1)                                                    */
/* ------------------------------------------------------------------------ */

/* gather the nc components of node i from SoA storage */
static void load(const double *U, long N, int nc, long i, double *u) {
  for (int c = 0; c < nc; ++c) u[c] = U[(size_t)c * N + i];
}
static void store(double *U, long N, int nc, long i, const double *u) {
  for (int c = 0; c < nc; ++c) U[(size_t)c * N + i] = u[c];
}

/* internal energy per unit volume, eps = E - |m|^2 / (2 rho) */
static double internal_energy(int dim, const double *u) {
  double m2 = 0.0;
  for (int k = 0; k < dim; ++k) m2 += u[1 + k] * u[1 + k];
  return u[dim + 1] - 0.5 * m2 / u[0];
}

/* ideal gas law p = (gamma - 1) rho e = (gamma - 1) eps */
double orc_pressure(double gamma, int dim, const double *u) {
  return (gamma - 1.0) * internal_energy(dim, u);
}

/* Phi(U) = eps rho^(-gamma), the exponential of the specific entropy */
static double entropy_phi(double gamma, int dim, const double *u) {
  return internal_energy(dim, u) * pow(u[0], -gamma);
}

/* flux contracted with a vector: f(u) c = (m.c, v (m.c) + p c, v.c (E + p)) */
static void flux_dot(double gamma, int dim, const double *u, const double *c,
                     double *fc) {
  const double p = orc_pressure(gamma, dim, u);
  double vc = 0.0;
  for (int k = 0; k < dim; ++k) vc += u[1 + k] / u[0] * c[k];
  fc[0] = u[0] * vc;
  for (int k = 0; k < dim; ++k) fc[1 + k] = u[1 + k] * vc + p * c[k];
  fc[dim + 1] = vc * (u[dim + 1] + p);
}

/* ------------------------------------------------------------------------ */
/* Guaranteed upper bound on the maximum wave speed (Sec. 3.1).               */
/* Reading: the two-rarefaction bound on the intermediate pressure, valid     */
/* for 1 < gamma <= 5/3, inserted in the extreme wave speeds of the 1D        */
/* Riemann problem along n with left state ui and right state uj.             */
/* ------------------------------------------------------------------------ */
double orc_lambda_max(double gamma, int dim, const double *ui, const double *uj,
                      const double *nij) {
  const double rhoL = ui[0], rhoR = uj[0];
  double uL = 0.0, uR = 0.0;
  for (int k = 0; k < dim; ++k) {
    uL += ui[1 + k] / rhoL * nij[k];
    uR += uj[1 + k] / rhoR * nij[k];
  }
  const double pL = orc_pressure(gamma, dim, ui);
  const double pR = orc_pressure(gamma, dim, uj);
  const double aL = sqrt(gamma * pL / rhoL);
  const double aR = sqrt(gamma * pR / rhoR);
  const double ex = (gamma - 1.0) / (2.0 * gamma);
  const double num = aL + aR - 0.5 * (gamma - 1.0) * (uR - uL);
  double ptr = 0.0;
  if (num > 0.0) {
    const double den = aL * pow(pL, -ex) + aR * pow(pR, -ex);
    ptr = pow(num / den, 1.0 / ex);
  }
  const double cg = (gamma + 1.0) / (2.0 * gamma);
  const double lam1 = uL - aL * sqrt(1.0 + cg * fmax(ptr / pL - 1.0, 0.0));
  const double lam3 = uR + aR * sqrt(1.0 + cg * fmax(ptr / pR - 1.0, 0.0));
  return fmax(fmax(-lam1, 0.0), fmax(lam3, 0.0));
}

/* ------------------------------------------------------------------------ */
/* Limiter line search (Sec. 3.3).                                            */
/* Largest l in [0,1] with rho_min <= rho(u + l P) <= rho_max and             */
/* Phi(u + l P) >= Phi_min.  Density is affine in l; for the entropy the      */
/* function psi(l) = eps(u + l P) - Phi_min rho(u + l P)^gamma is concave, so */
/* its feasible set is an interval; the root is found by plain bisection.     */
/* ------------------------------------------------------------------------ */
static double psi_at(double gamma, int dim, const double *u, const double *P,
                     double l, double phi_min) {
  double s[5];
  for (int c = 0; c < dim + 2; ++c) s[c] = u[c] + l * P[c];
  return internal_energy(dim, s) - phi_min * pow(s[0], gamma);
}

double orc_line_search(double gamma, int dim, const double *u, const double *P,
                       double rho_min, double rho_max, double phi_min) {
  double lr;
  if (P[0] > 0.0) lr = (rho_max - u[0]) / P[0];
  else if (P[0] < 0.0) lr = (rho_min - u[0]) / P[0];
  else lr = 1.0;
  if (lr > 1.0) lr = 1.0;
  if (lr < 0.0) lr = 0.0;
  if (psi_at(gamma, dim, u, P, lr, phi_min) >= 0.0) return lr;
  if (psi_at(gamma, dim, u, P, 0.0, phi_min) < 0.0) return 0.0;
  double a = 0.0, b = lr;
  for (int it = 0; it < 80; ++it) {
    const double m = 0.5 * (a + b);
    if (m <= a || m >= b) break; /* interval at round-off resolution */
    if (psi_at(gamma, dim, u, P, m, phi_min) >= 0.0) a = m;
    else b = m;
  }
  return a;
}

/* ------------------------------------------------------------------------ */
/* Graph viscosity (Sec. 3.1): d_ij = max(lambda(Ui,Uj,n_ij)|c_ij|,          */
/* lambda(Uj,Ui,n_ji)|c_ji|), d_ii = -sum_{j != i} d_ij.                      */
/* ------------------------------------------------------------------------ */
static void graph_viscosity(const orc_graph *g, double gamma, const double *U,
                            double *d) {
  const int dim = g->dim, nc = dim + 2;
  const long N = g->N, nnz = g->nnz;
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) {
    double ui[5];
    load(U, N, nc, i, ui);
    long ediag = -1;
    double dsum = 0.0;
    for (long e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) {
      const long j = g->col[e];
      if (j == i) { ediag = e; continue; }
      double uj[5], cij[3], cji[3], nij[3], nji[3];
      load(U, N, nc, j, uj);
      double ncij = 0.0, ncji = 0.0;
      for (int k = 0; k < dim; ++k) {
        cij[k] = g->cij[(size_t)k * nnz + e];
        cji[k] = g->cij[(size_t)k * nnz + g->tr[e]];
        ncij += cij[k] * cij[k];
        ncji += cji[k] * cji[k];
      }
      ncij = sqrt(ncij);
      ncji = sqrt(ncji);
      for (int k = 0; k < dim; ++k) {
        nij[k] = cij[k] / ncij;
        nji[k] = cji[k] / ncji;
      }
      const double a = orc_lambda_max(gamma, dim, ui, uj, nij) * ncij;
      const double b = orc_lambda_max(gamma, dim, uj, ui, nji) * ncji;
      d[e] = fmax(a, b);
      dsum += d[e];
    }
    d[ediag] = -dsum;
  }
}

int orc_compute_dt(const orc_graph *g, const orc_params *p, const double *U,
                   double *tau) {
  double *d = (double *)malloc(sizeof(double) * g->nnz);
  graph_viscosity(g, p->gamma, U, d);
  double t = INFINITY;
#pragma omp parallel for reduction(min : t)
  for (long i = 0; i < g->N; ++i) {
    const long e = find_entry(g, i, i);
    const double r = -g->mi[i] / (2.0 * d[e]);
    if (r < t) t = r;
  }
  free(d);
  *tau = p->cfl * t;
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Entropy-production indicator alpha_i (Sec. 3.2).                           */
/* Reading: normalised entropy-viscosity commutator.  With the mathematical   */
/* entropy eta = -rho s, s = ln(eps rho^-gamma), entropy flux F = v eta,      */
/* t_ij = F(U_j).c_ij - eta'(U_i).(f(U_j) c_ij), N_i = sum t_ij,              */
/* D_i = sum |t_ij|, S_i = sum |c_ij| a_j (rho_j + |eta_j|) (a = sound speed), */
/* alpha_i = |N_i| / (D_i + 1e-2 S_i).  Every t_ij vanishes with the velocity, */
/* so without the acoustic-flux floor S_i alpha would be a ratio of round-off */
/* noise wherever the gas is (nearly) at rest; alpha stays in [0, 1).          */
/* ------------------------------------------------------------------------ */
static void indicator(const orc_graph *g, const orc_params *p, const double *U,
                      double *alpha) {
  const int dim = g->dim, nc = dim + 2;
  const long N = g->N, nnz = g->nnz;
  const double gamma = p->gamma;
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) {
    if (p->indicator == ORC_IND_ONE) { alpha[i] = 1.0; continue; }
    if (p->indicator == ORC_IND_ZERO) { alpha[i] = 0.0; continue; }
    double ui[5];
    load(U, N, nc, i, ui);
    const double epsi = internal_energy(dim, ui);
    const double si = log(epsi * pow(ui[0], -gamma));
    double m2 = 0.0;
    for (int k = 0; k < dim; ++k) m2 += ui[1 + k] * ui[1 + k];
    double etap[5];
    etap[0] = gamma - si - m2 / (2.0 * ui[0] * epsi);
    for (int k = 0; k < dim; ++k) etap[1 + k] = ui[1 + k] / epsi;
    etap[dim + 1] = -ui[0] / epsi;
    double num = 0.0, den = 0.0, scale = 0.0;
    for (long e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) {
      const long j = g->col[e];
      double uj[5], c[3], fc[5];
      load(U, N, nc, j, uj);
      for (int k = 0; k < dim; ++k) c[k] = g->cij[(size_t)k * nnz + e];
      const double sj = log(internal_energy(dim, uj) * pow(uj[0], -gamma));
      const double etaj = -uj[0] * sj;
      double vc = 0.0;
      for (int k = 0; k < dim; ++k) vc += uj[1 + k] / uj[0] * c[k];
      flux_dot(gamma, dim, uj, c, fc);
      double t = etaj * vc;
      for (int q = 0; q < nc; ++q) t -= etap[q] * fc[q];
      num += t;
      den += fabs(t);
      double cn = 0.0;
      for (int k = 0; k < dim; ++k) cn += c[k] * c[k];
      const double aj = sqrt(gamma * orc_pressure(gamma, dim, uj) / uj[0]);
      scale += sqrt(cn) * aj * (uj[0] + fabs(etaj));
    }
    alpha[i] = fabs(num) / (den + 1e-2 * scale);
  }
}

/* ------------------------------------------------------------------------ */
/* One forward-Euler stage (Algorithm 1, Sec. 3).                             */
/* ------------------------------------------------------------------------ */
int orc_fe_stage(const orc_graph *g, const orc_params *p, const double *U,
                 double tau, double *Uout, orc_debug *dbg) {
  const int dim = g->dim, nc = dim + 2;
  const long N = g->N, nnz = g->nnz;
  const double gamma = p->gamma;
  int status = 0;

  double *d = (double *)malloc(sizeof(double) * nnz);
  double *alpha = (double *)malloc(sizeof(double) * N);
  double *UL = (double *)malloc(sizeof(double) * nc * N);
  double *FH = (double *)malloc(sizeof(double) * nc * N);
  double *bounds = (double *)malloc(sizeof(double) * 3 * N);
  double *P = (double *)calloc((size_t)nc * nnz, sizeof(double));
  double *lt = (double *)calloc(nnz, sizeof(double));
  double *l = (double *)calloc(nnz, sizeof(double));
  double *Ucur = (double *)malloc(sizeof(double) * nc * N);
  double *Unew = (double *)malloc(sizeof(double) * nc * N);

  /* Step 1-2: graph viscosity, d_ii, stage CFL check, indicator */
  graph_viscosity(g, gamma, U, d);
#pragma omp parallel for reduction(| : status)
  for (long i = 0; i < N; ++i) {
    const long e = find_entry(g, i, i);
    if (tau > -g->mi[i] / (2.0 * d[e])) status = 1;
  }
  indicator(g, p, U, alpha);

  /* Step 3: bar states, low-order update, local bounds, high-order flux */
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) {
    double ui[5], sum[5] = {0, 0, 0, 0, 0}, fh[5] = {0, 0, 0, 0, 0};
    load(U, N, nc, i, ui);
    double rho_min = INFINITY, rho_max = -INFINITY, phi_min = INFINITY;
    for (long e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) {
      const long j = g->col[e];
      double uj[5], c[3], fi[5], fj[5], ubar[5];
      load(U, N, nc, j, uj);
      for (int k = 0; k < dim; ++k) c[k] = g->cij[(size_t)k * nnz + e];
      flux_dot(gamma, dim, ui, c, fi);
      flux_dot(gamma, dim, uj, c, fj);
      if (j == i) {
        for (int q = 0; q < nc; ++q) ubar[q] = ui[q];
      } else {
        for (int q = 0; q < nc; ++q)
          ubar[q] = 0.5 * (ui[q] + uj[q]) - (fj[q] - fi[q]) / (2.0 * d[e]);
      }
      for (int q = 0; q < nc; ++q) sum[q] += d[e] * ubar[q];
      if (ubar[0] < rho_min) rho_min = ubar[0];
      if (ubar[0] > rho_max) rho_max = ubar[0];
      const double phij = entropy_phi(gamma, dim, uj);
      if (phij < phi_min) phi_min = phij;
      const double dH = 0.5 * (alpha[i] + alpha[j]) * d[e];
      for (int q = 0; q < nc; ++q) fh[q] += -fj[q] + dH * (uj[q] - ui[q]);
    }
    double ul[5];
    for (int q = 0; q < nc; ++q) ul[q] = ui[q] + 2.0 * tau / g->mi[i] * sum[q];
    store(UL, N, nc, i, ul);
    store(FH, N, nc, i, fh);
    bounds[i] = rho_min;
    bounds[N + i] = rho_max;
    bounds[2 * N + i] = phi_min;
  }

  /* Step 4: P_ij = tau/(m_i lambda_i) (b_ij F_j - b_ji F_i + (dH - dL)(Uj - Ui)) */
#pragma omp parallel for schedule(static)
  for (long i = 0; i < N; ++i) {
    const long nrow = g->row_ptr[i + 1] - g->row_ptr[i];
    const double lambda_i = 1.0 / (double)(nrow - 1);
    double ui[5], fi[5];
    load(U, N, nc, i, ui);
    load(FH, N, nc, i, fi);
    for (long e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) {
      const long j = g->col[e];
      if (j == i) continue;
      double uj[5], fj[5];
      load(U, N, nc, j, uj);
      load(FH, N, nc, j, fj);
      const double bij = -g->mij[e] / g->mi[j];
      const double bji = -g->mij[g->tr[e]] / g->mi[i];
      const double dH = 0.5 * (alpha[i] + alpha[j]) * d[e];
      for (int q = 0; q < nc; ++q)
        P[(size_t)q * nnz + e] =
            tau / (g->mi[i] * lambda_i) *
            (bij * fj[q] - bji * fi[q] + (dH - d[e]) * (uj[q] - ui[q]));
    }
  }

  /* Relaxed bounds used by the line search: rho in [(1-r_i) rho_min,
   * (1+r_i) rho_max], Phi >= (1-r_i) Phi_min with r_i = r0 (m_i/|Omega|)^(3/(2d)). */
  double *rb = (double *)malloc(sizeof(double) * 3 * N);
  {
    double vol = 0.0;
    for (long i = 0; i < N; ++i) vol += g->mi[i];
    if (p->volume > 0.0) vol = p->volume;
    for (long i = 0; i < N; ++i) {
      const double r = p->relax * pow(g->mi[i] / vol, 1.5 / dim);
      rb[i] = (1.0 - r) * bounds[i];
      rb[N + i] = (1.0 + r) * bounds[N + i];
      rb[2 * N + i] = (1.0 - r) * bounds[2 * N + i];
    }
  }

  /* Steps 5-6: limiting, U = U^L + sum_j lambda_i l_ij P_ij */
  memcpy(Ucur, UL, sizeof(double) * nc * N);
  if (p->limiter == ORC_LIM_HIGH) {
    for (long e = 0; e < nnz; ++e) l[e] = 1.0;
  }
  const int npass = p->limiter == ORC_LIM_CONVEX ? p->passes
                    : p->limiter == ORC_LIM_HIGH ? 1 : 0;
  for (int pass = 0; pass < npass; ++pass) {
    if (p->limiter == ORC_LIM_CONVEX) {
#pragma omp parallel for schedule(dynamic, 256)
      for (long i = 0; i < N; ++i) {
        double ui[5];
        load(Ucur, N, nc, i, ui);
        for (long e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) {
          if (g->col[e] == i) { lt[e] = 0.0; continue; }
          double pe[5];
          for (int q = 0; q < nc; ++q) pe[q] = P[(size_t)q * nnz + e];
          lt[e] = orc_line_search(gamma, dim, ui, pe, rb[i], rb[N + i],
                                  rb[2 * N + i]);
        }
      }
      /* symmetrise (in every pass): l_ij = min(l~_ij, l~_ji) */
      for (long e = 0; e < nnz; ++e) l[e] = fmin(lt[e], lt[g->tr[e]]);
      if (dbg) {
        double *dl = pass == 0 ? dbg->lt1 : dbg->lt2;
        double *dls = pass == 0 ? dbg->l1 : dbg->l2;
        if (dl) memcpy(dl, lt, sizeof(double) * nnz);
        if (dls) memcpy(dls, l, sizeof(double) * nnz);
      }
    }
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; ++i) {
      const long nrow = g->row_ptr[i + 1] - g->row_ptr[i];
      const double lambda_i = 1.0 / (double)(nrow - 1);
      double u[5];
      load(Ucur, N, nc, i, u);
      for (long e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) {
        if (g->col[e] == i) continue;
        for (int q = 0; q < nc; ++q)
          u[q] += lambda_i * l[e] * P[(size_t)q * nnz + e];
      }
      store(Unew, N, nc, i, u);
    }
    /* next pass: U^L <- the limited state, P_ij <- (1 - l_ij) P_ij */
    for (long e = 0; e < nnz; ++e)
      for (int q = 0; q < nc; ++q) P[(size_t)q * nnz + e] *= (1.0 - l[e]);
    memcpy(Ucur, Unew, sizeof(double) * nc * N);
    if (pass == 0 && dbg && dbg->U1)
      memcpy(dbg->U1, Ucur, sizeof(double) * nc * N);
  }
  memcpy(Uout, Ucur, sizeof(double) * nc * N);

  if (dbg) {
    if (dbg->d) memcpy(dbg->d, d, sizeof(double) * nnz);
    if (dbg->alpha) memcpy(dbg->alpha, alpha, sizeof(double) * N);
    if (dbg->UL) memcpy(dbg->UL, UL, sizeof(double) * nc * N);
    if (dbg->FH) memcpy(dbg->FH, FH, sizeof(double) * nc * N);
    if (dbg->bounds) memcpy(dbg->bounds, bounds, sizeof(double) * 3 * N);
  }
  free(d); free(alpha); free(UL); free(FH); free(bounds); free(rb); free(P); free(lt);
  free(l); free(Ucur); free(Unew);
  return status;
}

/* ------------------------------------------------------------------------ */
/* Slip post-processing (Sec. 4.2, eq. slip_bc): M <- M - (M.n_i) n_i with    */
/* n_i = int phi_i n / |int phi_i n| at every wall node.                      */
/* ------------------------------------------------------------------------ */
void orc_slip_bc(const orc_graph *g, double *U) {
  const int dim = g->dim;
  const long N = g->N;
  for (long i = 0; i < N; ++i) {
    if (!g->on_wall[i]) continue;
    double nv[3], nn = 0.0;
    for (int k = 0; k < dim; ++k) {
      nv[k] = g->bnd[(size_t)k * N + i];
      nn += nv[k] * nv[k];
    }
    nn = sqrt(nn);
    double mn = 0.0;
    for (int k = 0; k < dim; ++k) {
      nv[k] /= nn;
      mn += U[(size_t)(1 + k) * N + i] * nv[k];
    }
    for (int k = 0; k < dim; ++k) U[(size_t)(1 + k) * N + i] -= mn * nv[k];
  }
}

/* ------------------------------------------------------------------------ */
/* SSPRK(3,3) (Sec. 4.1, eq. SPPRK33) with post-processing after each stage.  */
/* ------------------------------------------------------------------------ */
int orc_ssprk3_step(const orc_graph *g, const orc_params *p, const double *U,
                    double tau, double *Uout) {
  const int nc = g->dim + 2;
  const size_t len = (size_t)nc * g->N;
  double *w1 = (double *)malloc(sizeof(double) * len);
  double *w2 = (double *)malloc(sizeof(double) * len);
  double *t = (double *)malloc(sizeof(double) * len);
  int st = 0;
  st |= orc_fe_stage(g, p, U, tau, w1, NULL);
  orc_slip_bc(g, w1);
  st |= orc_fe_stage(g, p, w1, tau, t, NULL);
  for (size_t k = 0; k < len; ++k) w2[k] = 0.75 * U[k] + 0.25 * t[k];
  orc_slip_bc(g, w2);
  st |= orc_fe_stage(g, p, w2, tau, t, NULL);
  for (size_t k = 0; k < len; ++k) Uout[k] = U[k] / 3.0 + 2.0 / 3.0 * t[k];
  orc_slip_bc(g, Uout);
  free(w1); free(w2); free(t);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Unlimited high-order update straight from eq. highorderCompact:            */
/* M_L (U^H - U) = tau (I + B) F^H with b_ij = delta_ij - m_ij / m_j.         */
/* ------------------------------------------------------------------------ */
int orc_high_order_direct(const orc_graph *g, const orc_params *p,
                          const double *U, double tau, double *UH) {
  const int dim = g->dim, nc = dim + 2;
  const long N = g->N;
  orc_params q = *p;
  q.limiter = ORC_LIM_LOW;
  double *FH = (double *)malloc(sizeof(double) * nc * N);
  double *tmp = (double *)malloc(sizeof(double) * nc * N);
  orc_debug dbg;
  memset(&dbg, 0, sizeof(dbg));
  dbg.FH = FH;
  orc_fe_stage(g, &q, U, tau, tmp, &dbg);
  for (long i = 0; i < N; ++i) {
    double acc[5];
    load(FH, N, nc, i, acc);
    for (long e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e) {
      const long j = g->col[e];
      const double bij = (j == i ? 1.0 : 0.0) - g->mij[e] / g->mi[j];
      for (int c = 0; c < nc; ++c) acc[c] += bij * FH[(size_t)c * N + j];
    }
    for (int c = 0; c < nc; ++c)
      UH[(size_t)c * N + i] = U[(size_t)c * N + i] + tau / g->mi[i] * acc[c];
  }
  (void)dim;
  free(FH); free(tmp);
  return 0;
}
