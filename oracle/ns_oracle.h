/*
 * ns_oracle.h -- plain, slow CPU oracle for the explicit hyperbolic (Euler)
 * step of Guermond, Kronbichler, Maier, Popov, Tomas (arXiv:2106.02159).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link
 * or call this code: it exists so that the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark have an independent reference.  It
 * shares no source with the HIP library (its own graph assembly by Gauss
 * quadrature, its own flux, wave-speed and limiter code).
 *
 * All floating point is IEEE double.  State vectors are structure-of-arrays:
 * U[c*N + i] is component c of node i, with c = 0 density, 1..dim momentum,
 * dim+1 total energy.
 */
#ifndef NS_ORACLE_H
#define NS_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_graph {
  int dim;              /* 2 or 3 */
  long n[3];            /* nodes per direction */
  int periodic[3];      /* 1 = periodic direction */
  double lo[3], hi[3];  /* box */
  double h[3];          /* mesh size per direction */
  long N;               /* number of nodes */
  long nnz;             /* number of stencil entries (diagonal included) */
  long *row_ptr;        /* N+1 */
  long *col;            /* nnz, ascending within each row */
  long *tr;             /* nnz: position of entry (j,i) for entry (i,j) */
  double *mij;          /* nnz: consistent mass  int phi_i phi_j */
  double *cij;          /* dim*nnz: cij[k*nnz+e] = int phi_i d_k phi_j */
  double *bpair;        /* dim*nnz: int_{dOmega} phi_i phi_j n_k */
  double *mi;           /* N: lumped mass int phi_i */
  double *bnd;          /* dim*N: int_{dOmega} phi_i n_k */
  double *bface;        /* 6*N: int_{face f} phi_i over face f = 2*dir + side
                           (side 0: low end, outward normal -e_dir; side 1:
                           high end, +e_dir); 0 for periodic directions */
  int *on_wall;         /* N: 1 if the node lies on a non-periodic wall */
} orc_graph;

enum { ORC_IND_ENTROPY = 0, ORC_IND_ONE = 1, ORC_IND_ZERO = 2 };
enum { ORC_LIM_CONVEX = 0, ORC_LIM_LOW = 1, ORC_LIM_HIGH = 2 };

typedef struct orc_params {
  double gamma;
  double cfl;
  int indicator;      /* ORC_IND_* */
  int limiter;        /* ORC_LIM_* */
  int passes;         /* limiter passes for ORC_LIM_CONVEX (1 or 2) */
  double relax;       /* bound relaxation factor r0 (0 = strict bounds) */
  double volume;      /* |Omega| in the relaxation; 0 = sum of the graph's m_i
                         (a sub-mesh cut from a larger domain passes the
                         larger domain's volume) */
} orc_params;

/* Optional per-stage intermediate results (any pointer may be NULL). */
typedef struct orc_debug {
  double *d;       /* nnz: d^L_ij (diagonal holds d^L_ii) */
  double *alpha;   /* N */
  double *UL;      /* nc*N low-order update */
  double *FH;      /* nc*N high-order flux F^H_i */
  double *bounds;  /* 3*N: rho_min, rho_max, Phi_min */
  double *lt1;     /* nnz: pass-1 limiter before symmetrisation */
  double *l1;      /* nnz: pass-1 limiter after symmetrisation */
  double *lt2;     /* nnz: pass-2 limiter before symmetrisation */
  double *l2;      /* nnz */
  double *U1;      /* nc*N state after pass 1 */
} orc_debug;

int orc_graph_build(int dim, const long *n, const double *lo, const double *hi,
                    const int *periodic, orc_graph **out);
void orc_graph_free(orc_graph *g);
long orc_graph_N(const orc_graph *g);
/* Number of OpenMP threads the row loops use (1 without OpenMP). */
int orc_num_threads(void);
void orc_set_num_threads(int n);
long orc_graph_nnz(const orc_graph *g);
/* Copies the graph out into caller-owned arrays (any may be NULL). */
void orc_graph_export(const orc_graph *g, long *row_ptr, long *col, long *tr,
                      double *mij, double *cij, double *bpair, double *mi,
                      double *bnd, int *on_wall);

double orc_pressure(double gamma, int dim, const double *u);
double orc_lambda_max(double gamma, int dim, const double *ui, const double *uj,
                      const double *nij);
double orc_line_search(double gamma, int dim, const double *u, const double *P,
                       double rho_min, double rho_max, double phi_min);

/* tau = cfl * min_i(-m_i / (2 d_ii)); returns 0. */
int orc_compute_dt(const orc_graph *g, const orc_params *p, const double *U,
                   double *tau);
/* One forward-Euler stage (no boundary post-processing).  Returns 0, or 1 if
 * tau exceeds min_i(-m_i/(2 d_ii)) (the stage CFL limit at c_cfl = 1); the
 * output is computed either way. */
int orc_fe_stage(const orc_graph *g, const orc_params *p, const double *U,
                 double tau, double *Uout, orc_debug *dbg);
/* Slip post-processing at every wall node, in place. */
void orc_slip_bc(const orc_graph *g, double *U);
/* One SSPRK(3,3) step with slip post-processing after every stage.
 * Returns 0, or 1 if any stage violated its CFL limit. */
int orc_ssprk3_step(const orc_graph *g, const orc_params *p, const double *U,
                    double tau, double *Uout);
/* ---- boundary post-processing with non-reflecting faces (ns_oracle_bc.c)
 * Faces f = 2*dir + side of non-periodic directions are slip or
 * non-reflecting (Sec. 4.3).  A node lies in the slip set if some slip face
 * touches it, in the non-reflecting set if some non-reflecting face does;
 * its normal in each set is int phi_i n over that set's faces, normalised
 * (eq. def_ns_nio).  After a stage the non-reflecting post-processing runs
 * first, then the slip projection (a node in both sets keeps no normal
 * momentum through its slip faces).  A node on several non-reflecting faces
 * takes the far-field state of the lowest-numbered one. */
enum { ORC_BC_SLIP = 0, ORC_BC_NONREFLECTING = 1 };
enum { ORC_NR_CHARACTERISTIC = 0, ORC_NR_GODUNOV = 1 };
typedef struct orc_boundary {
  int kind[6];          /* per face: ORC_BC_*                              */
  int method;           /* ORC_NR_*                                        */
  double state[6][5];   /* far-field state of each non-reflecting face:    */
                        /* rho, m (dim components), E                      */
} orc_boundary;
/* Exact Riemann problem of the gamma-law gas in 1D (Sec. 4.3.1, Godunov's
 * method): star pressure by bisection on the monotone pressure function,
 * star velocity, and the solution at x/t = xi.  side_out is -1 if xi lies
 * left of the contact, +1 if right.  Returns 0, or 1 if the data generate
 * vacuum (no positive star pressure). */
int orc_riemann_star(double gamma, double rl, double ul, double pl, double rr,
                     double ur, double pr, double *pstar, double *ustar);
int orc_riemann_sample(double gamma, double rl, double ul, double pl, double rr,
                       double ur, double pr, double xi, double *rho, double *u,
                       double *p, int *side_out);
/* Post-processed state of one non-reflecting node: U, the far-field state UD
 * and the unit outward normal n (eq. Godunov_bc, or eqs. Supersonic_inflow,
 * Subsonic_inflow, Subsonic_outflow, Supersonic_outflow).  Returns 0, or 1
 * if the result is not admissible (Godunov with vacuum: then UP = U). */
int orc_nr_state(double gamma, int dim, int method, const double *U, const double *UD,
                 const double *n, double *UP);
/* Post-processing of a stage result in place; returns 0 or 1 (as above). */
int orc_boundary_bc(const orc_graph *g, const orc_params *p, const orc_boundary *b,
                    double *U);
/* One SSPRK(3,3) step with this post-processing after every stage; returns
 * bit 0 as orc_ssprk3_step, bit 1 if a post-processed state was not
 * admissible. */
int orc_ssprk3_step_bc(const orc_graph *g, const orc_params *p, const orc_boundary *b,
                       const double *U, double tau, double *Uout);

/* One SSPRK(3,3) step with the adaptive CFL number of the Remark on high
 * aspect-ratio meshes (Sec. 3.1): tau = c min_i(-m_i/(2 d_ii)) with c
 * starting at c_start (may exceed 1); the stage CFL limit is not imposed,
 * instead every stage's low-order update U^L and every stage result (after
 * the SSP combination, before the boundary post-processing) must be
 * admissible, and so must the post-processed states; if any is not, the
 * step restarts from U with c halved.  b may be NULL (slip everywhere).
 * Returns 0 with tau_out, c_out and Uout, or 1 if no c in the sequence
 * c_start 2^-k, k < 24, works. */
int orc_ssprk3_step_adaptive(const orc_graph *g, const orc_params *p,
                             const orc_boundary *b, const double *U, double c_start,
                             double *tau_out, double *c_out, double *Uout);

/* Unlimited high-order update computed directly from M_L (U^H - U) =
 * tau (I + B) F^H, used to check the limiter's l = 1 special case. */
int orc_high_order_direct(const orc_graph *g, const orc_params *p,
                          const double *U, double tau, double *UH);

/* ---- parabolic sub-step and Strang composition (ns_oracle_parabolic.c) --
 * Viscous and thermal data: sigma(v) = 2 mu eps(v) + (lambda - 2/3 mu)
 * div(v) I; the heat operator has the coefficient kappa / cv.  Walls of
 * non-periodic directions are no-slip for the velocity (all components of
 * a wall node prescribed to 0) and homogeneous Neumann for the internal
 * energy. */
typedef struct orc_visc {
  double mu, lambda, kappa, cv;
  double cg_rtol;     /* stop when ||r||_2 <= cg_rtol ||b||_2 */
  int cg_maxit;
  int fct;            /* 0: limit only if min e^H <= 0; 1: always limit */
} orc_visc;

typedef struct orc_par_info {
  int it_v, it_e, it_l;  /* CG iterations (velocity, energy, low order);
                            -1 = not converged */
  int fct;               /* 1 if the limited update was used */
  double min_eH;         /* min of the high-order internal energy */
  double min_e;          /* min of the final internal energy */
} orc_par_info;

/* Y = A V with a(v, phi_i e_k) (no boundary conditions); V, Y: dim*N */
void orc_stress_apply(const orc_graph *g, const orc_visc *vp, const double *V,
                      double *Y);
/* Y = B e with b(e, phi_i) = kappa/cv int grad e . grad phi_i */
void orc_heat_apply(const orc_graph *g, const orc_visc *vp, const double *e,
                    double *Y);
/* B_ij = b(phi_j, phi_i) on the CSR pattern (nnz) */
void orc_heat_matrix(const orc_graph *g, const orc_visc *vp, double *B);
/* K_i = (1/m_i) int sigma(v) : eps(v) phi_i */
void orc_dissipation(const orc_graph *g, const orc_visc *vp, const double *V,
                     double *K);
/* One parabolic step over dt (the Strang composition passes 2 tau).
 * Returns 0, or -1 if a CG solve did not converge. */
int orc_parabolic_step(const orc_graph *g, const orc_visc *vp, const double *U,
                       double dt, double *Uout, orc_par_info *info);
/* H(tau) P(2 tau) H(tau); returns a bit mask: 1 stage CFL violated, 2 CG
 * did not converge. */
int orc_strang_step(const orc_graph *g, const orc_params *p, const orc_visc *vp,
                    const double *U, double tau, double *Uout,
                    orc_par_info *info);

#ifdef __cplusplus
}
#endif
#endif
