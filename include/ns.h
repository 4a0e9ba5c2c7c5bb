/*
 * ns.h -- C ABI of libns: the explicit hyperbolic (Euler) step of
 * Guermond, Kronbichler, Maier, Popov, Tomas, "On the implementation of a
 * robust and efficient finite element-based parallel solver for the
 * compressible Navier-Stokes equations" (arXiv:2106.02159), on AMD MI355X.
 *
 * Scope: continuous Q1 elements on uniform box meshes (2D quadrilaterals,
 * 3D hexahedra), ideal-gas Euler flux, graph viscosity from a guaranteed
 * maximum wave speed, low-order update, local bounds, high-order flux with
 * the approximate inverse mass matrix, convex limiting (Sec. 3, Algorithm 1),
 * SSPRK(3,3) with slip post-processing after every stage (Sec. 4.1-4.2) or
 * non-reflecting post-processing on chosen faces (Sec. 4.3), the adaptive
 * CFL number of the Remark on high aspect-ratio meshes; the parabolic
 * (viscous) sub-step with matrix-free conjugate gradients (diagonal or
 * single-precision multigrid preconditioner) and the Strang composition of
 * the Navier-Stokes step (Sec. 2, Sec. 5); FP32 storage of the
 * bandwidth-bound arrays; asynchronous stepping, packs of meshes advanced by
 * shared launches and a server for many independent simulations.
 *
 * Conventions shared by every call:
 *   - Status codes: NS_OK (0) or a negative NS_E* value.  No call throws.
 *   - A state is structure-of-arrays double precision: U[c*N + i] is
 *     component c of node i; c = 0 density rho, 1..dim momentum m,
 *     dim+1 total energy E; nc = dim+2 components.  (On the device the
 *     library keeps node vectors with components 2p and 2p+1 of a node side
 *     by side; the state and debug calls convert, host buffers on the host,
 *     device buffers by a kernel on the solver's stream.)
 *   - Nodes are numbered lexicographically, x fastest:
 *     i = ix + nx*(iy + ny*iz).
 *   - All device work of a solver is ordered on one HIP stream.  Calls on
 *     one solver must not overlap (one solver per host thread).
 *   - Host buffers passed in are read or written before the call returns;
 *     device buffers (flag NS_ON_DEVICE) must be hipMalloc'ed on the
 *     solver's device and hold nc*N doubles.
 */
#ifndef NS_H
#define NS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define NS_OK 0
#define NS_EINVAL (-1)          /* bad argument                              */
#define NS_ENOMEM (-2)          /* device or host allocation failed          */
#define NS_EHIP (-3)            /* a HIP runtime call failed                 */
#define NS_ENOTADMISSIBLE (-4)  /* a state has rho <= 0, eps <= 0 or a NaN   */
#define NS_ECFL (-5)            /* dt above the stage CFL limit (c_cfl = 1)  */
#define NS_EBOUNDS (-6)         /* a stage produced an inadmissible state    */
#define NS_ESTATE (-7)          /* no state has been set                     */
#define NS_ECG (-8)             /* a CG solve of the parabolic step did not
                                   converge within its iteration limit      */
#define NS_EABORT (-9)          /* persistent steps gave up waiting (wait
                                   limit reached or give-up word set): the
                                   state is undefined until a new one is set */

/* ---- options ------------------------------------------------------------ */
/* Entropy-production indicator alpha_i of Sec. 3.2 (d^H_ij = (alpha_i +
 * alpha_j)/2 d^L_ij): the entropy-viscosity commutator, or the constants
 * alpha = 1 (d^H = d^L) and alpha = 0 (d^H = 0). */
enum { NS_IND_ENTROPY = 0, NS_IND_ONE = 1, NS_IND_ZERO = 2 };
/* Limiter of Sec. 3.3: convex limiting; l = 0 (returns the low-order update
 * U^L of eq. loworder); l = 1 (returns the unlimited high-order update of
 * eq. highorderCompact). */
enum { NS_LIM_CONVEX = 0, NS_LIM_LOW = 1, NS_LIM_HIGH = 2 };

/* set_state / get_state flags */
#define NS_ON_DEVICE 1   /* the buffer is a device pointer                    */
#define NS_NO_PROJECT 2  /* set_state: skip the slip projection of wall nodes */

/* ---- mesh and graph (Sec. 2.2) ----------------------------------------- */
/* Uniform box mesh.  n[d] counts nodes in direction d.  A periodic direction
 * has mesh size (hi-lo)/n and needs n >= 3; a direction bounded by walls has
 * mesh size (hi-lo)/(n-1) and needs n >= 2.  Every non-periodic face is a
 * slip (reflecting) wall for the hyperbolic step (Sec. 4.2, eq. slip_bc)
 * unless ns_set_boundary makes it non-reflecting. */
typedef struct ns_mesh_desc {
  int dim;          /* 2 or 3 */
  int64_t n[3];     /* nodes per direction (n[2] ignored when dim == 2) */
  double lo[3];
  double hi[3];
  int periodic[3];  /* nonzero = periodic */
} ns_mesh_desc;

typedef struct ns_graph ns_graph;

/* Builds the stencil graph I(i) of the Q1 space and the quantities of
 * Sec. 2.2: m_i = int phi_i, m_ij = int phi_i phi_j, c_ij = int phi_i
 * grad phi_j, and the boundary integrals int_{dOmega} phi_i n used for the
 * slip normals (eq. unit_normal_vector).  The library owns the graph (host
 * memory); it must outlive every solver created from it.
 * Errors: NS_EINVAL for dim not in {2,3}, n below the limits above, lo >= hi,
 * more than 2^31-1 nodes, or a NULL pointer; NS_ENOMEM. */
int ns_graph_create(const ns_mesh_desc *mesh, ns_graph **out);
void ns_graph_destroy(ns_graph *g);

/* Sizes of the graph: N nodes, nnz stencil entries (diagonal included),
 * spatial dimension and the row width W = 3^dim of its ELL storage. */
int ns_graph_info(const ns_graph *g, int64_t *n_nodes, int64_t *nnz, int *dim,
                  int *width);

/* Copies the graph into caller-owned host arrays in slot-major ELL layout:
 * entry (slot k, node i) sits at index k*N + i, k < W.  Missing entries
 * (rows shorter than W at walls) have col = -1 and zero coefficients.
 * col: W*N int32; mij: W*N; cij: dim*W*N (component-major, cij[(d*W+k)*N+i]);
 * mi: N; bnd: dim*N (int_{dOmega} phi_i n_d).  Any pointer may be NULL. */
int ns_graph_export(const ns_graph *g, int32_t *col, double *mij, double *cij,
                    double *mi, double *bnd);

/* ---- solver ------------------------------------------------------------ */
typedef struct ns_params {
  double gamma;   /* ratio of specific heats, 1 < gamma <= 5/3            */
  double cfl;     /* c_cfl of eq. dtCfl, 0 < cfl <= 1                      */
  int indicator;  /* NS_IND_*                                              */
  int limiter;    /* NS_LIM_*                                              */
  int passes;     /* limiter passes for NS_LIM_CONVEX: 1 or 2 (paper: 2)   */
  double relax;   /* bound relaxation r0 >= 0: the line search accepts
                     rho in [(1-r_i) rho_min, (1+r_i) rho_max] and
                     Phi >= (1-r_i) Phi_min, r_i = r0 (m_i/|Omega|)^(3/(2d));
                     0 = the strict bounds of Sec. 3.3                      */
  int precision;  /* NS_PREC_FP64, NS_PREC_MIXED_FP32 (below), or
                     NS_PREC_MIXED: the intermediates
                     alpha_i, d^L_ij, F^H_i and the limiter coefficients are
                     stored in FP32 (d_ij rounded up, so it stays an upper
                     bound of the wave-speed term; limiter coefficients
                     rounded down, so they stay feasible); the state, the
                     bounds, the line search and all arithmetic stay FP64
                     (m_ij and c_ij are computed, never stored)             */
} ns_params;

/* NS_PREC_MIXED_FP32: the storage of NS_PREC_MIXED, and the graph-viscosity
 * sweep (Sec. 3.1, 3.2) evaluated in FP32 for gamma = 7/5: the normal
 * velocities, pressures, |c_ij|, lambda_max and the entropy indicator.
 * lambda_max is used only where its FP32 rounding error is certified below
 * 2^-16 relative (no cancellation beyond fixed factors), and is then
 * inflated by 2^-16 and rounded up, so d^L_ij stays an upper bound; on the
 * other entries it is evaluated in FP64.  Every stage re-checks U^L of every
 * row in FP64 (rho > 0, internal energy > 0); a synchronous step whose
 * re-check fails is redone from the unchanged state in FP64 arithmetic
 * (counted in ns_stats_t.fp64_redo), an asynchronous one reports
 * NS_EBOUNDS; persistent steps are not offered (NS_EINVAL).  Other gamma:
 * as NS_PREC_MIXED.  The limiter, the bounds, the line search and the state
 * stay FP64. */
enum { NS_PREC_FP64 = 0, NS_PREC_MIXED = 1, NS_PREC_MIXED_FP32 = 2 };

typedef struct ns_solver ns_solver;

/* Creates a solver on the current HIP device.  `stream` is a hipStream_t to
 * order all work on, or NULL for a stream the solver creates and owns.  All
 * device memory (per-node graph data -- m_i, 1/m_i, |I(i)| - 1, r_i, wall
 * flags; the column indices, m_ij and c_ij are computed in the kernels from
 * the box mesh -- three state buffers, per-edge d_ij and limiter arrays,
 * per-node scratch, the limiter's root work lists) is allocated here.
 * Errors: NS_EINVAL for bad parameters or a mesh whose edge count (width x
 * N rounded up to 64) exceeds 2^32 - 1; NS_ENOMEM if the device footprint
 * does not fit; NS_EHIP. */
int ns_solver_create(const ns_graph *g, const ns_params *p, void *stream,
                     ns_solver **out);
void ns_solver_destroy(ns_solver *s);

/* Device bytes ns_solver_create would allocate for this graph and these
 * parameters (without ns_set_viscous); equals ns_device_bytes of the
 * created solver.  Used to admit work by memory footprint. */
int ns_solver_footprint(const ns_graph *g, const ns_params *p, int64_t *bytes);

/* Copies a state in (host or, with NS_ON_DEVICE, device buffer of nc*N
 * doubles).  The state is checked: NS_ENOTADMISSIBLE if any rho <= 0,
 * eps = E - |m|^2/(2 rho) <= 0 or a value is not finite (ns_last_error
 * names the first such node), and the previous state is kept.  Unless
 * NS_NO_PROJECT is given the momentum of every wall node is projected on
 * the wall (eq. slip_bc), so that the initial data satisfy the slip
 * condition that the global-conservation lemma assumes. */
int ns_set_state(ns_solver *s, const double *U, int flags);

/* Copies the current state out (stream-ordered, synchronous). */
int ns_get_state(ns_solver *s, double *U, int flags);

/* tau = c_cfl * min_i(-m_i / (2 d^L_ii)) for the current state (Sec. 3.1,
 * eq. dtCfl).  Synchronous; NS_ESTATE without a state. */
int ns_compute_dt(ns_solver *s, double *dt);

/* One SSPRK(3,3) step of size dt (Sec. 4.1, eq. SPPRK33): three
 * forward-Euler stages with the same dt, each followed by the SSP
 * combination and the slip post-processing.  Transactional: on any error
 * the state is left unchanged.  NS_ECFL if dt exceeds min_i(-m_i/(2 d_ii))
 * (the stage limit at c_cfl = 1) in any stage -- the caller restarts with a
 * smaller dt; NS_EBOUNDS if a stage produced an inadmissible state. */
int ns_step(ns_solver *s, double dt);

/* Same, with dt = c_cfl * min_i(-m_i/(2 d_ii)) computed on the device in the
 * first stage from that stage's own d_ij and reused by stages 2 and 3
 * (Sec. 3.1).  The dt used is returned in *dt (may be NULL). */
int ns_step_cfl(ns_solver *s, double *dt);
/* One SSPRK(3,3) step with the adaptive CFL number of the Remark on high
 * aspect-ratio meshes (Sec. 3.1): dt = c min_i(-m_i/(2 d_ii)) with c
 * starting at c_start (0 < c_start <= 64; above 1 is the point), the stage
 * CFL limit not imposed; instead every stage's low-order update U^L and
 * every stage result must be admissible (and the boundary post-processing
 * must succeed), else the step restarts from the same state with c halved.
 * Transactional; *dt and *c_used (either may be NULL) report the accepted
 * step.  NS_EBOUNDS if no c_start / 2^k, k < 24, works. */
int ns_step_adaptive(ns_solver *s, double c_start, double *dt, double *c_used);

/* ---- parabolic sub-step and Strang composition (Sec. 5) ----------------
 * Viscous and thermal data of the Navier-Stokes system: the viscous stress
 * sigma(v) = 2 mu eps(v) + (lambda - 2/3 mu) div(v) I, eps(v) the symmetric
 * velocity gradient, and the heat flux -(kappa/cv) grad e.  In the parabolic
 * step every wall node (non-periodic face) is no-slip for the velocity (its
 * velocity is prescribed to 0 at both time levels) and the internal energy
 * satisfies homogeneous Neumann conditions (thermally insulated walls).
 * The two linear systems are solved by conjugate gradients preconditioned
 * as `precond` selects, started from the values at t^n and stopped when
 * ||r||_2 <= cg_rtol ||b||_2 (unpreconditioned residual). */
enum { NS_FCT_AUTO = 0, NS_FCT_ALWAYS = 1 };
typedef struct ns_viscous {
  double mu;       /* shear viscosity, >= 0                                 */
  double lambda;   /* bulk viscosity, >= 0                                  */
  double kappa;    /* thermal conductivity, >= 0                            */
  double cv;       /* heat capacity at constant volume, > 0                 */
  double cg_rtol;  /* relative residual of both CG solves, in (0, 1)        */
  int cg_maxit;    /* iteration limit of each CG solve, >= 1                */
  int fct;         /* NS_FCT_AUTO: limit the internal energy only when the
                      Crank-Nicolson value is not positive somewhere;
                      NS_FCT_ALWAYS: always (tests)                         */
  int precond;     /* NS_PC_JACOBI: diagonal preconditioner;
                      NS_PC_GMG: geometric multigrid V-cycle in FP32 with a
                      Chebyshev(3)-Jacobi smoother (the viscous-dominated
                      regime); coarse levels halve the cells of every
                      direction (rounded up; non-nested interpolation) down
                      to about 512 nodes                                    */
} ns_viscous;
enum { NS_PC_JACOBI = 0, NS_PC_GMG = 1 };

/* Enables the parabolic step: validates the data, builds the Q1 element
 * matrices of the stress and heat operators and allocates the CG vectors
 * (about 7 dim N + 8 N doubles; with NS_PC_GMG about 4 dim N doubles
 * more for the FP32 levels) and a fourth state buffer that keeps Strang
 * steps transactional.  May be called again to change the data; the
 * multigrid levels are built once and their element tables redone.
 * NS_EINVAL for a NULL pointer or data out of range; NS_ENOMEM. */
int ns_set_viscous(ns_solver *s, const ns_viscous *v);

/* One parabolic step of size dt from the current state (the
 * parabolic-step algorithm of the appendix): density unchanged; velocity
 * by Crank-Nicolson, eq. mt_parabolic_discrete (f = 0) and
 * vel_parabolic_discrete; K_i of eq. def_Ki_nplusone from V^{n+1/2};
 * internal energy by Crank-Nicolson, eq. high_int_energy_CN; if the
 * resulting internal energy is not positive somewhere (or with
 * NS_FCT_ALWAYS), the low-order backward-Euler energy with source
 * dt m_i K_i and flux-corrected limiting of A_ij (eq. Aij_for_internal_energy)
 * towards the local bounds [min_j e^L_j, max_j e^L_j]; total energy by eq.
 * energy_parabolic_discrete.  Transactional.  NS_ESTATE without
 * ns_set_viscous or a state; NS_ECG if a CG solve did not converge;
 * NS_EBOUNDS if the result is not admissible. */
int ns_step_parabolic(ns_solver *s, double dt);

/* One Strang step (eq. continuous_Strang): SSPRK(3,3) step with tau,
 * parabolic step with 2 tau, SSPRK(3,3) step with tau; time advances by
 * 2 tau.  The second hyperbolic step reuses tau and checks the stage CFL
 * limit in all its stages.  Transactional: on any error the state at the
 * start is restored. */
int ns_step_strang(ns_solver *s, double tau);
/* Same, tau computed on the device in the first stage of the first
 * hyperbolic step (returned in *tau, may be NULL). */
int ns_step_strang_cfl(ns_solver *s, double *tau);

typedef struct ns_par_info {
  int it_v, it_e, it_l;  /* CG iterations: velocity, energy, low-order energy
                            (0 when the limiting was not needed)            */
  int fct;               /* 1 if the limited internal energy was used       */
  double min_eH;         /* minimum of the Crank-Nicolson internal energy   */
} ns_par_info;
/* Diagnostics of the last parabolic step. */
int ns_parabolic_info(ns_solver *s, ns_par_info *out);

/* ---- boundary kinds: slip and non-reflecting faces ----------------------
 * Every face of a non-periodic direction (f = 2*dir + side: side 0 the low
 * end with outward normal -e_dir, side 1 the high end) is slip (the
 * default: eq. slip_bc) or non-reflecting (Sec. 4.3) with a far-field
 * (Dirichlet) state: post-processing by the characteristic variables (eqs.
 * Supersonic_inflow, Subsonic_inflow, Subsonic_outflow, Supersonic_outflow)
 * or by Godunov's method (eq. Godunov_bc, the exact Riemann solution at the
 * boundary).  A node belongs to the slip set if a slip face touches it and
 * to the non-reflecting set if a non-reflecting face does; its normal in
 * each set is the normalised integral of phi_i n over that set's faces (eq.
 * def_ns_nio).  After every stage the non-reflecting nodes are post-processed
 * first, then the slip nodes (a node in both keeps no normal momentum
 * through its slip faces); a node on several non-reflecting faces takes the
 * far-field state of the lowest-numbered one.  An inadmissible result
 * (Godunov with vacuum) keeps the node's state and the step returns
 * NS_EBOUNDS.  Non-reflecting faces are for the Euler step: with any,
 * ns_step_parabolic and the Strang steps return NS_ESTATE.  NS_EINVAL for
 * unknown kinds or methods, a non-admissible far-field state, or one that
 * violates (gamma-1)/2 v_n^D <= a^D on its face (the Lemma's condition). */
enum { NS_BC_SLIP = 0, NS_BC_NONREFLECTING = 1 };
enum { NS_NR_CHARACTERISTIC = 0, NS_NR_GODUNOV = 1 };
typedef struct ns_boundary {
  int kind[6];         /* per face: NS_BC_*; faces of periodic directions   */
                       /* and beyond dim are ignored                        */
  int method;          /* NS_NR_*                                           */
  double state[6][5];  /* far-field state per non-reflecting face: rho,     */
                       /* m (dim components), E                             */
} ns_boundary;
int ns_set_boundary(ns_solver *s, const ns_boundary *b);

/* ---- asynchronous stepping (serving) ------------------------------------
 * ns_step_cfl_async enqueues nsteps SSPRK(3,3) steps, each with its own CFL
 * time step computed on the device as in ns_step_cfl, and returns without
 * waiting for the device.  The status of all steps enqueued since the last
 * ns_async_finish is kept on the device (sticky): the steps are not
 * transactional -- after a failure the state is that of the failed run.
 * ns_query tells without blocking whether the enqueued work has finished;
 * ns_async_finish waits for it and returns NS_OK, NS_ECFL or NS_EBOUNDS for
 * the whole run and the time advanced (sum of the steps' dt) in *t. */
int ns_step_cfl_async(ns_solver *s, int nsteps);
int ns_query(ns_solver *s, int *done);
/* Number of ns_step_cfl_async calls whose steps have not all finished. */
int ns_inflight(ns_solver *s, int *calls);
int ns_async_finish(ns_solver *s, double *t);

/* Persistent steps: as ns_step_cfl_async, but the nsteps SSPRK(3,3) steps
 * (each with its CFL time step, eq. dtCfl, computed on the device) run as ONE
 * kernel launch instead of about 30 launches per step.  The launch's
 * workgroups stay resident and take work items -- (step, stage, phase,
 * member, row block) -- in order from a counter; the phases of a stage are
 * the sweeps of Algorithm 1 (node precompute, graph viscosity and time
 * step, low-order update and bounds, the two limiter passes with their
 * root work lists, final update, slip projection of Sec. 4.2).  An item runs
 * once its member has finished the earlier phases (a completion counter per
 * member), so each member of a pack moves through the stage on its own.
 * Results are bit-identical to those of ns_step_cfl_async (same per-row
 * arithmetic, same time steps).  Every wait of the kernel is bounded: by
 * wait_s seconds of the device's wall clock (> 0), and by the give-up word
 * that ns_cancel sets; a wait that ends either way stops the whole launch
 * (every workgroup exits at its next item), later launches of the run stop
 * as well, and ns_async_finish / ns_pack_finish report NS_EABORT (the state
 * is then undefined until ns_set_state / ns_pack_set_state).  Needs
 * NS_IND_ENTROPY, NS_LIM_CONVEX with 2 passes and no non-reflecting nodes
 * (else NS_EINVAL); NS_ENOMEM if no give-up word is left (one per solver,
 * 1024 per process, in pinned host memory).  Status, time and completion
 * are those of ns_step_cfl_async (ns_query, ns_inflight, ns_async_finish);
 * both kinds of call may be mixed in one run. */
int ns_step_cfl_persistent(ns_solver *s, int nsteps, double wait_s);
/* Sets the solver's give-up word: its persistent launches in flight stop at
 * their next wait or item (a run's first call clears the word). */
int ns_cancel(ns_solver *s);

/* ---- packs: several meshes advanced by the same kernel launches ---------
 * A pack holds `count` independent problems (graphs of one dimension) in one
 * solver.  Every member's rows start at a 256-row workgroup boundary (the
 * rows up to the next member are isolated padding nodes holding a constant
 * state), so each workgroup belongs to one member; the CFL time step, the
 * CFL and admissibility status and the time advanced are per member.  One
 * ns_pack_step_cfl_async call enqueues nsteps SSPRK(3,3) steps of all
 * members, each step with each member's own CFL time step.  A member's
 * result is bit-identical to that of its own solver stepped with
 * ns_step_cfl: the kernels see the same rows, neighbours and time steps.
 * For serving many small meshes, whose own launches would leave most of
 * the device idle.  Parameters as ns_solver_create (NS_EINVAL also for
 * count < 1 or graphs of different dimensions). */
typedef struct ns_pack ns_pack;
int ns_pack_footprint(const ns_graph *const *graphs, int count, const ns_params *p,
                      int64_t *bytes);
int ns_pack_create(const ns_graph *const *graphs, int count, const ns_params *p,
                   void *hip_stream, ns_pack **out);
/* Waits for the pack's work and frees it. */
void ns_pack_destroy(ns_pack *k);
/* State of member r from host memory (nc*N_r doubles, SoA): checked
 * (NS_ENOTADMISSIBLE) and its wall nodes projected, as ns_set_state.  Every
 * member needs a state before the first step. */
int ns_pack_set_state(ns_pack *k, int r, const double *U);
/* State of member r into host memory; waits for the enqueued steps. */
int ns_pack_get_state(ns_pack *k, int r, double *U);
/* As ns_step_cfl_async / ns_inflight, for all members. */
int ns_pack_step_cfl_async(ns_pack *k, int nsteps);
int ns_pack_inflight(ns_pack *k, int *calls);
/* Waits for the enqueued steps; for every member r, status[r] (NS_OK,
 * NS_ECFL or NS_EBOUNDS, sticky since the last finish) and t[r] (time
 * advanced since then).  Returns NS_OK, or NS_EHIP if the device failed. */
int ns_pack_finish(ns_pack *k, int *status, double *t);
/* As ns_step_cfl_persistent / ns_cancel, for all members (status NS_EABORT
 * for every member of a run that gave up). */
int ns_pack_step_cfl_persistent(ns_pack *k, int nsteps, double wait_s);
int ns_pack_cancel(ns_pack *k);
const char *ns_pack_error(const ns_pack *k);

/* ---- serving: continuous batching of independent simulations ------------
 * A server holds a FIFO queue of requests (uniform-mesh Euler problems: mesh,
 * initial state, number of SSPRK(3,3) steps with the CFL time step).
 * Requests are admitted in order as units: a request whose mesh has at most
 * pack_nodes / 2 rows (N rounded up to 256) is packed (ns_pack_*) with the
 * consecutive queued requests of the same step count and dimension, up to
 * pack_nodes rows and pack_max members; any other request gets its own
 * solver.  A unit is admitted when its device footprint (ns_pack_footprint,
 * ns_solver_footprint) fits in mem_bytes beside the running ones and fewer
 * than max_running units are running; it runs on its own HIP stream; its
 * steps are enqueued in chunks of `chunk` steps, at most `depth` chunks in
 * flight, one new chunk per unit per progress call (round robin), so
 * running units advance together and overlap on the device.
 * ns_server_progress never blocks on the device: it tops up the running
 * units' chunks, collects finished units (their states are copied to host
 * memory and their device memory freed) and admits queued requests.  A
 * request's result depends only on its input (deterministic kernels, no
 * shared device data, pack members bit-identical to their own solvers): it
 * is bit-identical alone and in any mix. */
typedef struct ns_server ns_server;
typedef struct ns_server_params {
  int64_t mem_bytes;  /* device memory the running requests may use        */
  int max_running;    /* running units (solvers or packs) at most, >= 1    */
  int chunk;          /* steps per enqueued chunk, >= 1                    */
  int depth;          /* chunks in flight per unit, >= 1                   */
  ns_params solver;   /* parameters of every request's solver              */
  int64_t pack_nodes; /* rows of a pack at most (meshes rounded up to 256  */
                      /* rows; 0: every request gets its own solver)       */
  int pack_max;       /* members of a pack at most, >= 2 with packs        */
  int64_t persistent_rows; /* units (solvers or packs) of at most this many
                              rows are stepped by persistent launches
                              (ns_step_cfl_persistent, one launch per
                              chunk, 10 s wait limit); larger ones by
                              ns_step_cfl_async; 0: none                  */
} ns_server_params;
enum { NS_REQ_QUEUED = 0, NS_REQ_RUNNING = 1, NS_REQ_FINISHED = 2 };
typedef struct ns_request_info {
  int state;          /* NS_REQ_*                                          */
  int status;         /* status of a finished request (NS_OK, NS_ECFL...)  */
  int steps;
  int64_t bytes;      /* device footprint                                  */
  int64_t n_nodes;
  double t_submit, t_admit, t_finish;  /* host steady clock, seconds       */
  double t_sim;       /* simulated time reached (sum of the steps' dt)     */
} ns_request_info;
typedef struct ns_server_stats {
  int64_t submitted, finished, queued, running;
  int64_t peak_running, peak_bytes, bytes_in_use;
  int64_t units;                        /* units admitted (solvers + packs)  */
  double host_admit_s, host_topup_s, host_finish_s;  /* host time spent in */
                                        /* admissions, top-ups, collections  */
} ns_server_stats;

/* NS_EINVAL for bad parameters. */
int ns_server_create(const ns_server_params *p, ns_server **out);
/* Waits for running requests, frees everything. */
void ns_server_destroy(ns_server *sv);
/* Queues a request; U0 (host, nc*N doubles for the mesh's N) is copied.
 * NS_EINVAL for a bad mesh, NS_ENOTADMISSIBLE for a state with rho <= 0,
 * internal energy <= 0 or a non-finite value, NS_ENOMEM if the request
 * alone exceeds mem_bytes.  *id identifies the request.  A unit whose
 * set-up fails (device memory, a HIP error) finishes all its requests with
 * that status. */
int ns_server_submit(ns_server *sv, const ns_mesh_desc *mesh, const double *U0,
                     int steps, int64_t *id);
/* Collects finished requests and admits queued ones; *n_finished (may be
 * NULL) is the number of requests that finished in this call. */
int ns_server_progress(ns_server *sv, int *n_finished);
/* State and timing of a request (until its result is taken). */
int ns_server_request(ns_server *sv, int64_t id, ns_request_info *info);
/* Copies the final state of a finished request into U (host) and forgets
 * the request; returns the request's status, NS_ESTATE if it has not
 * finished, NS_EINVAL for an unknown id. */
int ns_server_result(ns_server *sv, int64_t id, double *U);
int ns_server_stats_get(const ns_server *sv, ns_server_stats *out);
/* Error message of a request, or of the last failed submit (id <= 0). */
const char *ns_server_error(const ns_server *sv, int64_t id);

/* Test access: one forward-Euler stage of size dt from the current state,
 * without SSP combination or post-processing; the result and every
 * intermediate are kept for ns_get_debug and the state is not changed.
 * Returns NS_ECFL (after computing everything) if dt exceeds the stage
 * limit, like the step. */
int ns_fe_stage(ns_solver *s, double dt);

/* Test access: the stencil entries as the kernels derive them from the box
 * mesh (no graph array is stored on the device), for the mesh placed at row
 * `base` of a solver and followed by padding rows up to base + rows - 1
 * (rows >= N; padding rows are isolated nodes: only their diagonal entry,
 * with m_ii = 1 and c_ii = 0).  Host-only.  Layout as ns_graph_export with
 * `rows` in place of N: col W*rows int32, entry (slot k, row base + r) at
 * k*rows + r, -1 where absent; slot k holds the neighbour at offset
 * (dx,dy,dz), k = (dx+1) + 3(dy+1) + 9(dz+1), and the transposed entry of
 * (i, k) is (col, W-1-k); mij W*rows; cij dim*W*rows, component-major.  The
 * coefficients of absent entries are unspecified.  Any output may be NULL.
 * NS_EINVAL for rows < N, a negative base or base + rows > 2^31 - 1. */
int ns_graph_stencil(const ns_graph *g, int64_t base, int64_t rows, int32_t *col,
                     double *mij, double *cij);

/* Intermediates of the last stage run (ns_fe_stage, or the last stage of
 * the last step).  Edge arrays use the ELL layout of ns_graph_export. */
enum {
  NS_DBG_STAGE_OUT = 0, /* nc*N   stage result                            */
  NS_DBG_D = 1,         /* W*N    d^L_ij (off-diagonal entries)           */
  NS_DBG_ALPHA = 2,     /* N      alpha_i                                 */
  NS_DBG_UL = 3,        /* nc*N   low-order update U^L                    */
  NS_DBG_FH = 4,        /* nc*N   high-order flux F^H_i divided by m_i    */
  NS_DBG_BOUNDS = 5,    /* 3*N    relaxed rho_min, rho_max, Phi_min       */
  NS_DBG_LT1 = 6,       /* W*N    pass-1 limiter before symmetrisation    */
  NS_DBG_LT2 = 7,       /* W*N    pass-2 limiter before symmetrisation,
                                  times (1 - l_ij), l_ij the symmetric pass-1
                                  limiter                                 */
  NS_DBG_U1 = 8,        /* nc*N   state after limiter pass 1              */
  NS_DBG_ROOTS = 9      /* 2      edges whose line search needed the root  */
                        /*        finder, limiter passes 1 and 2          */
};
int ns_get_debug(ns_solver *s, int what, double *out);

/* ---- statistics ------------------------------------------------------- *
 * Admissibility of the current state (Sec. 3: rho > 0 and internal energy
 * > 0, preserved by every stage, Lemma 3.1) and the activity of the convex
 * limiter of Sec. 3.3 in the last forward-Euler stage run (the last stage
 * of the last step, or ns_fe_stage): l_ij = min(l~_ij, l~_ji) is the
 * symmetric pass-1 limiter, l'_ij the pass-2 one; an entry counts as limited
 * after pass 2 when the fraction of P_ij finally applied,
 * l_ij + l'_ij (1 - l_ij), is below 1.  The parabolic counts are those of
 * the last parabolic step (0 before any). */
typedef struct ns_stats_t {
  double min_rho;      /* min_i rho_i of the current state                  */
  double min_eps;      /* min_i E_i - |m_i|^2 / (2 rho_i) (internal energy
                          per unit volume)                                  */
  int64_t argmin_rho;  /* first node attaining min_rho                      */
  int64_t argmin_eps;  /* first node attaining min_eps                      */
  int64_t edges;       /* off-diagonal stencil entries (i != j)             */
  int64_t limited1;    /* entries with l_ij < 1 after pass 1; -1 without
                          convex limiting or before the first stage         */
  int64_t limited2;    /* entries still limited after pass 2; -1 unless
                          two passes have run                               */
  int64_t roots1;      /* entries whose pass-1 line search needed the root
                          of the entropy bound (-1 as limited1)             */
  int64_t roots2;      /* same, pass 2 (-1 as limited2)                     */
  int cg_it_v, cg_it_e, cg_it_l;  /* CG iterations of the last parabolic
                                     step: velocity, energy, low-order    */
  int fct;             /* 1 if that step used the limited internal energy   */
  double min_eH;       /* its minimum Crank-Nicolson internal energy        */
  int fp64_redo;       /* NS_PREC_MIXED_FP32: synchronous steps redone in
                          FP64 arithmetic after a failed FP64 re-check     */
} ns_stats_t;
/* Computes the statistics on the device (a reduction over all rows) and
 * waits for it; device scratch for the partial results (about 57 KB) is
 * allocated from the stream-ordered pool for the call.  NS_ESTATE without
 * a state; NS_ENOMEM if the scratch does not fit. */
int ns_stats(ns_solver *s, ns_stats_t *out);

/* ns_stats for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same statistics, bit for bit, with the partial results kept in a
 * fixed array of 7 * 1024 + 7 doubles (about 57 KB) that the library holds
 * in each device's memory until the process ends; the kernels stride over
 * the rows with at most 1024 workgroups, so every mesh fits.  No
 * hipMalloc/hipFree; the device address of the array is looked up once per
 * device on the first call there.  Every call on one GPU shares that
 * GPU's array (each call overwrites the slots it reads, nothing needs to
 * start at zero): calls that overlap on one GPU -- from several threads,
 * or on solvers with different streams -- race.  Waits for the solver's
 * stream; NS_ESTATE without a state; NS_EHIP if the array's address
 * cannot be found. */
int ns_stats_noalloc(ns_solver *s, ns_stats_t *out);

/* ---- timing and diagnostics ------------------------------------------- */
/* Waits for all work queued on the solver's stream. */
int ns_sync(ns_solver *s);
/* The hipStream_t the solver launches on. */
void *ns_stream(ns_solver *s);
/* Per-kernel timing: while enabled, every kernel launch is bracketed by a
 * pair of HIP events on the solver's stream; enabling resets the counters. */
int ns_profile_enable(ns_solver *s, int on);
/* Number of distinct kernels timed so far. */
int ns_profile_count(ns_solver *s);
/* For the k-th timed kernel: its name, number of launches and summed
 * duration in milliseconds.  Synchronises.  NS_EINVAL if k is out of range. */
int ns_profile_get(ns_solver *s, int k, const char **name, int64_t *launches,
                   double *total_ms);
/* Measurement utility: copies `bytes` (rounded down to a multiple of 16)
 * between two scratch device buffers with a plain streaming copy kernel
 * that moves `word` bytes per lane (8 or 16; the kernels are profiled as
 * "copy8" and "copy"), `reps` times on the solver's stream, and returns the
 * average kernel time in *avg_ms.  Used to state the achievable device copy
 * bandwidth and to calibrate hardware byte counters against a kernel of
 * known traffic.  Allocates (and frees) the two buffers; NS_EINVAL for a
 * word size other than 8 or 16, NS_ENOMEM if the buffers do not fit. */
int ns_copy_bench(ns_solver *s, int64_t bytes, int reps, int word,
                  double *avg_ms);
/* Device bytes allocated by the solver. */
int64_t ns_device_bytes(const ns_solver *s);
/* Message describing the last error of the solver (never NULL). */
const char *ns_last_error(const ns_solver *s);
/* Message of the last failed ns_graph_create / ns_solver_create on this
 * thread. */
const char *ns_create_error(void);
const char *ns_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* NS_H */
