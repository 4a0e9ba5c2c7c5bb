// hyp_kernels.hpp -- HIP kernels of one forward-Euler stage of the
// hyperbolic step (Algorithm 1 of arXiv:2106.02159), gfx950.
//
// Layout: node vectors (states, U^L, F^H, U^(1)) in component pairs
// (node_layout.hpp), the other node arrays component-major (component c of
// node i at c*N + i); edge arrays are sliced ELL (rows in slices of 64, slot-major
// within a slice: slot k of row i at ((i/64) W + k) 64 + i%64), so lane i of
// a wavefront reading slot k of its row produces one coalesced access.  One
// lane owns one row; neighbour data are gathered through the L1/L2 caches.  Sweeps, in dependency order (each needs the
// previous one complete over the whole mesh):
//   k_prim   per node: v, p, sound speed a, a p^(-(g-1)/(2g)), eta, Phi
//   k_visc   d^L_ij for j > i (Sec. 3.1), written to (i,j) and (j,i);
//            indicator alpha_i (Sec. 3.2)
//   k_dt     (auto time step only) per-block min of m_i / (2 sum_j d_ij)
//   k_lo     d_ii, stage CFL check, U^L (eq. loworder), local bounds from
//            the bar states (eq. bar_state), F^H_i (Sec. 3.2)
//   k_lim1   P_ij (Sec. 3.3) and the pass-1 line search l~_ij; entries
//            whose entropy bound cuts inside (0, l_rho) go to a work list
//   k_root   roots of the entropy bound for the listed entries, one lane
//            per entry (the rare slow path, kept out of the row sweeps)
//   k_lim2   l_ij = min(l~_ij, l~_ji), U^(1) = U^L + lambda_i sum l P;
//            pass-2 line search on (1 - l) P, stored as l~'_ij (1 - l_ij)
//            (or the final state for one pass)
//   k_fin    l' (1-l) symmetrised, U = U^(1) + lambda_i sum l' (1-l) P, SSP
//            combination a U^n + b U and admissibility flag
//   k_slip   slip post-processing at wall nodes (eq. slip_bc)
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

#include "box_nbr.hpp"
#include "euler.hpp"
#include "node_layout.hpp"

namespace ns {

constexpr int kBlock = 256;

// Np: N rounded up to a multiple of 64 (whole slices).  LT is the storage
// type of the graph coefficients and of the per-edge and flux intermediates:
// double, or float in the mixed-precision mode (all arithmetic stays FP64).
template <typename LT>
struct DevGraphT {
  int64_t N;
  int W;
  // column indices, m_ij and c_ij: derived from the box mesh of the row
  // (box_nbr.hpp); geo has one entry per mesh, seg maps each 256-row block
  // to its mesh (null for a single mesh)
  const BoxGeom *geo;
  const int32_t *seg;
  const double *mi;     // N
  const double *rmi;    // N: 1 / m_i
  const double *lfac;   // N: |I(i)| - 1 = 1 / lambda_i
  const double *crm;    // N: (|I(i)| - 1) / m_i = 1 / (lambda_i m_i)
  const double *rrel;   // N: bound relaxation r_i
  const uint8_t *wall;  // N
};

template <typename LT>
struct StageArgsT {
  const double *U;   // stage input, nc*N
  const double *Un;  // state at the start of the step (SSP combination)
  double *out;       // stage output, nc*N
  double *aux;       // (dim+5)*N
  LT *alpha;         // N
  LT *d;             // W*Np (FP32: rounded up, still an upper bound)
  double *UL;        // nc*N
  LT *FH;            // nc*N: F^H_i / m_i, a node vector (3D: (nc+1)*N, with
                     // alpha_i as component nc)
  double *bnds;      // 3*N: rho_min, rho_max, Phi_min (a node vector,
                     // node_layout.hpp)
  LT *lt1;           // W*Np (FP32: rounded down, still feasible)
  LT *lt2;           // W*Np: l~'_ij (1 - l_ij) (FP32: rounded down)
  double *U1;        // nc*N
  double *partial;   // per-block minima for the time step
  double *tau;       // device scalar
  int *flags;        // [0] CFL violated, [1] inadmissible state
  double sa, sb;     // SSP combination out = sa*Un + sb*E(U)
  int check_cfl;
  // adaptive CFL steps: flags[3] (of the member) is set where the low-order
  // update U^L is not admissible
  int check_low = 0;
  // (host side) mixed precision with FP32 arithmetic: the graph viscosity
  // sweep evaluates lambda_max, |c_ij| and the indicator in FP32
  int fp32_eval = 0;
  // Work list of the edges (sliced ELL index) whose line search needs the
  // root of the entropy bound; W*Np entries, so that it holds every edge.
  // Pass 1 fills it and k_root<1> drains it before pass 2 fills it again;
  // qcnt[p] counts the entries of pass p+1 (reset by k_lo).
  uint32_t *q;
  uint32_t *qcnt;
  // 2D two-pass limiting in one sweep (k_lim2 MODE 4): the pass-2 work list
  // q2 (W*Np entries; null: q, filled after q is emptied) and the deferred
  // rows drow (Np entries, qcnt[2] of them; null: not used, qcnt has two
  // counters)
  uint32_t *q2 = nullptr;
  uint32_t *drow = nullptr;
  // 2D: per row, bit k set where the stored pass-2 product of slot k may be
  // nonzero (written by the pass-2 search, read by k_fin); N entries
  uint32_t *nzm = nullptr;
  // A pack of several meshes stepped together: member of every 256-row
  // workgroup (each member's rows start at a workgroup boundary; padding
  // rows are isolated nodes), member count and workgroup offsets of the
  // members (nmem + 1 entries).  tau, tacc and flags (4 ints) are then per
  // member.  seg == nullptr: one mesh.
  const int32_t *seg = nullptr;
  const int32_t *mblk = nullptr;
  int nmem = 1;
};

using DevGraph = DevGraphT<double>;
using StageArgs = StageArgsT<double>;

// ---------------------------------------------------------------------------
// Persistent execution of whole SSPRK(3,3) steps with the CFL time step (the
// serving path): one launch runs `nsteps` steps of every member of a solver
// or pack.  The work is a sequence of items -- (step, stage, phase, member,
// block) -- in phase-major order; a phase is one of the sweeps above over
// one member (its row blocks, its work-list slices, its slip nodes or its
// time-step reduction).  Workgroups take items in sequence order from a
// ticket counter and run each item after the member has finished all its
// items of earlier phases (one completion counter per member).
constexpr int kMaxPhases = 40;
enum PersistPhase : int8_t {
  PP_PRIM = 0, PP_VISC, PP_DTP, PP_DTF, PP_LO, PP_LIM1, PP_ROOT1, PP_LIM2, PP_LIM2B,
  PP_ROOT2, PP_FIN, PP_SLIP
};
// item kinds: one per row block, one per work-list slice, one per 256 slip
// nodes, one per member
enum PersistKind { PK_ROW = 0, PK_ROOT = 1, PK_SLIP = 2, PK_ONE = 3 };
__host__ __device__ constexpr int persist_kind(int ph) {
  return ph == PP_ROOT1 || ph == PP_ROOT2 ? PK_ROOT
         : ph == PP_SLIP                  ? PK_SLIP
         : ph == PP_DTF                   ? PK_ONE
                                          : PK_ROW;
}

// The phase sequence of one step, with the prefix counts every item needs:
// member m has cnt(m, kind) items of each phase of that kind, so its items
// before phase p number pre[p][ROW] nb_m + pre[p][ROOT] nr_m +
// pre[p][SLIP] ns_m + pre[p][ONE]; off[p] is the first item of phase p
// within a step (all members).
struct PersistPlan {
  int nph;
  int8_t phase[kMaxPhases], stage[kMaxPhases];
  int16_t pre[kMaxPhases + 1][4];
  int64_t off[kMaxPhases + 1];
};
// Phases of one step (2D: 29, 3D: 32) for the entropy indicator, convex
// limiting with two passes; totals of the members' row blocks, work-list
// slices and slip slices; nmem members.
void persist_plan(int dim, int64_t rows_tot, int64_t roots_tot, int64_t slips_tot,
                  int nmem, PersistPlan *plan);

template <typename LT>
struct PersistArgsT {
  StageArgsT<LT> A;  // U, Un, out, sa, sb, check_cfl, q and qcnt set per item
  double *S[3];      // state buffers; step 0 starts from S[cur]
  int cur, nsteps;
  double cfl;
  double *tacc;      // per member: time advanced
  // per member (nmem + 1 entries): first row block, first work-list slice,
  // first slip slice, first slip entry
  const int32_t *mblk, *rblk, *sblk, *mslip;
  const int32_t *slip_idx;
  const double *slip_n;  // normal component k of slip entry t at k*nslip + t
  int nslip;
  uint32_t *pcnt;    // 2 per member: work-list lengths of the two passes
  uint32_t *done;    // per member: completed items
  uint32_t *ticket;  // next item
  int *stop;         // [0] set: every workgroup exits; [1] why (1 wait
                     // limit, 2 give-up word); [2] bit `why` of every stop
                     // since it was last cleared (not cleared per launch)
  const int *give_up;    // host-written word (pinned host memory), or null
  uint64_t wait_ticks;   // bound of one wait, in wall-clock ticks
  uint32_t items;        // items of the launch (nsteps steps)
  uint32_t items_step;
  PersistPlan plan;
};

// Workgroups of a persistent launch that fit on the device at once.
int persist_grid(int dim, bool seven, bool fp32);
template <typename LT>
void launch_persistent(int dim, const Gas &gas, const DevGraphT<LT> &g,
                       const PersistArgsT<LT> &p, int grid, hipStream_t s);
// Before a launch: zeroes done[0..nmem), pcnt[0..2 nmem), *ticket and
// stop[1]; stop[0] is set only if a launch of the run gave up (stop[2]);
// run_start: a new run, stop[2] is zeroed first.
void launch_persist_reset(uint32_t *done, uint32_t *pcnt, uint32_t *ticket, int *stop,
                          int nmem, bool run_start, hipStream_t s);

template <typename LT>
void launch_stage(int dim, const Gas &gas, const DevGraphT<LT> &g,
                  const StageArgsT<LT> &a, int indicator, int limiter, int passes,
                  bool auto_dt, double cfl, hipStream_t s,
                  void (*before)(void *, const char *), void (*after)(void *),
                  void *prof);

// prim + graph viscosity + time-step reduction only (writes *a.tau).
template <typename LT>
void launch_dt_only(int dim, const Gas &gas, const DevGraphT<LT> &g,
                    const StageArgsT<LT> &a, double cfl, hipStream_t s,
                    void (*before)(void *, const char *), void (*after)(void *),
                    void *prof);

// Slip projection of the listed nodes; the k-th normal component of entry
// t is nrm[k*stride + t] (stride < 0: nslip).
void launch_slip(int dim, int64_t N, int nslip, const int32_t *idx,
                 const double *nrm, double *U, hipStream_t s, int stride = -1);
// Non-reflecting post-processing (bc_kernels.hip) of n listed nodes: method
// 0 characteristic variables, 1 Godunov; normal component k of entry t at
// nrm[k*n + t], far-field state component c at ud[c*n + t]; flags[1] is set
// for an inadmissible result.
void launch_nonreflecting(int dim, const Gas &gas, int method, int n, const int32_t *idx,
                          const double *nrm, const double *ud, int64_t N, double *U,
                          int *flags, hipStream_t s);
// Rows first .. first+count-1 of the node vector dst (N rows, nc = 4 or 5
// components, node_layout.hpp) from the component-major array src
// (component c of row t at c*ns + t), and back; both arrays on the device.
void launch_nodes_from_cm(int nc, const double *src, int64_t ns, double *dst, int64_t N,
                          int64_t first, int64_t count, hipStream_t s);
void launch_nodes_to_cm(int nc, const double *src, int64_t N, int64_t first, int64_t count,
                        double *dst, int64_t ns, hipStream_t s);
void launch_set_scalar(double *p, double v, hipStream_t s, int n = 1);  // p[0..n) = v
void launch_add_scalar(double *acc, const double *v, hipStream_t s,
                       int n = 1);  // acc[k] += v[k], k < n
// plain streaming copy of 16*n16 bytes, `word` (8 or 16) bytes per lane
// (bandwidth and counter calibration)
void launch_copy(const void *src, void *dst, int64_t n16, int word,
                 hipStream_t s);
// Diagnostics of a state U (nc*N, on the device) and of the limiter arrays
// of the last stage: out[0..6] = min rho, its node, min (E - |m|^2/(2 rho)),
// its node, off-diagonal entries, entries with l_ij < 1 after pass 1,
// entries with l_ij + l'_ij (1 - l_ij) < 1 after pass 2 (mode 0: no limiter
// arrays, counts 0; 1: pass 1 only; 2: both passes).  part must hold
// 7 * kStatsParts doubles; returns the number of partial slots used.
constexpr int kStatsParts = 1024;
template <typename LT>
int launch_stats(int dim, const DevGraphT<LT> &g, const double *U, const LT *lt1,
                 const LT *lt2, int mode, double *part, double *out, hipStream_t s);
void launch_clear_flags(int *flags, hipStream_t s, int n = 1);  // n groups of 4
void launch_check_state(int dim, int64_t N, const double *U, int *flags,
                        hipStream_t s);

}  // namespace ns
