// hyp_kernels.hpp -- HIP kernels of one forward-Euler stage of the
// hyperbolic step (Algorithm 1 of arXiv:2106.02159), gfx950.
//
// Layout: node arrays are structure-of-arrays (component c of node i at
// c*N + i); edge arrays are sliced ELL (rows in slices of 64, slot-major
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
  LT *FH;            // nc*N
  double *bnds;      // 3*N
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
  // Work list of the edges (sliced ELL index) whose line search needs the
  // root of the entropy bound; W*Np entries, so that it holds every edge.
  // Pass 1 fills it and k_root<1> drains it before pass 2 fills it again;
  // qcnt[p] counts the entries of pass p+1 (reset by k_lo).
  uint32_t *q;
  uint32_t *qcnt;
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
