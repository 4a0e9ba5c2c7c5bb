// par_kernels.hpp -- HIP kernels of the parabolic sub-step (Sec. 5 of
// arXiv:2106.02159; the parabolic-step algorithm of the appendix), gfx950.
//
// Operators are applied matrix-free, one lane per node (par_ops.hpp): at a
// node all of whose 2^dim cells exist by the pre-summed 3^dim-point stencil
// of the uniform mesh, at wall nodes cell by cell with the constant Q1
// element matrix (element.hpp; the tables are wave-uniform and read through
// the scalar cache).  No atomics: results are deterministic and independent
// of the launch shape.
//
// The linear systems (velocity with no-slip rows eliminated, internal
// energy with homogeneous Neumann conditions) are solved by conjugate
// gradients with the diagonal preconditioner or a multigrid V-cycle
// (mg_kernels.hip), kept entirely on the device:
// block partial sums are reduced in a fixed order by a one-block kernel
// that also updates the CG scalars; every kernel of an iteration returns
// at once when the solve has converged, so the host launches iterations in
// batches and checks convergence only between batches.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace ns {

constexpr int kParBlock = 256;

struct ParGrid {
  int64_t N;
  int64_t n[3];
  int per[3];
};

struct CGState {
  double rz, rr, bb, pq, alpha, beta, rtol2;
  int done, it, maxit, pad;
};

// One level of the geometric multigrid preconditioner (FP32 V-cycle,
// mg_kernels.hip).  Level 0 is the mesh of the solver; level l+1 halves the
// cells of every direction (rounded up), so coarse grids need not nest: the
// prolongation interpolates the coarse Q1 function at the fine nodes (two
// weights per direction), the restriction is its exact transpose.  The
// operator of a level is rediscretised on its own mesh size; its mass-term
// coefficient rho m is restricted from the finer level (the restriction of
// the lumped masses of Q1 is the coarse lumped mass).
struct MGLevel {
  ParGrid G;
  const float *tab;  // element tables at this level's mesh size
  float *rm;         // N: rho m
  float *diag;       // NC*N: diagonal of the level operator
  float *x, *y;      // NC*N: iterate (two buffers, the smoother alternates)
  float *b, *d;      // NC*N: right-hand side, Chebyshev direction
  float *lmax;       // 1: Gershgorin bound of the spectrum of D^-1 A
  float *gpart;      // block maxima for lmax
};

// Coefficients and spectral bounds of all levels for one system: rho m from
// the fine rm (FP64), diagonals, lmax; ncomp = dim (velocity, no-slip rows
// fixed) or 1 (energy).
void mg_setup(int dim, int ncomp, MGLevel *lv, int nlev, const double *rm, double cdt,
              hipStream_t s);
// z = V-cycle(r) (Chebyshev(deg)-Jacobi pre- and post-smoothing, coarsest
// level smoothed `coarse_deg` times from zero); no-op once st->done.
void mg_vcycle(int dim, int ncomp, const MGLevel *lv, int nlev, const double *r, double *z,
               double cdt, const CGState *st, int deg, int coarse_deg, hipStream_t s);

struct ParBufs {
  const double *tab;    // element tables (Q1Tables::packed)
  const double *mi;     // N lumped masses
  const uint8_t *fixed; // N: 1 at no-slip (wall) nodes
  double *Vn;           // dim*N velocity at t^n
  double *x, *r, *p, *q, *b, *diag;  // dim*N CG vectors (first N for energy)
  double *rm;           // N: rho_i m_i
  double *en;           // N: e^n
  double *K;            // N: dissipation K_i
  double *eH, *eL, *w, *Rp, *Rm;  // N: limiting
  double *cellK;        // 2^dim * N: per-cell shares of the dissipation
  double *partial;      // 3 * nblocks block partial sums
  CGState *cg;
  double *scal;         // [0] min e^H
  int *flags;           // [1] inadmissible result
};

// velocity system set-up from the state U (nc*N): V^n, rho m, RHS m M^n,
// start x = V^n, diagonal rho m + dt/2 a_ii; e^n
void par_prep(int dim, const ParGrid &g, const ParBufs &B, const double *U,
              double dt, hipStream_t s);
// CG: start from x (residual, first direction); then `iters` iterations
// (no-ops once converged).  ncomp = dim (velocity, stress operator) or 1
// (energy, heat operator with coefficient cdt).
void par_cg_start(int dim, int ncomp, const ParGrid &g, const ParBufs &B,
                  double cdt, double rtol, int maxit, hipStream_t s);
void par_cg_iterate(int dim, int ncomp, const ParGrid &g, const ParBufs &B,
                    double cdt, int iters, hipStream_t s);
// The same with the multigrid preconditioner (z in B.q's sibling buffer zb).
void par_cg_start_mg(int dim, int ncomp, const ParGrid &g, const ParBufs &B, double *zb,
                     double cdt, double rtol, int maxit, const MGLevel *lv, int nlev,
                     int deg, int coarse_deg, hipStream_t s);
void par_cg_iterate_mg(int dim, int ncomp, const ParGrid &g, const ParBufs &B, double *zb,
                       double cdt, int iters, const MGLevel *lv, int nlev, int deg,
                       int coarse_deg, hipStream_t s);
// V^{n+1} = 2 V^{1/2} - V^n (0 at no-slip nodes) into Vn and out (momentum
// rows), K_i from V^{1/2} (x); then the energy system: RHS rho m e^n +
// ksrc m K, start e^n, diagonal rho m + cdt b_ii
void par_velocity_done(int dim, const ParGrid &g, const ParBufs &B,
                       const double *U, double *out, double mu, double lambda,
                       hipStream_t s);
void par_energy_setup(int dim, const ParGrid &g, const ParBufs &B, double cdt,
                      double ksrc, hipStream_t s);
// e^H = 2 x - e^n and min e^H into scal[0]
void par_energy_high(int dim, const ParGrid &g, const ParBufs &B, hipStream_t s);
// after the low-order solve (x = e^L): FCT of A_ij towards the local bounds
void par_fct(int dim, const ParGrid &g, const ParBufs &B, double dt,
             hipStream_t s);
// rho, E = rho e + rho |V^{n+1}|^2 / 2 with e from `e` (e^H or the limited
// value in w); admissibility flag
void par_finish(int dim, const ParGrid &g, const ParBufs &B, const double *U,
                const double *e, double *out, hipStream_t s);

}  // namespace ns
