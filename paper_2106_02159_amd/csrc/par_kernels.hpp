// par_kernels.hpp -- HIP kernels of the parabolic sub-step (Sec. 5 of
// arXiv:2106.02159; the parabolic-step algorithm of the appendix), gfx950.
//
// Operators are applied matrix-free, one lane per node: the lane gathers
// the 3^dim values of its neighbourhood into registers once and then, for
// each of its (up to) 2^dim cells, multiplies by the constant Q1 element
// matrix of the uniform mesh (element.hpp; its entries are wave-uniform
// and read through the scalar cache).  No atomics: results are
// deterministic and independent of the launch shape.
//
// The linear systems (velocity with no-slip rows eliminated, internal
// energy with homogeneous Neumann conditions) are solved by conjugate
// gradients with the diagonal preconditioner, kept entirely on the device:
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
