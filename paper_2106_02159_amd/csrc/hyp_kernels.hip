// hyp_kernels.hip -- forward-Euler stage of the hyperbolic step on gfx950.
// See hyp_kernels.hpp for the sweep structure and data layout.
#include "hyp_kernels.hpp"

#include <climits>

namespace ns {

namespace {

enum { AP_OFF = 0 };  // aux layout: v[0..DIM-1], p, a, b, eta, Phi

template <int DIM> struct Aux {
  static constexpr int P = DIM, A = DIM + 1, B = DIM + 2, ETA = DIM + 3,
                       PHI = DIM + 4, COUNT = DIM + 5;
};

__device__ __forceinline__ int64_t row_id() {
  return (int64_t)blockIdx.x * kBlock + threadIdx.x;
}

template <int DIM>
__device__ __forceinline__ void load_c(const DevGraph &G, int64_t e, double *c) {
  c[0] = G.c0[e];
  c[1] = G.c1[e];
  if constexpr (DIM == 3) c[2] = G.c2[e];
}

template <int NC>
__device__ __forceinline__ void load_state(const double *__restrict__ U,
                                           int64_t N, int64_t i, double *u) {
#pragma unroll
  for (int q = 0; q < NC; ++q) u[q] = U[q * N + i];
}

// f(u) c = (rho v.c, m (v.c) + p c, (v.c)(E + p)) from primitives v, p.
template <int DIM>
__device__ __forceinline__ void flux_dot(const double *u, const double *v,
                                         double p, const double *c,
                                         double *fc) {
  double vc = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) vc += v[k] * c[k];
  fc[0] = u[0] * vc;
#pragma unroll
  for (int k = 0; k < DIM; ++k) fc[1 + k] = u[1 + k] * vc + p * c[k];
  fc[DIM + 1] = vc * (u[DIM + 1] + p);
}

__device__ __forceinline__ double block_min(double v) {
  __shared__ double red[kBlock / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / 64; ++w) v = fmin(v, red[w]);
  }
  return v;
}

// ---------------------------------------------------------------------------
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_prim(int64_t N,
                                                 const double *__restrict__ U,
                                                 double *__restrict__ aux,
                                                 Gas g) {
  const int64_t i = row_id();
  if (i >= N) return;
  using X = Aux<DIM>;
  const double r = U[i];
  double m[DIM], m2 = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    m[k] = U[(1 + k) * N + i];
    m2 += m[k] * m[k];
  }
  const double E = U[(DIM + 1) * N + i];
  const double ir = 1.0 / r;
  const double eps = E - 0.5 * m2 * ir;
  const double p = g.gm1 * eps;
  const double a = sqrt(g.gamma * p * ir);
  const double s = log(eps) - g.gamma * log(r);
#pragma unroll
  for (int k = 0; k < DIM; ++k) aux[k * N + i] = m[k] * ir;
  aux[X::P * N + i] = p;
  aux[X::A * N + i] = a;
  aux[X::B * N + i] = a * pow(p, -g.ex);
  aux[X::ETA * N + i] = -r * s;
  aux[X::PHI * N + i] = exp(s);
}

// ---------------------------------------------------------------------------
// Graph viscosity d^L_ij (j > i, stored at (i,j) and (j,i)) and alpha_i.
template <int DIM, int IND>
__global__ __launch_bounds__(kBlock) void k_visc(DevGraph G,
                                                 const double *__restrict__ U,
                                                 const double *__restrict__ aux,
                                                 double *__restrict__ d,
                                                 double *__restrict__ alpha,
                                                 Gas g) {
  using X = Aux<DIM>;
  constexpr int NC = DIM + 2;
  const int64_t N = G.N;
  const int64_t i = row_id();
  if (i >= N) return;
  const int W = G.W;
  double vi[DIM];
#pragma unroll
  for (int k = 0; k < DIM; ++k) vi[k] = aux[k * N + i];
  const double pi = aux[X::P * N + i], ai = aux[X::A * N + i],
               bi = aux[X::B * N + i];
  const bool wall_i = G.wall[i] != 0;
  double etap[NC];
  if constexpr (IND == 0) {
    const double ri = U[i];
    double m2 = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      const double mk = U[(1 + k) * N + i];
      m2 += mk * mk;
      etap[1 + k] = mk;
    }
    const double eps = pi / g.gm1;
    const double s = -aux[X::ETA * N + i] / ri;
    const double ie = 1.0 / eps;
    etap[0] = g.gamma - s - m2 / (2.0 * ri * eps);
#pragma unroll
    for (int k = 0; k < DIM; ++k) etap[1 + k] *= ie;
    etap[NC - 1] = -ri * ie;
  }
  double num = 0.0, den = 0.0, scl = 0.0;
  for (int k = 0; k < W; ++k) {
    const int64_t e = (int64_t)k * N + i;
    const int32_t j = G.col[e];
    if (j < 0) continue;
    double c[DIM];
    load_c<DIM>(G, e, c);
    double vj[DIM];
#pragma unroll
    for (int q = 0; q < DIM; ++q) vj[q] = aux[q * N + j];
    const double pj = aux[X::P * N + j], aj = aux[X::A * N + j];
    if constexpr (IND == 0) {
      double uj[NC], fc[NC];
      load_state<NC>(U, N, j, uj);
      const double etaj = aux[X::ETA * N + j];
      double vc = 0.0, c2 = 0.0;
#pragma unroll
      for (int q = 0; q < DIM; ++q) {
        vc += vj[q] * c[q];
        c2 += c[q] * c[q];
      }
      flux_dot<DIM>(uj, vj, pj, c, fc);
      double t = etaj * vc;
#pragma unroll
      for (int q = 0; q < NC; ++q) t -= etap[q] * fc[q];
      num += t;
      den += fabs(t);
      scl += sqrt(c2) * aj * (uj[0] + fabs(etaj));
    }
    if (j > i) {
      const double bj = aux[X::B * N + j];
      double c2 = 0.0;
#pragma unroll
      for (int q = 0; q < DIM; ++q) c2 += c[q] * c[q];
      const double cn = sqrt(c2);
      const double icn = 1.0 / cn;
      double uL = 0.0, uR = 0.0;
#pragma unroll
      for (int q = 0; q < DIM; ++q) {
        uL += vi[q] * c[q] * icn;
        uR += vj[q] * c[q] * icn;
      }
      double dij = lambda_max(g, uL, pi, ai, bi, uR, pj, aj, bj) * cn;
      const int kt = G.trk[e];
      const int64_t et = (int64_t)kt * N + j;
      if (wall_i) {
        // both ends may be on the wall: c_ji != -c_ij, take both directions
        double ct[DIM];
        load_c<DIM>(G, et, ct);
        double ct2 = 0.0;
#pragma unroll
        for (int q = 0; q < DIM; ++q) ct2 += ct[q] * ct[q];
        const double ctn = sqrt(ct2);
        const double ictn = 1.0 / ctn;
        double uLt = 0.0, uRt = 0.0;
#pragma unroll
        for (int q = 0; q < DIM; ++q) {
          uLt += vj[q] * ct[q] * ictn;
          uRt += vi[q] * ct[q] * ictn;
        }
        dij = fmax(dij, lambda_max(g, uLt, pj, aj, bj, uRt, pi, ai, bi) * ctn);
      }
      d[e] = dij;
      d[et] = dij;
    }
  }
  if constexpr (IND == 0) alpha[i] = fabs(num) / (den + 1e-2 * scl);
  else if constexpr (IND == 1) alpha[i] = 1.0;
  else alpha[i] = 0.0;
}

// ---------------------------------------------------------------------------
// Time step: per-block min of m_i / (2 sum_{j != i} d_ij) = -m_i / (2 d_ii).
__global__ __launch_bounds__(kBlock) void k_dt_partial(DevGraph G,
                                                       const double *__restrict__ d,
                                                       double *__restrict__ partial) {
  const int64_t N = G.N;
  const int64_t i = row_id();
  double r = INFINITY;
  if (i < N) {
    double dsum = 0.0;
    for (int k = 0; k < G.W; ++k) {
      const int64_t e = (int64_t)k * N + i;
      const int32_t j = G.col[e];
      if (j >= 0 && j != i) dsum += d[e];
    }
    r = G.mi[i] / (2.0 * dsum);
  }
  r = block_min(r);
  if (threadIdx.x == 0) partial[blockIdx.x] = r;
}

__global__ __launch_bounds__(1024) void k_dt_final(const double *__restrict__ partial,
                                                   int64_t nb, double cfl,
                                                   double *__restrict__ tau) {
  __shared__ double red[16];
  double v = INFINITY;
  for (int64_t b = threadIdx.x; b < nb; b += 1024) v = fmin(v, partial[b]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 16; ++w) v = fmin(v, red[w]);
    *tau = cfl * v;
  }
}

// ---------------------------------------------------------------------------
// Low-order update, bounds and high-order flux.
template <int DIM>
__global__ __launch_bounds__(kBlock) void k_lo(DevGraph G, StageArgs A, Gas g) {
  using X = Aux<DIM>;
  constexpr int NC = DIM + 2;
  const int64_t N = G.N;
  const int64_t i = row_id();
  if (i >= N) return;
  const double *__restrict__ U = A.U;
  const double *__restrict__ aux = A.aux;
  double ui[NC], vi[DIM];
  load_state<NC>(U, N, i, ui);
#pragma unroll
  for (int k = 0; k < DIM; ++k) vi[k] = aux[k * N + i];
  const double pi = aux[X::P * N + i];
  const double ali = A.alpha[i];
  const double tau = *A.tau;
  double acc[NC], fh[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) { acc[q] = 0.0; fh[q] = 0.0; }
  double rmin = ui[0], rmax = ui[0], phimin = aux[X::PHI * N + i], dsum = 0.0;
  for (int k = 0; k < G.W; ++k) {
    const int64_t e = (int64_t)k * N + i;
    const int32_t j = G.col[e];
    if (j < 0) continue;
    double c[DIM], fci[NC];
    load_c<DIM>(G, e, c);
    flux_dot<DIM>(ui, vi, pi, c, fci);
    if (j == i) {
#pragma unroll
      for (int q = 0; q < NC; ++q) fh[q] -= fci[q];
      continue;
    }
    double uj[NC], vj[DIM], fcj[NC];
    load_state<NC>(U, N, j, uj);
#pragma unroll
    for (int q = 0; q < DIM; ++q) vj[q] = aux[q * N + j];
    const double pj = aux[X::P * N + j];
    flux_dot<DIM>(uj, vj, pj, c, fcj);
    const double dij = A.d[e];
    // density of the bar state (eq. bar_state) for the local bounds
    const double rbar = 0.5 * (ui[0] + uj[0]) - (fcj[0] - fci[0]) / (2.0 * dij);
    rmin = fmin(rmin, rbar);
    rmax = fmax(rmax, rbar);
    phimin = fmin(phimin, aux[X::PHI * N + j]);
    const double dH = 0.5 * (ali + A.alpha[j]) * dij;
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const double du = uj[q] - ui[q];
      acc[q] += dij * du - (fcj[q] - fci[q]);
      fh[q] += -fcj[q] + dH * du;
    }
    dsum += dij;
  }
  const double tm = tau * G.rmi[i];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    A.UL[q * N + i] = ui[q] + tm * acc[q];
    A.FH[q * N + i] = fh[q];
  }
  if (A.check_cfl && tau > G.mi[i] / (2.0 * dsum)) A.flags[0] = 1;
  const double r = G.rrel[i];
  A.bnds[i] = (1.0 - r) * rmin;
  A.bnds[N + i] = (1.0 + r) * rmax;
  A.bnds[2 * N + i] = (1.0 - r) * phimin;
}

// P_ij = tau/(m_i lambda_i) (b_ij F_j - b_ji F_i + (dH - d)(U_j - U_i)) with
// b_ij = -m_ij/m_j, b_ji = -m_ij/m_i (Sec. 3.3).
template <int DIM>
struct RowCtx {
  static constexpr int NC = DIM + 2;
  double ui[NC], fi[NC];
  double ali, rmi_i, coef;
};

template <int DIM>
__device__ __forceinline__ void load_row(const DevGraph &G, const StageArgs &A,
                                         int64_t i, double tau, RowCtx<DIM> &R) {
  constexpr int NC = DIM + 2;
  const int64_t N = G.N;
  load_state<NC>(A.U, N, i, R.ui);
  load_state<NC>(A.FH, N, i, R.fi);
  R.ali = A.alpha[i];
  R.rmi_i = G.rmi[i];
  R.coef = tau * G.lfac[i] * R.rmi_i;
}

template <int DIM>
__device__ __forceinline__ void compute_P(const DevGraph &G, const StageArgs &A,
                                          const RowCtx<DIM> &R, int64_t e,
                                          int32_t j, double *P) {
  constexpr int NC = DIM + 2;
  const int64_t N = G.N;
  double uj[NC], fj[NC];
  load_state<NC>(A.U, N, j, uj);
  load_state<NC>(A.FH, N, j, fj);
  const double dij = A.d[e];
  const double dH = 0.5 * (R.ali + A.alpha[j]) * dij;
  const double mij = G.mij[e];
  const double rmj = G.rmi[j];
#pragma unroll
  for (int q = 0; q < NC; ++q)
    P[q] = R.coef * (mij * (R.fi[q] * R.rmi_i - fj[q] * rmj) +
                     (dH - dij) * (uj[q] - R.ui[q]));
}

template <int DIM>
__device__ __forceinline__ void finish(const DevGraph &G, const StageArgs &A,
                                       int64_t i, const double *u) {
  constexpr int NC = DIM + 2;
  const int64_t N = G.N;
  double w[NC];
  if (A.sa != 0.0) {
    double un[NC];
    load_state<NC>(A.Un, N, i, un);
#pragma unroll
    for (int q = 0; q < NC; ++q) w[q] = A.sa * un[q] + A.sb * u[q];
  } else {
#pragma unroll
    for (int q = 0; q < NC; ++q) w[q] = A.sb * u[q];
  }
  double m2 = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) m2 += w[1 + k] * w[1 + k];
  const double eps = w[NC - 1] - 0.5 * m2 / w[0];
  if (!(w[0] > 0.0) || !(eps > 0.0)) A.flags[1] = 1;
#pragma unroll
  for (int q = 0; q < NC; ++q) A.out[q * N + i] = w[q];
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_lim1(DevGraph G, StageArgs A, Gas g) {
  constexpr int NC = DIM + 2;
  const int64_t N = G.N;
  const int64_t i = row_id();
  if (i >= N) return;
  RowCtx<DIM> R;
  load_row<DIM>(G, A, i, *A.tau, R);
  double ul[NC];
  load_state<NC>(A.UL, N, i, ul);
  const double rmin = A.bnds[i], rmax = A.bnds[N + i], pmin = A.bnds[2 * N + i];
  for (int k = 0; k < G.W; ++k) {
    const int64_t e = (int64_t)k * N + i;
    const int32_t j = G.col[e];
    if (j < 0 || j == i) continue;
    double P[NC];
    compute_P<DIM>(G, A, R, e, j, P);
    A.lt1[e] = line_search<DIM>(g, ul, P, rmin, rmax, pmin);
  }
}

// MODE 0: convex, pass 1 update + pass-2 line search; 1: convex with one
// pass, final; 2: l = 1 (unlimited high order), final.
template <int DIM, int MODE>
__global__ __launch_bounds__(kBlock) void k_lim2(DevGraph G, StageArgs A, Gas g) {
  constexpr int NC = DIM + 2;
  const int64_t N = G.N;
  const int64_t i = row_id();
  if (i >= N) return;
  RowCtx<DIM> R;
  load_row<DIM>(G, A, i, *A.tau, R);
  const double lam = 1.0 / G.lfac[i];
  double u1[NC];
  load_state<NC>(A.UL, N, i, u1);
  for (int k = 0; k < G.W; ++k) {
    const int64_t e = (int64_t)k * N + i;
    const int32_t j = G.col[e];
    if (j < 0 || j == i) continue;
    double l = 1.0;
    if constexpr (MODE != 2) {
      const int64_t et = (int64_t)G.trk[e] * N + j;
      l = fmin(A.lt1[e], A.lt1[et]);
    }
    double P[NC];
    compute_P<DIM>(G, A, R, e, j, P);
#pragma unroll
    for (int q = 0; q < NC; ++q) u1[q] += lam * l * P[q];
  }
  if constexpr (MODE != 0) {
    finish<DIM>(G, A, i, u1);
  } else {
#pragma unroll
    for (int q = 0; q < NC; ++q) A.U1[q * N + i] = u1[q];
    const double rmin = A.bnds[i], rmax = A.bnds[N + i],
                 pmin = A.bnds[2 * N + i];
    for (int k = 0; k < G.W; ++k) {
      const int64_t e = (int64_t)k * N + i;
      const int32_t j = G.col[e];
      if (j < 0 || j == i) continue;
      const int64_t et = (int64_t)G.trk[e] * N + j;
      const double l = fmin(A.lt1[e], A.lt1[et]);
      double P[NC];
      compute_P<DIM>(G, A, R, e, j, P);
#pragma unroll
      for (int q = 0; q < NC; ++q) P[q] *= (1.0 - l);
      A.lt2[e] = line_search<DIM>(g, u1, P, rmin, rmax, pmin);
    }
  }
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_fin(DevGraph G, StageArgs A, Gas g) {
  constexpr int NC = DIM + 2;
  const int64_t N = G.N;
  const int64_t i = row_id();
  if (i >= N) return;
  RowCtx<DIM> R;
  load_row<DIM>(G, A, i, *A.tau, R);
  const double lam = 1.0 / G.lfac[i];
  double u2[NC];
  load_state<NC>(A.U1, N, i, u2);
  for (int k = 0; k < G.W; ++k) {
    const int64_t e = (int64_t)k * N + i;
    const int32_t j = G.col[e];
    if (j < 0 || j == i) continue;
    const int64_t et = (int64_t)G.trk[e] * N + j;
    const double l1 = fmin(A.lt1[e], A.lt1[et]);
    const double l2 = fmin(A.lt2[e], A.lt2[et]);
    double P[NC];
    compute_P<DIM>(G, A, R, e, j, P);
#pragma unroll
    for (int q = 0; q < NC; ++q) u2[q] += lam * l2 * ((1.0 - l1) * P[q]);
  }
  finish<DIM>(G, A, i, u2);
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_combine_low(DevGraph G, StageArgs A) {
  constexpr int NC = DIM + 2;
  const int64_t i = row_id();
  if (i >= G.N) return;
  double u[NC];
  load_state<NC>(A.UL, G.N, i, u);
  finish<DIM>(G, A, i, u);
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_slip(int nslip,
                                                 const int32_t *__restrict__ idx,
                                                 const double *__restrict__ nrm,
                                                 int64_t N, double *__restrict__ U) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  if (t >= nslip) return;
  const int64_t i = idx[t];
  double n[DIM], mn = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    n[k] = nrm[(int64_t)k * nslip + t];
    mn += U[(1 + k) * N + i] * n[k];
  }
#pragma unroll
  for (int k = 0; k < DIM; ++k) U[(1 + k) * N + i] -= mn * n[k];
}

__global__ __launch_bounds__(kBlock) void k_copy(const double2 *__restrict__ src,
                                                 double2 *__restrict__ dst,
                                                 int64_t n16) {
  const int64_t t = row_id();
  if (t < n16) dst[t] = src[t];
}

__global__ void k_set_scalar(double *p, double v) {
  if (threadIdx.x == 0) p[0] = v;
}

__global__ void k_clear_flags(int *flags) {
  const int t = threadIdx.x;
  if (t < 4) flags[t] = t == 2 ? INT_MAX : 0;
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_check_state(int64_t N,
                                                        const double *__restrict__ U,
                                                        int *__restrict__ flags) {
  constexpr int NC = DIM + 2;
  const int64_t i = row_id();
  if (i >= N) return;
  double u[NC];
  load_state<NC>(U, N, i, u);
  bool ok = u[0] > 0.0;
  double m2 = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) m2 += u[1 + k] * u[1 + k];
  const double eps = u[NC - 1] - 0.5 * m2 / u[0];
  ok = ok && eps > 0.0 && isfinite(eps);
#pragma unroll
  for (int q = 0; q < NC; ++q) ok = ok && isfinite(u[q]);
  if (!ok) {
    flags[1] = 1;
    atomicMin(&flags[2], (int)i);
  }
}

inline dim3 grid_for(int64_t n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

template <int DIM>
void stage_impl(const Gas &gas, const DevGraph &G, const StageArgs &A,
                int indicator, int limiter, int passes, bool auto_dt,
                double cfl, hipStream_t s, void (*before)(void *, const char *),
                void (*after)(void *), void *prof) {
  const dim3 grid = grid_for(G.N), block(kBlock);
#define NS_LAUNCH(name, ...)                                  \
  do {                                                        \
    before(prof, name);                                       \
    __VA_ARGS__;                                              \
    after(prof);                                              \
  } while (0)
  NS_LAUNCH("prim", hipLaunchKernelGGL(k_prim<DIM>, grid, block, 0, s, G.N, A.U,
                                       A.aux, gas));
  if (indicator == 0)
    NS_LAUNCH("visc", hipLaunchKernelGGL((k_visc<DIM, 0>), grid, block, 0, s, G,
                                         A.U, A.aux, A.d, A.alpha, gas));
  else if (indicator == 1)
    NS_LAUNCH("visc", hipLaunchKernelGGL((k_visc<DIM, 1>), grid, block, 0, s, G,
                                         A.U, A.aux, A.d, A.alpha, gas));
  else
    NS_LAUNCH("visc", hipLaunchKernelGGL((k_visc<DIM, 2>), grid, block, 0, s, G,
                                         A.U, A.aux, A.d, A.alpha, gas));
  if (auto_dt) {
    NS_LAUNCH("dt_partial", hipLaunchKernelGGL(k_dt_partial, grid, block, 0, s, G,
                                               A.d, A.partial));
    NS_LAUNCH("dt_final", hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(1024), 0, s,
                                             A.partial, (int64_t)grid.x, cfl,
                                             A.tau));
  }
  NS_LAUNCH("lo", hipLaunchKernelGGL(k_lo<DIM>, grid, block, 0, s, G, A, gas));
  if (limiter == 1) {
    NS_LAUNCH("combine", hipLaunchKernelGGL(k_combine_low<DIM>, grid, block, 0, s,
                                            G, A));
  } else if (limiter == 2) {
    NS_LAUNCH("lim2", hipLaunchKernelGGL((k_lim2<DIM, 2>), grid, block, 0, s, G, A,
                                         gas));
  } else {
    NS_LAUNCH("lim1", hipLaunchKernelGGL(k_lim1<DIM>, grid, block, 0, s, G, A, gas));
    if (passes == 1) {
      NS_LAUNCH("lim2", hipLaunchKernelGGL((k_lim2<DIM, 1>), grid, block, 0, s, G,
                                           A, gas));
    } else {
      NS_LAUNCH("lim2", hipLaunchKernelGGL((k_lim2<DIM, 0>), grid, block, 0, s, G,
                                           A, gas));
      NS_LAUNCH("fin", hipLaunchKernelGGL(k_fin<DIM>, grid, block, 0, s, G, A, gas));
    }
  }
#undef NS_LAUNCH
}

template <int DIM>
void dt_impl(const Gas &gas, const DevGraph &G, const StageArgs &A, double cfl,
             hipStream_t s, void (*before)(void *, const char *),
             void (*after)(void *), void *prof) {
  const dim3 grid = grid_for(G.N), block(kBlock);
  before(prof, "prim");
  hipLaunchKernelGGL(k_prim<DIM>, grid, block, 0, s, G.N, A.U, A.aux, gas);
  after(prof);
  before(prof, "visc_dt");
  hipLaunchKernelGGL((k_visc<DIM, 2>), grid, block, 0, s, G, A.U, A.aux, A.d,
                     A.alpha, gas);
  after(prof);
  before(prof, "dt_partial");
  hipLaunchKernelGGL(k_dt_partial, grid, block, 0, s, G, A.d, A.partial);
  after(prof);
  before(prof, "dt_final");
  hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(1024), 0, s, A.partial,
                     (int64_t)grid.x, cfl, A.tau);
  after(prof);
}

}  // namespace

void launch_dt_only(int dim, const Gas &gas, const DevGraph &g,
                    const StageArgs &a, double cfl, hipStream_t s,
                    void (*before)(void *, const char *), void (*after)(void *),
                    void *prof) {
  if (dim == 2) dt_impl<2>(gas, g, a, cfl, s, before, after, prof);
  else dt_impl<3>(gas, g, a, cfl, s, before, after, prof);
}

void launch_stage(int dim, const Gas &gas, const DevGraph &g,
                  const StageArgs &a, int indicator, int limiter, int passes,
                  bool auto_dt, double cfl, hipStream_t s,
                  void (*before)(void *, const char *), void (*after)(void *),
                  void *prof) {
  if (dim == 2)
    stage_impl<2>(gas, g, a, indicator, limiter, passes, auto_dt, cfl, s, before,
                  after, prof);
  else
    stage_impl<3>(gas, g, a, indicator, limiter, passes, auto_dt, cfl, s, before,
                  after, prof);
}

void launch_slip(int dim, int64_t N, int nslip, const int32_t *idx,
                 const double *nrm, double *U, hipStream_t s) {
  if (nslip <= 0) return;
  const dim3 grid((unsigned)((nslip + kBlock - 1) / kBlock)), block(kBlock);
  if (dim == 2)
    hipLaunchKernelGGL(k_slip<2>, grid, block, 0, s, nslip, idx, nrm, N, U);
  else
    hipLaunchKernelGGL(k_slip<3>, grid, block, 0, s, nslip, idx, nrm, N, U);
}

void launch_set_scalar(double *p, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(64), 0, s, p, v);
}

void launch_copy(const void *src, void *dst, int64_t n16, hipStream_t s) {
  hipLaunchKernelGGL(k_copy, grid_for(n16), dim3(kBlock), 0, s,
                     static_cast<const double2 *>(src), static_cast<double2 *>(dst),
                     n16);
}

void launch_clear_flags(int *flags, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(64), 0, s, flags);
}

void launch_check_state(int dim, int64_t N, const double *U, int *flags,
                        hipStream_t s) {
  const dim3 grid = grid_for(N), block(kBlock);
  if (dim == 2)
    hipLaunchKernelGGL(k_check_state<2>, grid, block, 0, s, N, U, flags);
  else
    hipLaunchKernelGGL(k_check_state<3>, grid, block, 0, s, N, U, flags);
}

}  // namespace ns
