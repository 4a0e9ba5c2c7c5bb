// mg_kernels.hip -- geometric multigrid V-cycle in FP32 preconditioning the
// parabolic CG (the paper's viscous-dominated regime: a V-cycle in single
// precision with a Chebyshev-Jacobi smoother inside the double-precision CG).
//
// Smoother: Chebyshev iteration of degree deg for A x = b preconditioned by
// the diagonal D, on the interval [lmax/10, lmax] where lmax is the
// Gershgorin bound of D^-1 A (an upper bound of its spectrum, so the
// iteration cannot diverge); theta, delta the interval's centre and half
// width, sigma = theta/delta, rho_0 = 1/sigma, rho_k = 1/(2 sigma - rho_{k-1}):
//   d_0 = D^-1 r_0 / theta,  d_k = rho_k rho_{k-1} d_{k-1} + 2 rho_k/delta D^-1 r_k,
//   x_{k+1} = x_k + d_k,  r_k = b - A x_k.
// The same polynomial before and after the coarse correction and R = P^T
// make the V-cycle symmetric, as the preconditioned CG needs.  Rows of
// no-slip nodes (velocity) are kept at zero on every level.
#include "par_kernels.hpp"

#include <cmath>

#include "par_ops.hpp"

namespace ns {
namespace {
using namespace pops;

__device__ __forceinline__ int64_t mgid() {
  return (int64_t)blockIdx.x * kParBlock + threadIdx.x;
}
inline dim3 mgrid(int64_t n) { return dim3((unsigned)((n + kParBlock - 1) / kParBlock)); }

template <int DIM>
__device__ __forceinline__ bool wall_node(const ParGrid &G, const int64_t c[3]) {
  bool w = false;
#pragma unroll
  for (int d = 0; d < DIM; ++d)
    if (!G.per[d] && (c[d] == 0 || c[d] == G.n[d] - 1)) w = true;
  return w;
}

// coarse nodes (at most 2) and weights interpolating at fine index i of one
// direction: the fine node sits at i cc/cf coarse cells
__device__ __forceinline__ int interp1(int64_t i, int64_t nf, int64_t nc, int per,
                                       int64_t *I, float *w) {
  const int64_t cf = per ? nf : nf - 1, cc = per ? nc : nc - 1;
  const double xi = (double)i * (double)cc / (double)cf;
  const int64_t i0 = (int64_t)floor(xi);
  const double t = xi - (double)i0;
  if (!per && i0 >= cc) {
    I[0] = cc;
    w[0] = 1.0f;
    return 1;
  }
  I[0] = i0;
  w[0] = (float)(1.0 - t);
  if (!(t > 0.0)) return 1;
  I[1] = per ? (i0 + 1) % nc : i0 + 1;
  w[1] = (float)t;
  return 2;
}

// fine indices (at most 6) and weights with which coarse index I enters the
// interpolation: the transpose of interp1, with the same arithmetic
__device__ __forceinline__ int restrict1(int64_t I, int64_t nf, int64_t nc, int per,
                                         int64_t *fi, float *w) {
  const int64_t cf = per ? nf : nf - 1, cc = per ? nc : nc - 1;
  const int64_t lo = (int64_t)floor((double)(I - 1) * (double)cf / (double)cc) - 1;
  const int64_t hi = (int64_t)ceil((double)(I + 1) * (double)cf / (double)cc) + 1;
  int n = 0;
  for (int64_t j = lo; j <= hi && n < 6; ++j) {
    int64_t i = j;
    if (per) i = ((j % nf) + nf) % nf;
    else if (j < 0 || j >= nf) continue;
    int64_t J[2];
    float ww[2];
    const int m = interp1(i, nf, nc, per, J, ww);
    for (int q = 0; q < m; ++q)
      if (J[q] == I) {
        fi[n] = i;
        w[n] = ww[q];
        ++n;
      }
  }
  return n;
}

// b_c = R r_f; VEL: zero at no-slip coarse nodes
template <int DIM, int NC, bool VEL>
__global__ __launch_bounds__(kParBlock) void k_mg_restrict(ParGrid Gf, ParGrid Gc,
                                                           const float *__restrict__ rf,
                                                           float *__restrict__ bc,
                                                           const CGState *st) {
  if (st && st->done) return;
  const int64_t I = mgid();
  if (I >= Gc.N) return;
  int64_t c[3];
  decode(Gc, I, c);
  float acc[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) acc[k] = 0.0f;
  if (!(VEL && wall_node<DIM>(Gc, c))) {
    int64_t fi[3][6];
    float w[3][6];
    int n[3] = {1, 1, 1};
    fi[2][0] = 0;
    w[2][0] = 1.0f;
#pragma unroll
    for (int d = 0; d < DIM; ++d) n[d] = restrict1(c[d], Gf.n[d], Gc.n[d], Gf.per[d], fi[d], w[d]);
    for (int a2 = 0; a2 < n[2]; ++a2)
      for (int a1 = 0; a1 < n[1]; ++a1)
        for (int a0 = 0; a0 < n[0]; ++a0) {
          const int64_t j = fi[0][a0] + Gf.n[0] * (fi[1][a1] + Gf.n[1] * fi[2][a2]);
          const float ww = w[0][a0] * w[1][a1] * w[2][a2];
#pragma unroll
          for (int k = 0; k < NC; ++k) acc[k] += ww * rf[k * Gf.N + j];
        }
  }
#pragma unroll
  for (int k = 0; k < NC; ++k) bc[k * Gc.N + I] = acc[k];
}

// x_f += P x_c; VEL: no-slip fine nodes untouched (they stay zero)
template <int DIM, int NC, bool VEL>
__global__ __launch_bounds__(kParBlock) void k_mg_prolong(ParGrid Gf, ParGrid Gc,
                                                          const float *__restrict__ xc,
                                                          float *__restrict__ xf,
                                                          const CGState *st) {
  if (st && st->done) return;
  const int64_t i = mgid();
  if (i >= Gf.N) return;
  int64_t c[3];
  decode(Gf, i, c);
  if (VEL && wall_node<DIM>(Gf, c)) return;
  int64_t I[3][2];
  float w[3][2];
  int n[3] = {1, 1, 1};
  I[2][0] = 0;
  w[2][0] = 1.0f;
#pragma unroll
  for (int d = 0; d < DIM; ++d) n[d] = interp1(c[d], Gf.n[d], Gc.n[d], Gf.per[d], I[d], w[d]);
  float acc[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) acc[k] = 0.0f;
  for (int a2 = 0; a2 < n[2]; ++a2)
    for (int a1 = 0; a1 < n[1]; ++a1)
      for (int a0 = 0; a0 < n[0]; ++a0) {
        const int64_t J = I[0][a0] + Gc.n[0] * (I[1][a1] + Gc.n[1] * I[2][a2]);
        const float ww = w[0][a0] * w[1][a1] * w[2][a2];
#pragma unroll
        for (int k = 0; k < NC; ++k) acc[k] += ww * xc[k * Gc.N + J];
      }
#pragma unroll
  for (int k = 0; k < NC; ++k) xf[k * Gf.N + i] += acc[k];
}

// diagonal and the Gershgorin ratio (rm + cdt sum_j |a_ij|) / (rm + cdt a_ii),
// row sums over the element entries of the node's cells (an upper bound of
// the assembled row's); block maxima into gpart
template <int DIM, int NC, bool VEL>
__global__ __launch_bounds__(kParBlock) void k_mg_diag(MGLevel L, float cdt) {
  constexpr int NL = 1 << DIM;
  const int64_t i = mgid();
  const int64_t N = L.G.N;
  float ratio = 0.0f;
  if (i < N) {
    int64_t c[3];
    decode(L.G, i, c);
    const bool fx = VEL && wall_node<DIM>(L.G, c);
    const float *E = L.tab + (NC > 1 ? 0 : TabOff<DIM>::heat);
    const float rm = L.rm[i];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      if (fx) {
        L.diag[k * N + i] = 1.0f;
        ratio = fmaxf(ratio, 1.0f);
        continue;
      }
      const float dk = rm + cdt * op_diag<DIM, NC, float>(L.G, E, c, k);
      float s = 0.0f;
      for (int a = 0; a < NL; ++a) {
        if (!cell_exists<DIM>(L.G, c, a)) continue;
        for (int b = 0; b < NL; ++b)
#pragma unroll
          for (int l = 0; l < NC; ++l) s += fabsf(E[((k * NC + l) * NL + a) * NL + b]);
      }
      L.diag[k * N + i] = dk;
      ratio = fmaxf(ratio, (rm + cdt * s) / dk);
    }
  }
  __shared__ float sh[kParBlock / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) ratio = fmaxf(ratio, __shfl_xor(ratio, off));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = ratio;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kParBlock / 64; ++w) ratio = fmaxf(ratio, sh[w]);
    L.gpart[blockIdx.x] = ratio;
  }
}

__global__ __launch_bounds__(kParBlock) void k_mg_lmax(const float *__restrict__ gpart, int nb,
                                                       float *lmax) {
  float m = 0.0f;
  for (int j = threadIdx.x; j < nb; j += kParBlock) m = fmaxf(m, gpart[j]);
  __shared__ float sh[kParBlock / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kParBlock / 64; ++w) m = fmaxf(m, sh[w]);
    *lmax = m;
  }
}

__global__ __launch_bounds__(kParBlock) void k_mg_narrow(int64_t n, const double *__restrict__ a,
                                                         float *__restrict__ b) {
  const int64_t t = mgid();
  if (t < n) b[t] = (float)a[t];
}

// level 0 right-hand side from the CG residual; VEL: zero at no-slip nodes
template <int DIM, int NC, bool VEL>
__global__ __launch_bounds__(kParBlock) void k_mg_from_residual(ParGrid G,
                                                                const double *__restrict__ r,
                                                                float *__restrict__ b,
                                                                const CGState *st) {
  if (st && st->done) return;
  const int64_t i = mgid();
  if (i >= G.N) return;
  int64_t c[3];
  decode(G, i, c);
  const bool fx = VEL && wall_node<DIM>(G, c);
#pragma unroll
  for (int k = 0; k < NC; ++k) b[k * G.N + i] = fx ? 0.0f : (float)r[k * G.N + i];
}

template <int NC>
__global__ __launch_bounds__(kParBlock) void k_mg_widen(int64_t N, const float *__restrict__ x,
                                                        double *__restrict__ z,
                                                        const CGState *st) {
  if (st && st->done) return;
  const int64_t t = mgid();
  if (t < NC * N) z[t] = (double)x[t];
}

// one Chebyshev iteration k: from xin (zero when zs and k == 0) to xout
template <int DIM, int NC, bool VEL>
__global__ __launch_bounds__(kParBlock) void k_mg_cheb(MGLevel L, float cdt, int k, int zs,
                                                       const float *__restrict__ xin,
                                                       float *__restrict__ xout,
                                                       const CGState *st) {
  if (st && st->done) return;
  const int64_t i = mgid();
  const int64_t N = L.G.N;
  if (i >= N) return;
  int64_t c[3];
  decode(L.G, i, c);
  if (VEL && wall_node<DIM>(L.G, c)) {
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      xout[q * N + i] = 0.0f;
      L.d[q * N + i] = 0.0f;
    }
    return;
  }
  const float lmax = *L.lmax, lmin = 0.1f * lmax;
  const float theta = 0.5f * (lmax + lmin), delta = 0.5f * (lmax - lmin);
  const float sigma = theta / delta;
  float rho_prev = 1.0f / sigma, rho = rho_prev;
  for (int j = 1; j <= k; ++j) {
    rho_prev = rho;
    rho = 1.0f / (2.0f * sigma - rho_prev);
  }
  float r[NC];
  const float rm = L.rm[i];
  if (zs && k == 0) {
#pragma unroll
    for (int q = 0; q < NC; ++q) r[q] = L.b[q * N + i];
  } else {
    float acc[NC];
    op_apply<DIM, NC, float>(L.G, L.tab, xin, c, acc);
#pragma unroll
    for (int q = 0; q < NC; ++q) r[q] = L.b[q * N + i] - (rm * xin[q * N + i] + cdt * acc[q]);
  }
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const float zr = r[q] / L.diag[q * N + i];
    const float d = k == 0 ? zr / theta : rho * rho_prev * L.d[q * N + i] + 2.0f * rho / delta * zr;
    L.d[q * N + i] = d;
    xout[q * N + i] = (zs && k == 0 ? 0.0f : xin[q * N + i]) + d;
  }
}

// res = b - A x (VEL: zero at no-slip nodes)
template <int DIM, int NC, bool VEL>
__global__ __launch_bounds__(kParBlock) void k_mg_residual(MGLevel L, float cdt,
                                                           const float *__restrict__ x,
                                                           float *__restrict__ res,
                                                           const CGState *st) {
  if (st && st->done) return;
  const int64_t i = mgid();
  const int64_t N = L.G.N;
  if (i >= N) return;
  int64_t c[3];
  decode(L.G, i, c);
  if (VEL && wall_node<DIM>(L.G, c)) {
#pragma unroll
    for (int q = 0; q < NC; ++q) res[q * N + i] = 0.0f;
    return;
  }
  float acc[NC];
  op_apply<DIM, NC, float>(L.G, L.tab, x, c, acc);
  const float rm = L.rm[i];
#pragma unroll
  for (int q = 0; q < NC; ++q) res[q * N + i] = L.b[q * N + i] - (rm * x[q * N + i] + cdt * acc[q]);
}

template <int DIM, int NC, bool VEL>
void setup_t(MGLevel *lv, int nlev, const double *rm, double cdt, hipStream_t s) {
  hipLaunchKernelGGL(k_mg_narrow, mgrid(lv[0].G.N), dim3(kParBlock), 0, s, lv[0].G.N, rm,
                     lv[0].rm);
  for (int l = 1; l < nlev; ++l)
    hipLaunchKernelGGL((k_mg_restrict<DIM, 1, false>), mgrid(lv[l].G.N), dim3(kParBlock), 0, s,
                       lv[l - 1].G, lv[l].G, (const float *)lv[l - 1].rm, lv[l].rm,
                       (const CGState *)nullptr);
  for (int l = 0; l < nlev; ++l) {
    const dim3 g = mgrid(lv[l].G.N);
    hipLaunchKernelGGL((k_mg_diag<DIM, NC, VEL>), g, dim3(kParBlock), 0, s, lv[l], (float)cdt);
    hipLaunchKernelGGL(k_mg_lmax, dim3(1), dim3(kParBlock), 0, s, (const float *)lv[l].gpart,
                       (int)g.x, lv[l].lmax);
  }
}

// smooth `deg` times on level l starting from *cur (zero if zs); the
// iterate alternates between the level's x and y; returns the result
template <int DIM, int NC, bool VEL>
float *smooth(const MGLevel &L, float *cur, int deg, int zs, float cdt, const CGState *st,
              hipStream_t s) {
  const dim3 g = mgrid(L.G.N);
  for (int k = 0; k < deg; ++k) {
    float *out = cur == L.x ? L.y : L.x;
    hipLaunchKernelGGL((k_mg_cheb<DIM, NC, VEL>), g, dim3(kParBlock), 0, s, L, cdt, k, zs,
                       (const float *)cur, out, st);
    cur = out;
  }
  return cur;
}

template <int DIM, int NC, bool VEL>
float *vcycle_level(const MGLevel *lv, int l, int nlev, float cdt, const CGState *st, int deg,
                    int coarse_deg, hipStream_t s) {
  const MGLevel &L = lv[l];
  if (l == nlev - 1) return smooth<DIM, NC, VEL>(L, L.x, coarse_deg, 1, cdt, st, s);
  float *cur = smooth<DIM, NC, VEL>(L, L.x, deg, 1, cdt, st, s);
  float *res = cur == L.x ? L.y : L.x;
  const dim3 g = mgrid(L.G.N), gc = mgrid(lv[l + 1].G.N);
  hipLaunchKernelGGL((k_mg_residual<DIM, NC, VEL>), g, dim3(kParBlock), 0, s, L, cdt,
                     (const float *)cur, res, st);
  hipLaunchKernelGGL((k_mg_restrict<DIM, NC, VEL>), gc, dim3(kParBlock), 0, s, L.G, lv[l + 1].G,
                     (const float *)res, lv[l + 1].b, st);
  const float *xc = vcycle_level<DIM, NC, VEL>(lv, l + 1, nlev, cdt, st, deg, coarse_deg, s);
  hipLaunchKernelGGL((k_mg_prolong<DIM, NC, VEL>), g, dim3(kParBlock), 0, s, L.G, lv[l + 1].G, xc,
                     cur, st);
  return smooth<DIM, NC, VEL>(L, cur, deg, 0, cdt, st, s);
}

template <int DIM, int NC, bool VEL>
void vcycle_t(const MGLevel *lv, int nlev, const double *r, double *z, double cdt,
              const CGState *st, int deg, int coarse_deg, hipStream_t s) {
  const dim3 g = mgrid(lv[0].G.N);
  hipLaunchKernelGGL((k_mg_from_residual<DIM, NC, VEL>), g, dim3(kParBlock), 0, s, lv[0].G, r,
                     lv[0].b, st);
  const float *x = vcycle_level<DIM, NC, VEL>(lv, 0, nlev, (float)cdt, st, deg, coarse_deg, s);
  hipLaunchKernelGGL(k_mg_widen<NC>, mgrid(NC * lv[0].G.N), dim3(kParBlock), 0, s, lv[0].G.N, x,
                     z, st);
}

}  // namespace

void mg_setup(int dim, int ncomp, MGLevel *lv, int nlev, const double *rm, double cdt,
              hipStream_t s) {
  if (dim == 2) {
    if (ncomp == 2) setup_t<2, 2, true>(lv, nlev, rm, cdt, s);
    else setup_t<2, 1, false>(lv, nlev, rm, cdt, s);
  } else {
    if (ncomp == 3) setup_t<3, 3, true>(lv, nlev, rm, cdt, s);
    else setup_t<3, 1, false>(lv, nlev, rm, cdt, s);
  }
}

void mg_vcycle(int dim, int ncomp, const MGLevel *lv, int nlev, const double *r, double *z,
               double cdt, const CGState *st, int deg, int coarse_deg, hipStream_t s) {
  if (dim == 2) {
    if (ncomp == 2) vcycle_t<2, 2, true>(lv, nlev, r, z, cdt, st, deg, coarse_deg, s);
    else vcycle_t<2, 1, false>(lv, nlev, r, z, cdt, st, deg, coarse_deg, s);
  } else {
    if (ncomp == 3) vcycle_t<3, 3, true>(lv, nlev, r, z, cdt, st, deg, coarse_deg, s);
    else vcycle_t<3, 1, false>(lv, nlev, r, z, cdt, st, deg, coarse_deg, s);
  }
}

}  // namespace ns
