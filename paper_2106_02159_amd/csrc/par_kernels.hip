// par_kernels.hip -- parabolic sub-step on gfx950 (see par_kernels.hpp).
#include "par_kernels.hpp"

#include <cmath>

#include "node_layout.hpp"
#include "par_ops.hpp"

namespace ns {

namespace {
using namespace pops;

// deterministic block sum of K values into partial[k * gridDim.x + block]
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double *partial) {
  __shared__ double sh[K][kParBlock / 64];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) sh[k][w] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double t = 0.0;
      for (int j = 0; j < kParBlock / 64; ++j) t += sh[k][j];
      partial[k * gridDim.x + blockIdx.x] = t;
    }
}

__device__ __forceinline__ int64_t gid() {
  return (int64_t)blockIdx.x * kParBlock + threadIdx.x;
}

// ---------------------------------------------------------------------------
template <int DIM>
__global__ __launch_bounds__(kParBlock) void k_prep(ParGrid G, ParBufs B,
                                                    const double *__restrict__ U,
                                                    double dt) {
  const int64_t i = gid();
  const int64_t N = G.N;
  if (i >= N) return;
  int64_t c[3];
  decode(G, i, c);
  constexpr int NC = DIM + 2;  // U: a node vector (node_layout.hpp)
  const double rho = U[node_at(NC, 0, i, N)];
  const double m = B.mi[i];
  const double rm = rho * m;
  const bool fx = B.fixed[i] != 0;
  B.rm[i] = rm;
  double v2 = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const double M = U[node_at(NC, 1 + k, i, N)];
    const double V = M / rho;
    v2 += V * V;
    B.Vn[k * N + i] = V;
    B.b[k * N + i] = fx ? 0.0 : m * M;
    B.x[k * N + i] = fx ? 0.0 : V;
    B.diag[k * N + i] = fx ? 1.0 : rm + 0.5 * dt * op_diag<DIM, DIM>(G, B.tab, c, k);
  }
  B.en[i] = U[node_at(NC, DIM + 1, i, N)] / rho - 0.5 * v2;
}

// residual and first direction from the start value x; partial r.z, r.r, b.b
template <int DIM, int NC>
__global__ __launch_bounds__(kParBlock) void k_cg_start(ParGrid G, ParBufs B,
                                                        double cdt) {
  constexpr bool VEL = NC > 1;
  const int64_t i = gid();
  const int64_t N = G.N;
  double sums[3] = {0.0, 0.0, 0.0};
  if (i < N) {
    int64_t c[3];
    decode(G, i, c);
    double acc[NC];
    op_apply<DIM, NC>(G, B.tab, B.x, c, acc);
    const bool fx = VEL && B.fixed[i] != 0;
    const double rm = B.rm[i];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const double xi = B.x[k * N + i];
      const double y = fx ? xi : rm * xi + cdt * acc[k];
      const double bi = B.b[k * N + i];
      const double r = bi - y;
      const double z = r / B.diag[k * N + i];
      B.r[k * N + i] = r;
      B.p[k * N + i] = z;
      sums[0] += r * z;
      sums[1] += r * r;
      sums[2] += bi * bi;
    }
  }
  block_sum<3>(sums, B.partial);
}

// q = Op(p); partial p.q
template <int DIM, int NC>
__global__ __launch_bounds__(kParBlock) void k_cg_apply(ParGrid G, ParBufs B,
                                                        double cdt) {
  if (B.cg->done) return;
  constexpr bool VEL = NC > 1;
  const int64_t i = gid();
  const int64_t N = G.N;
  double sums[1] = {0.0};
  if (i < N) {
    int64_t c[3];
    decode(G, i, c);
    double acc[NC];
    op_apply<DIM, NC>(G, B.tab, B.p, c, acc);
    const bool fx = VEL && B.fixed[i] != 0;
    const double rm = B.rm[i];
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const double pi = B.p[k * N + i];
      const double q = fx ? pi : rm * pi + cdt * acc[k];
      B.q[k * N + i] = q;
      sums[0] += pi * q;
    }
  }
  block_sum<1>(sums, B.partial);
}

// x += alpha p, r -= alpha q; partial r.r, r.z
template <int NC>
__global__ __launch_bounds__(kParBlock) void k_cg_update(ParGrid G, ParBufs B) {
  if (B.cg->done) return;
  const int64_t i = gid();
  const int64_t N = G.N;
  const double alpha = B.cg->alpha;
  double sums[2] = {0.0, 0.0};
  if (i < N) {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int64_t t = k * N + i;
      B.x[t] += alpha * B.p[t];
      const double r = B.r[t] - alpha * B.q[t];
      B.r[t] = r;
      sums[0] += r * r;
      sums[1] += r * (r / B.diag[t]);
    }
  }
  block_sum<2>(sums, B.partial);
}

// p = r / diag + beta p
template <int NC>
__global__ __launch_bounds__(kParBlock) void k_cg_direction(ParGrid G, ParBufs B) {
  if (B.cg->done) return;
  const int64_t i = gid();
  const int64_t N = G.N;
  if (i >= N) return;
  const double beta = B.cg->beta;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int64_t t = k * N + i;
    B.p[t] = B.r[t] / B.diag[t] + beta * B.p[t];
  }
}

// ---- CG with an external preconditioner (z = M^-1 r in a separate vector)
// r = b - A x
template <int DIM, int NC>
__global__ __launch_bounds__(kParBlock) void k_cg_residual(ParGrid G, ParBufs B, double cdt) {
  constexpr bool VEL = NC > 1;
  const int64_t i = gid();
  const int64_t N = G.N;
  if (i >= N) return;
  int64_t c[3];
  decode(G, i, c);
  double acc[NC];
  op_apply<DIM, NC>(G, B.tab, B.x, c, acc);
  const bool fx = VEL && B.fixed[i] != 0;
  const double rm = B.rm[i];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const double xi = B.x[k * N + i];
    const double y = fx ? xi : rm * xi + cdt * acc[k];
    B.r[k * N + i] = B.b[k * N + i] - y;
  }
}

// p = z; partial r.z, r.r, b.b
template <int NC>
__global__ __launch_bounds__(kParBlock) void k_cg_first(ParGrid G, ParBufs B,
                                                        const double *__restrict__ z) {
  const int64_t i = gid();
  const int64_t N = G.N;
  double sums[3] = {0.0, 0.0, 0.0};
  if (i < N) {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int64_t t = k * N + i;
      const double r = B.r[t], bi = B.b[t];
      B.p[t] = z[t];
      sums[0] += r * z[t];
      sums[1] += r * r;
      sums[2] += bi * bi;
    }
  }
  block_sum<3>(sums, B.partial);
}

// x += alpha p, r -= alpha q
template <int NC>
__global__ __launch_bounds__(kParBlock) void k_cg_update_xr(ParGrid G, ParBufs B) {
  if (B.cg->done) return;
  const int64_t i = gid();
  const int64_t N = G.N;
  if (i >= N) return;
  const double alpha = B.cg->alpha;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int64_t t = k * N + i;
    B.x[t] += alpha * B.p[t];
    B.r[t] -= alpha * B.q[t];
  }
}

// partial r.r, r.z
template <int NC>
__global__ __launch_bounds__(kParBlock) void k_cg_sums_rz(ParGrid G, ParBufs B,
                                                          const double *__restrict__ z) {
  if (B.cg->done) return;
  const int64_t i = gid();
  const int64_t N = G.N;
  double sums[2] = {0.0, 0.0};
  if (i < N) {
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      const int64_t t = k * N + i;
      const double r = B.r[t];
      sums[0] += r * r;
      sums[1] += r * z[t];
    }
  }
  block_sum<2>(sums, B.partial);
}

// p = z + beta p
template <int NC>
__global__ __launch_bounds__(kParBlock) void k_cg_direction_z(ParGrid G, ParBufs B,
                                                              const double *__restrict__ z) {
  if (B.cg->done) return;
  const int64_t i = gid();
  const int64_t N = G.N;
  if (i >= N) return;
  const double beta = B.cg->beta;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    const int64_t t = k * N + i;
    B.p[t] = z[t] + beta * B.p[t];
  }
}

// one block: reduce the block partials (fixed order) and update the scalars
// PHASE 0: start (r.z, r.r, b.b); 1: alpha from p.q; 2: convergence, beta
template <int PHASE>
__global__ __launch_bounds__(kParBlock) void k_cg_scalars(const double *__restrict__ partial,
                                                          int nb, CGState *st,
                                                          double rtol2, int maxit) {
  if (PHASE != 0 && st->done) return;
  constexpr int K = PHASE == 0 ? 3 : (PHASE == 1 ? 1 : 2);
  double v[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double t = 0.0;
    for (int j = threadIdx.x; j < nb; j += kParBlock) t += partial[k * nb + j];
    v[k] = t;
  }
  __shared__ double sh[K][kParBlock / 64];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) sh[k][w] = v[k];
  __syncthreads();
  if (threadIdx.x != 0) return;
  double s[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    s[k] = 0.0;
    for (int j = 0; j < kParBlock / 64; ++j) s[k] += sh[k][j];
  }
  if constexpr (PHASE == 0) {
    st->rz = s[0];
    st->rr = s[1];
    st->bb = s[2];
    st->rtol2 = rtol2;
    st->maxit = maxit;
    st->it = 0;
    st->alpha = st->beta = st->pq = 0.0;
    st->done = (s[2] == 0.0 || s[1] <= rtol2 * s[2]) ? 1 : 0;
  } else if constexpr (PHASE == 1) {
    st->pq = s[0];
    st->alpha = st->rz / s[0];
  } else {
    st->rr = s[0];
    st->it += 1;
    if (s[0] <= st->rtol2 * st->bb) {
      st->done = 1;
    } else {
      st->beta = s[1] / st->rz;
      st->rz = s[1];
      if (st->it >= st->maxit) st->done = 1;
    }
  }
}

// Dissipation, once per cell: the thread of node i handles the cell whose
// lowest corner is i (if it exists): sigma(V^{1/2}) : eps(V^{1/2}) at the
// 2^dim Gauss points, and for each node a of the cell its share
// sum_q w phi_a(x_q) (sigma : eps)(x_q), stored in cellK[a*N + i].
template <int DIM>
__global__ __launch_bounds__(kParBlock) void k_cell_diss(ParGrid G, ParBufs B,
                                                         double mu, double lam23) {
  using T = TabOff<DIM>;
  constexpr int L = T::L;
  const int64_t i = gid();
  const int64_t N = G.N;
  if (i >= N) return;
  int64_t c[3];
  decode(G, i, c);
  bool has = true;
#pragma unroll
  for (int d = 0; d < DIM; ++d)
    if (!G.per[d] && c[d] > G.n[d] - 2) has = false;
  if (!has) return;
  double v[L][DIM];
#pragma unroll
  for (int b = 0; b < L; ++b) {
    const int64_t j = nb_index<DIM>(G, c, slot_of<DIM>(0, b));
#pragma unroll
    for (int k = 0; k < DIM; ++k) v[b][k] = B.x[k * N + j];
  }
  const double *__restrict__ tab = B.tab;
  const double wq = tab[T::w];
  double share[L];
#pragma unroll
  for (int a = 0; a < L; ++a) share[a] = 0.0;
#pragma unroll
  for (int q = 0; q < L; ++q) {
    double Gm[DIM][DIM];
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
      for (int p = 0; p < DIM; ++p) Gm[k][p] = 0.0;
#pragma unroll
    for (int b = 0; b < L; ++b)
#pragma unroll
      for (int p = 0; p < DIM; ++p) {
        const double dp = tab[T::dphi + (q * L + b) * DIM + p];
#pragma unroll
        for (int k = 0; k < DIM; ++k) Gm[k][p] += v[b][k] * dp;
      }
    double tr = 0.0, ee = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) tr += Gm[k][k];
#pragma unroll
    for (int k = 0; k < DIM; ++k)
#pragma unroll
      for (int p = 0; p < DIM; ++p) {
        const double e = 0.5 * (Gm[k][p] + Gm[p][k]);
        ee += e * e;
      }
    // sigma : eps = 2 mu eps : eps + (lambda - 2/3 mu) (tr eps)^2
    const double se = wq * (2.0 * mu * ee + lam23 * tr * tr);
#pragma unroll
    for (int a = 0; a < L; ++a) share[a] += tab[T::phi + q * L + a] * se;
  }
#pragma unroll
  for (int a = 0; a < L; ++a) B.cellK[a * N + i] = share[a];
}

// V^{n+1} = 2 V^{1/2} - V^n (0 at no-slip nodes) stored in Vn and as
// momentum rho V^{n+1} in out; K_i = (1/m_i) sum over the node's cells of
// the node's share of int sigma : eps phi_i
template <int DIM>
__global__ __launch_bounds__(kParBlock) void k_vel_done(ParGrid G, ParBufs B,
                                                        const double *__restrict__ U,
                                                        double *__restrict__ out) {
  constexpr int L = 1 << DIM;
  const int64_t i = gid();
  const int64_t N = G.N;
  if (i >= N) return;
  int64_t c[3];
  decode(G, i, c);
  const bool fx = B.fixed[i] != 0;
  const double rho = U[node_at(DIM + 2, 0, i, N)];
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const double vn = fx ? 0.0 : 2.0 * B.x[k * N + i] - B.Vn[k * N + i];
    B.Vn[k * N + i] = vn;
    out[node_at(DIM + 2, 1 + k, i, N)] = rho * vn;
  }
  double K = 0.0;
#pragma unroll
  for (int a = 0; a < L; ++a) {
    if (!cell_exists<DIM>(G, c, a)) continue;
    // the cell's lowest corner is the node at offset -a
    const int64_t j = nb_index<DIM>(G, c, slot_of<DIM>(a, 0));
    K += B.cellK[a * N + j];
  }
  B.K[i] = K / B.mi[i];
}

// energy system: RHS rho m e^n + ksrc m K, start e^n, diagonal rho m + cdt b_ii
template <int DIM>
__global__ __launch_bounds__(kParBlock) void k_energy_setup(ParGrid G, ParBufs B,
                                                            double cdt, double ksrc) {
  const int64_t i = gid();
  if (i >= G.N) return;
  int64_t c[3];
  decode(G, i, c);
  constexpr int L = P<DIM>::L;
  const double *heat = B.tab + DIM * DIM * L * L;
  const double rm = B.rm[i];
  const double en = B.en[i];
  B.b[i] = rm * en + ksrc * B.mi[i] * B.K[i];
  B.x[i] = en;
  B.diag[i] = rm + cdt * op_diag<DIM, 1>(G, heat, c, 0);
}

// e^H = 2 e^{1/2} - e^n; block minima of e^H
__global__ __launch_bounds__(kParBlock) void k_energy_high(ParGrid G, ParBufs B) {
  const int64_t i = gid();
  double m = INFINITY;
  if (i < G.N) {
    const double e = 2.0 * B.x[i] - B.en[i];
    B.eH[i] = e;
    m = e;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmin(m, __shfl_xor(m, off));
  __shared__ double sh[kParBlock / 64];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int j = 1; j < kParBlock / 64; ++j) m = fmin(m, sh[j]);
    B.partial[blockIdx.x] = m;
  }
}

__global__ __launch_bounds__(kParBlock) void k_min_final(const double *__restrict__ partial,
                                                         int nb, double *out) {
  double m = INFINITY;
  for (int j = threadIdx.x; j < nb; j += kParBlock) m = fmin(m, partial[j]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmin(m, __shfl_xor(m, off));
  __shared__ double sh[kParBlock / 64];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int j = 1; j < kParBlock / 64; ++j) m = fmin(m, sh[j]);
    out[0] = m;
  }
}

// limiting: w = e^H + e^n - 2 e^L (x holds e^L)
__global__ __launch_bounds__(kParBlock) void k_fct_w(ParGrid G, ParBufs B) {
  const int64_t i = gid();
  if (i >= G.N) return;
  const double eL = B.x[i];
  B.eL[i] = eL;
  B.w[i] = B.eH[i] + B.en[i] - 2.0 * eL;
}

// heat-matrix row b_ij (neighbourhood slots) summed over the node's cells
template <int DIM>
__device__ __forceinline__ void heat_row(const ParGrid &G, const double *__restrict__ heat,
                                         const int64_t c[3], double (&bij)[P<DIM>::S]) {
  constexpr int L = P<DIM>::L;
#pragma unroll
  for (int s = 0; s < P<DIM>::S; ++s) bij[s] = 0.0;
#pragma unroll
  for (int a = 0; a < L; ++a) {
    if (!cell_exists<DIM>(G, c, a)) continue;
#pragma unroll
    for (int b = 0; b < L; ++b) bij[slot_of<DIM>(a, b)] += heat[a * L + b];
  }
}

// Zalesak ratios R+_i, R-_i for A_ij = -dt/2 b_ij (w_j - w_i) against the
// bounds [min_j e^L_j, max_j e^L_j] over the stencil (node included)
template <int DIM>
__global__ __launch_bounds__(kParBlock) void k_fct_ratios(ParGrid G, ParBufs B, double dt) {
  constexpr int S = P<DIM>::S, L = P<DIM>::L;
  const int64_t i = gid();
  if (i >= G.N) return;
  int64_t c[3];
  decode(G, i, c);
  double bij[S];
  heat_row<DIM>(G, B.tab + DIM * DIM * L * L, c, bij);
  const double wi = B.w[i], eLi = B.eL[i];
  double Pp = 0.0, Pm = 0.0, lo = eLi, hi = eLi;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int64_t j = nb_index<DIM>(G, c, s);
    if (j < 0) continue;
    const double eLj = B.eL[j];
    lo = fmin(lo, eLj);
    hi = fmax(hi, eLj);
    if (s == P<DIM>::C) continue;
    const double A = -0.5 * dt * bij[s] * (B.w[j] - wi);
    if (A > 0.0) Pp += A;
    else Pm += A;
  }
  const double rm = B.rm[i];
  const double Qp = rm * (hi - eLi), Qm = rm * (lo - eLi);
  B.Rp[i] = Pp > 0.0 ? fmin(1.0, Qp / Pp) : 1.0;
  B.Rm[i] = Pm < 0.0 ? fmin(1.0, Qm / Pm) : 1.0;
}

// e = e^L + (1/(rho_i m_i)) sum_j l_ij A_ij into eH
template <int DIM>
__global__ __launch_bounds__(kParBlock) void k_fct_apply(ParGrid G, ParBufs B, double dt) {
  constexpr int S = P<DIM>::S, L = P<DIM>::L;
  const int64_t i = gid();
  if (i >= G.N) return;
  int64_t c[3];
  decode(G, i, c);
  double bij[S];
  heat_row<DIM>(G, B.tab + DIM * DIM * L * L, c, bij);
  const double wi = B.w[i], Rpi = B.Rp[i], Rmi = B.Rm[i];
  double sum = 0.0;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    if (s == P<DIM>::C) continue;
    const int64_t j = nb_index<DIM>(G, c, s);
    if (j < 0) continue;
    const double A = -0.5 * dt * bij[s] * (B.w[j] - wi);
    const double l = A > 0.0 ? fmin(Rpi, B.Rm[j]) : fmin(Rmi, B.Rp[j]);
    sum += l * A;
  }
  B.eH[i] = B.eL[i] + sum / B.rm[i];
}

template <int DIM>
__global__ __launch_bounds__(kParBlock) void k_par_finish(ParGrid G, ParBufs B,
                                                          const double *__restrict__ U,
                                                          const double *__restrict__ e,
                                                          double *__restrict__ out) {
  const int64_t i = gid();
  const int64_t N = G.N;
  if (i >= N) return;
  const double rho = U[node_at(DIM + 2, 0, i, N)];
  double v2 = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    const double v = B.Vn[k * N + i];
    v2 += v * v;
  }
  const double ei = e[i];
  out[node_at(DIM + 2, 0, i, N)] = rho;
  out[node_at(DIM + 2, DIM + 1, i, N)] = rho * ei + 0.5 * rho * v2;
  if (!(ei > 0.0) || !isfinite(ei)) B.flags[1] = 1;
}

inline dim3 grid_of(int64_t n) { return dim3((unsigned)((n + kParBlock - 1) / kParBlock)); }

}  // namespace

void par_prep(int dim, const ParGrid &g, const ParBufs &B, const double *U,
              double dt, hipStream_t s) {
  if (dim == 2) hipLaunchKernelGGL(k_prep<2>, grid_of(g.N), dim3(kParBlock), 0, s, g, B, U, dt);
  else hipLaunchKernelGGL(k_prep<3>, grid_of(g.N), dim3(kParBlock), 0, s, g, B, U, dt);
}

namespace {
template <int DIM, int NC>
void cg_start(const ParGrid &g, const ParBufs &B, double cdt, double rtol, int maxit,
              hipStream_t s) {
  const dim3 grid = grid_of(g.N), blk(kParBlock);
  hipLaunchKernelGGL((k_cg_start<DIM, NC>), grid, blk, 0, s, g, B, cdt);
  hipLaunchKernelGGL(k_cg_scalars<0>, dim3(1), blk, 0, s, B.partial, (int)grid.x,
                     B.cg, rtol * rtol, maxit);
}

template <int DIM, int NC>
void cg_iterate(const ParGrid &g, const ParBufs &B, double cdt, int iters,
                hipStream_t s) {
  const dim3 grid = grid_of(g.N), blk(kParBlock);
  for (int it = 0; it < iters; ++it) {
    hipLaunchKernelGGL((k_cg_apply<DIM, NC>), grid, blk, 0, s, g, B, cdt);
    hipLaunchKernelGGL(k_cg_scalars<1>, dim3(1), blk, 0, s, B.partial, (int)grid.x,
                       B.cg, 0.0, 0);
    hipLaunchKernelGGL(k_cg_update<NC>, grid, blk, 0, s, g, B);
    hipLaunchKernelGGL(k_cg_scalars<2>, dim3(1), blk, 0, s, B.partial, (int)grid.x,
                       B.cg, 0.0, 0);
    hipLaunchKernelGGL(k_cg_direction<NC>, grid, blk, 0, s, g, B);
  }
}
template <int DIM, int NC>
void cg_start_mg(const ParGrid &g, const ParBufs &B, double *z, double cdt, double rtol,
                 int maxit, const MGLevel *lv, int nlev, int deg, int cdeg, hipStream_t s) {
  const dim3 grid = grid_of(g.N), blk(kParBlock);
  hipLaunchKernelGGL((k_cg_residual<DIM, NC>), grid, blk, 0, s, g, B, cdt);
  mg_vcycle(DIM, NC, lv, nlev, B.r, z, cdt, nullptr, deg, cdeg, s);
  hipLaunchKernelGGL(k_cg_first<NC>, grid, blk, 0, s, g, B, (const double *)z);
  hipLaunchKernelGGL(k_cg_scalars<0>, dim3(1), blk, 0, s, B.partial, (int)grid.x,
                     B.cg, rtol * rtol, maxit);
}

template <int DIM, int NC>
void cg_iterate_mg(const ParGrid &g, const ParBufs &B, double *z, double cdt, int iters,
                   const MGLevel *lv, int nlev, int deg, int cdeg, hipStream_t s) {
  const dim3 grid = grid_of(g.N), blk(kParBlock);
  for (int it = 0; it < iters; ++it) {
    hipLaunchKernelGGL((k_cg_apply<DIM, NC>), grid, blk, 0, s, g, B, cdt);
    hipLaunchKernelGGL(k_cg_scalars<1>, dim3(1), blk, 0, s, B.partial, (int)grid.x,
                       B.cg, 0.0, 0);
    hipLaunchKernelGGL(k_cg_update_xr<NC>, grid, blk, 0, s, g, B);
    mg_vcycle(DIM, NC, lv, nlev, B.r, z, cdt, B.cg, deg, cdeg, s);
    hipLaunchKernelGGL(k_cg_sums_rz<NC>, grid, blk, 0, s, g, B, (const double *)z);
    hipLaunchKernelGGL(k_cg_scalars<2>, dim3(1), blk, 0, s, B.partial, (int)grid.x,
                       B.cg, 0.0, 0);
    hipLaunchKernelGGL(k_cg_direction_z<NC>, grid, blk, 0, s, g, B, (const double *)z);
  }
}
}  // namespace

void par_cg_start_mg(int dim, int ncomp, const ParGrid &g, const ParBufs &B, double *zb,
                     double cdt, double rtol, int maxit, const MGLevel *lv, int nlev,
                     int deg, int coarse_deg, hipStream_t s) {
  if (dim == 2) {
    if (ncomp == 2) cg_start_mg<2, 2>(g, B, zb, cdt, rtol, maxit, lv, nlev, deg, coarse_deg, s);
    else cg_start_mg<2, 1>(g, B, zb, cdt, rtol, maxit, lv, nlev, deg, coarse_deg, s);
  } else {
    if (ncomp == 3) cg_start_mg<3, 3>(g, B, zb, cdt, rtol, maxit, lv, nlev, deg, coarse_deg, s);
    else cg_start_mg<3, 1>(g, B, zb, cdt, rtol, maxit, lv, nlev, deg, coarse_deg, s);
  }
}

void par_cg_iterate_mg(int dim, int ncomp, const ParGrid &g, const ParBufs &B, double *zb,
                       double cdt, int iters, const MGLevel *lv, int nlev, int deg,
                       int coarse_deg, hipStream_t s) {
  if (dim == 2) {
    if (ncomp == 2) cg_iterate_mg<2, 2>(g, B, zb, cdt, iters, lv, nlev, deg, coarse_deg, s);
    else cg_iterate_mg<2, 1>(g, B, zb, cdt, iters, lv, nlev, deg, coarse_deg, s);
  } else {
    if (ncomp == 3) cg_iterate_mg<3, 3>(g, B, zb, cdt, iters, lv, nlev, deg, coarse_deg, s);
    else cg_iterate_mg<3, 1>(g, B, zb, cdt, iters, lv, nlev, deg, coarse_deg, s);
  }
}

void par_cg_start(int dim, int ncomp, const ParGrid &g, const ParBufs &B,
                  double cdt, double rtol, int maxit, hipStream_t s) {
  if (dim == 2) {
    if (ncomp == 2) cg_start<2, 2>(g, B, cdt, rtol, maxit, s);
    else cg_start<2, 1>(g, B, cdt, rtol, maxit, s);
  } else {
    if (ncomp == 3) cg_start<3, 3>(g, B, cdt, rtol, maxit, s);
    else cg_start<3, 1>(g, B, cdt, rtol, maxit, s);
  }
}

void par_cg_iterate(int dim, int ncomp, const ParGrid &g, const ParBufs &B,
                    double cdt, int iters, hipStream_t s) {
  if (dim == 2) {
    if (ncomp == 2) cg_iterate<2, 2>(g, B, cdt, iters, s);
    else cg_iterate<2, 1>(g, B, cdt, iters, s);
  } else {
    if (ncomp == 3) cg_iterate<3, 3>(g, B, cdt, iters, s);
    else cg_iterate<3, 1>(g, B, cdt, iters, s);
  }
}

void par_velocity_done(int dim, const ParGrid &g, const ParBufs &B,
                       const double *U, double *out, double mu, double lambda,
                       hipStream_t s) {
  const double lam23 = lambda - 2.0 / 3.0 * mu;
  const dim3 grid = grid_of(g.N), blk(kParBlock);
  if (dim == 2) {
    hipLaunchKernelGGL(k_cell_diss<2>, grid, blk, 0, s, g, B, mu, lam23);
    hipLaunchKernelGGL(k_vel_done<2>, grid, blk, 0, s, g, B, U, out);
  } else {
    hipLaunchKernelGGL(k_cell_diss<3>, grid, blk, 0, s, g, B, mu, lam23);
    hipLaunchKernelGGL(k_vel_done<3>, grid, blk, 0, s, g, B, U, out);
  }
}

void par_energy_setup(int dim, const ParGrid &g, const ParBufs &B, double cdt,
                      double ksrc, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(k_energy_setup<2>, grid_of(g.N), dim3(kParBlock), 0, s, g, B, cdt,
                       ksrc);
  else
    hipLaunchKernelGGL(k_energy_setup<3>, grid_of(g.N), dim3(kParBlock), 0, s, g, B, cdt,
                       ksrc);
}

void par_energy_high(int dim, const ParGrid &g, const ParBufs &B, hipStream_t s) {
  (void)dim;
  const dim3 grid = grid_of(g.N);
  hipLaunchKernelGGL(k_energy_high, grid, dim3(kParBlock), 0, s, g, B);
  hipLaunchKernelGGL(k_min_final, dim3(1), dim3(kParBlock), 0, s, B.partial,
                     (int)grid.x, B.scal);
}

void par_fct(int dim, const ParGrid &g, const ParBufs &B, double dt, hipStream_t s) {
  const dim3 grid = grid_of(g.N), blk(kParBlock);
  hipLaunchKernelGGL(k_fct_w, grid, blk, 0, s, g, B);
  if (dim == 2) {
    hipLaunchKernelGGL(k_fct_ratios<2>, grid, blk, 0, s, g, B, dt);
    hipLaunchKernelGGL(k_fct_apply<2>, grid, blk, 0, s, g, B, dt);
  } else {
    hipLaunchKernelGGL(k_fct_ratios<3>, grid, blk, 0, s, g, B, dt);
    hipLaunchKernelGGL(k_fct_apply<3>, grid, blk, 0, s, g, B, dt);
  }
}

void par_finish(int dim, const ParGrid &g, const ParBufs &B, const double *U,
                const double *e, double *out, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(k_par_finish<2>, grid_of(g.N), dim3(kParBlock), 0, s, g, B, U, e,
                       out);
  else
    hipLaunchKernelGGL(k_par_finish<3>, grid_of(g.N), dim3(kParBlock), 0, s, g, B, U, e,
                       out);
}

}  // namespace ns
