// hyp_kernels.hip -- forward-Euler stage of the hyperbolic step on gfx950.
// See hyp_kernels.hpp for the sweep structure and data layout.
#include "hyp_kernels.hpp"

#include <algorithm>
#include <climits>
#include <type_traits>

namespace ns {

namespace {

enum { AP_OFF = 0 };  // aux layout: v[0..DIM-1], p, a, b, eta, Phi

template <int DIM> struct Aux {
  static constexpr int P = DIM, A = DIM + 1, B = DIM + 2, ETA = DIM + 3,
                       PHI = DIM + 4, COUNT = DIM + 5;
};

// Row width 3^DIM, processed in unrolled chunks of CH slots: the neighbour
// gathers of a chunk are issued together, while the chunk size bounds the
// registers a lane holds (and so the occupancy that hides gather latency).
#ifndef NS_CH_VISC
#define NS_CH_VISC 1
#endif
#ifndef NS_CH_LO
#define NS_CH_LO 1
#endif
#ifndef NS_CH_LIM1
#define NS_CH_LIM1 1
#endif
#ifndef NS_CH_LIM2
#define NS_CH_LIM2 1
#endif
#ifndef NS_CH_FIN
#define NS_CH_FIN 1
#endif
// 2D pass-2 search: off-diagonal P_ij kept in LDS instead of registers
#ifndef NS_LIM2_LDS
#define NS_LIM2_LDS 5
#endif
template <int DIM, int CHUNK = 9> struct Cfg {
  static constexpr int NC = DIM + 2;
  static constexpr int W = DIM == 2 ? 9 : 27;
  static constexpr int CH = CHUNK;
  static constexpr int NCH = W / CH;
  static_assert(W % CH == 0, "chunk must divide the row width");
};

// Edge arrays are sliced ELL: rows are grouped in slices of 64 (one
// wavefront) and within a slice stored slot-major, so the 64 lanes of a wave
// reading slot k touch 64 consecutive entries, and all slots of the slice
// share one contiguous block (one page) of every edge array.
template <int DIM>
__device__ __forceinline__ int64_t eidx(int k, int64_t i) {
  constexpr int W = DIM == 2 ? 9 : 27;
  return ((i >> 6) * W + k) * 64 + (i & 63);
}

// Loads of arrays that a sweep reads once per entry (graph coefficients,
// d_ij of the row): with NS_NT they carry the non-temporal hint so
// that they do not push the neighbour rows' node data out of L2.
#ifndef NS_NT
#define NS_NT 2
#endif
template <typename T>
__device__ __forceinline__ T ld_once(const T *p) {
  if constexpr (NS_NT >= 1) return __builtin_nontemporal_load(p);
  else return *p;
}
template <typename T>
__device__ __forceinline__ void st_once(T *p, T v) {
  if constexpr (NS_NT >= 2) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Neighbours of row i (in its box mesh); the rows of a workgroup belong to
// one mesh, so the mesh's geometry is a uniform (scalar) load.
// blk is the row block (kBlock rows) of i, uniform over the workgroup.
template <int DIM, typename LT>
__device__ __forceinline__ BoxNbr<DIM> block_nbr(const DevGraphT<LT> &G, uint32_t blk,
                                                 int64_t i) {
  return BoxNbr<DIM>(&G.geo[G.seg ? geo_ld(&G.seg[blk]) : 0], i);
}
// Same for a row that is not the lane's own (work-list entries).
template <int DIM, typename LT>
__device__ __forceinline__ BoxNbr<DIM> row_nbr(const DevGraphT<LT> &G, int64_t i) {
  return BoxNbr<DIM>(&G.geo[G.seg ? G.seg[i / kBlock] : 0], i);
}

__device__ __forceinline__ int64_t row_id() {
  return (int64_t)blockIdx.x * kBlock + threadIdx.x;
}

__device__ __forceinline__ int64_t plain_id() {
  return (int64_t)blockIdx.x * kBlock + threadIdx.x;
}

// Member of a pack that row i belongs to (0 for one mesh).
template <typename LT>
__device__ __forceinline__ int member(const StageArgsT<LT> &A, int64_t i) {
  return A.seg ? A.seg[i / kBlock] : 0;
}

// FP64 value to the storage type: nearest, upwards (graph viscosity stays an
// upper bound) or downwards (a limiter coefficient stays feasible)
template <typename LT> __device__ __forceinline__ LT to_lt(double x) { return (LT)x; }
template <typename LT> __device__ __forceinline__ LT to_lt_up(double x) {
  if constexpr (sizeof(LT) == 4) return __double2float_ru(x);
  else return x;
}
template <typename LT> __device__ __forceinline__ LT to_lt_down(double x) {
  if constexpr (sizeof(LT) == 4) return __double2float_rd(x);
  else return x;
}

// Node vectors in the paired layout of node_layout.hpp: one 16-byte (FP32:
// 8-byte) access per component pair.
template <typename T> struct Pair2;
template <> struct Pair2<double> { using type = double2; };
template <> struct Pair2<float> { using type = float2; };

template <int NC, typename T>
__device__ __forceinline__ void load_state(const T *__restrict__ U,
                                           int64_t N, int64_t i, double *u) {
  using T2 = typename Pair2<T>::type;
#pragma unroll
  for (int p = 0; p < NC / 2; ++p) {
    const T2 v = *reinterpret_cast<const T2 *>(U + 2 * p * N + 2 * i);
    u[2 * p] = v.x;
    u[2 * p + 1] = v.y;
  }
  if constexpr (NC & 1) u[NC - 1] = U[(NC - 1) * N + i];
}

template <int NC, typename T>
__device__ __forceinline__ void store_state(T *__restrict__ U, int64_t N, int64_t i,
                                            const T *u) {
  using T2 = typename Pair2<T>::type;
#pragma unroll
  for (int p = 0; p < NC / 2; ++p) {
    T2 v;
    v.x = u[2 * p];
    v.y = u[2 * p + 1];
    *reinterpret_cast<T2 *>(U + 2 * p * N + 2 * i) = v;
  }
  if constexpr (NC & 1) U[(NC - 1) * N + i] = u[NC - 1];
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

// Velocity and pressure of a conserved state.  k_prim stores them per node
// for k_visc without the indicator; the sweeps that gather a neighbour's
// whole state anyway compute them with this same function instead.
template <int DIM>
__device__ __forceinline__ double vel_pres(const Gas &g, const double *u, double *v,
                                           double &p) {
  const double ir = fast_rcp(u[0]);
  double m2 = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) m2 += u[1 + k] * u[1 + k];
  const double eps = u[DIM + 1] - 0.5 * m2 * ir;  // rho e
  p = g.gm1 * eps;
#pragma unroll
  for (int k = 0; k < DIM; ++k) v[k] = u[1 + k] * ir;
  return eps;
}

// ---------------------------------------------------------------------------
// VP: also store v and p (read only by k_visc without the indicator; the
// other sweeps compute them from the states they gather).
template <int DIM, bool VP>
__device__ __forceinline__ void prim_row(int64_t N, const double *__restrict__ U,
                                         double *__restrict__ aux, const Gas &g,
                                         int64_t i) {
  if (i >= N) return;
  using X = Aux<DIM>;
  double u[DIM + 2], v[DIM], p;
  load_state<DIM + 2>(U, N, i, u);
  const double r = u[0];
  const double eps = vel_pres<DIM>(g, u, v, p);
  const double a = sqrt(g.gamma * p * (1.0 / r));
  // log p = log(gamma - 1) + log(rho e): one logarithm serves the specific
  // entropy and p^(-(gamma-1)/(2 gamma)) = exp(-ex log p)
  const double le = log(eps);
  const double s = le - g.gamma * log(r);
  if constexpr (VP) {
#pragma unroll
    for (int k = 0; k < DIM; ++k) aux[k * N + i] = v[k];
    aux[X::P * N + i] = p;
  }
  aux[X::A * N + i] = a;
  aux[X::B * N + i] = a * exp(-g.ex * (g.lgm1 + le));
  aux[X::ETA * N + i] = -r * s;
  aux[X::PHI * N + i] = exp(s);
}

template <int DIM, bool VP>
__global__ __launch_bounds__(kBlock) void k_prim(int64_t N,
                                                 const double *__restrict__ U,
                                                 double *__restrict__ aux,
                                                 Gas g) {
  prim_row<DIM, VP>(N, U, aux, g, plain_id());
}

// ---------------------------------------------------------------------------
// Graph viscosity d^L_ij (j > i, stored at (i,j) and (j,i)) and alpha_i.
// The column indices of the row follow from its place in the box mesh; each
// chunk of slots gathers its neighbour data unconditionally (absent entries
// read row i itself) so that the loads of a chunk are in flight together, and the
// arithmetic is predicated on the entry being present.
template <int DIM, int IND, int SEV, typename LT>
__device__ __forceinline__ void visc_row(const DevGraphT<LT> &G,
                                         const double *__restrict__ U,
                                         const double *__restrict__ aux,
                                         LT *__restrict__ d, LT *__restrict__ alpha,
                                         const Gas &g, uint32_t blk, int64_t i) {
  using X = Aux<DIM>;
  using C = Cfg<DIM, NS_CH_VISC>;
  constexpr int NC = C::NC;
  const int64_t N = G.N;
  if (i >= N) return;
  BoxNbr<DIM> jv = block_nbr<DIM>(G, blk, i);
  double vi[DIM], pi;
  const double ai = aux[X::A * N + i], bi = aux[X::B * N + i];
  const bool wall_i = G.wall[i] != 0;
  double etap[NC];
  if constexpr (IND == 0) {
    double ui[NC];
    load_state<NC>(U, N, i, ui);
    const double eps = vel_pres<DIM>(g, ui, vi, pi);  // rho e
    const double ri = ui[0];
    double m2 = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      m2 += ui[1 + k] * ui[1 + k];
      etap[1 + k] = ui[1 + k];
    }
    const double s = -aux[X::ETA * N + i] / ri;
    const double ie = 1.0 / eps;
    etap[0] = g.gamma - s - m2 / (2.0 * ri * eps);
#pragma unroll
    for (int k = 0; k < DIM; ++k) etap[1 + k] *= ie;
    etap[NC - 1] = -ri * ie;
  } else {
#pragma unroll
    for (int k = 0; k < DIM; ++k) vi[k] = aux[k * N + i];
    pi = aux[X::P * N + i];
  }
  double num = 0.0, den = 0.0, scl = 0.0;
#pragma unroll
  for (int ch = 0; ch < C::NCH; ++ch) {
    jv.fence();
    double c[C::CH][DIM], vj[C::CH][DIM], pj[C::CH], aj[C::CH], bj[C::CH];
    double uj[C::CH][IND == 0 ? NC : 1], etaj[C::CH];
    int32_t jc[C::CH];
#pragma unroll
    for (int kk = 0; kk < C::CH; ++kk) {
      const int k = ch * C::CH + kk;
      jc[kk] = jv[k];
      const int64_t js = jc[kk] >= 0 ? jc[kk] : i;
      jv.grad(k, c[kk]);
      aj[kk] = aux[X::A * N + js];
      bj[kk] = aux[X::B * N + js];
      if constexpr (IND == 0) {
        // the indicator needs the whole state; v and p follow from it
        load_state<NC>(U, N, js, uj[kk]);
        etaj[kk] = aux[X::ETA * N + js];
      } else {
#pragma unroll
        for (int q = 0; q < DIM; ++q) vj[kk][q] = aux[q * N + js];
        pj[kk] = aux[X::P * N + js];
      }
    }
#pragma unroll
    for (int kk = 0; kk < C::CH; ++kk) {
      const int k = ch * C::CH + kk;
      const int32_t j = jc[kk];
      if (j < 0) continue;
      if constexpr (IND == 0) vel_pres<DIM>(g, uj[kk], vj[kk], pj[kk]);
      double c2 = 0.0;
#pragma unroll
      for (int q = 0; q < DIM; ++q) c2 += c[kk][q] * c[kk][q];
      const double cn = fast_sqrt(c2);
      if constexpr (IND == 0) {
        double fc[NC], vc = 0.0;
#pragma unroll
        for (int q = 0; q < DIM; ++q) vc += vj[kk][q] * c[kk][q];
        flux_dot<DIM>(uj[kk], vj[kk], pj[kk], c[kk], fc);
        double t = etaj[kk] * vc;
#pragma unroll
        for (int q = 0; q < NC; ++q) t -= etap[q] * fc[q];
        num += t;
        den += fabs(t);
        scl += cn * aj[kk] * (uj[kk][0] + fabs(etaj[kk]));
      }
      if (j > i) {
        const int64_t e = eidx<DIM>(k, i);
        const double icn = fast_rcp(cn);
        double uL = 0.0, uR = 0.0;
#pragma unroll
        for (int q = 0; q < DIM; ++q) {
          uL += vi[q] * c[kk][q] * icn;
          uR += vj[kk][q] * c[kk][q] * icn;
        }
        double dij = lambda_max<SEV>(g, uL, pi, ai, bi, uR, pj[kk], aj[kk], bj[kk]) * cn;
        const int kt = tslot<DIM>(k);
        const int64_t et = eidx<DIM>(kt, j);
        if (wall_i) {
          // both ends may be on the wall: c_ji != -c_ij, take both directions
          double ct[DIM];
          grad_transposed<DIM>(k, c[kk], ct);
          double ct2 = 0.0;
#pragma unroll
          for (int q = 0; q < DIM; ++q) ct2 += ct[q] * ct[q];
          const double ctn = fast_sqrt(ct2);
          const double ictn = fast_rcp(ctn);
          double uLt = 0.0, uRt = 0.0;
#pragma unroll
          for (int q = 0; q < DIM; ++q) {
            uLt += vj[kk][q] * ct[q] * ictn;
            uRt += vi[q] * ct[q] * ictn;
          }
          dij = fmax(dij, lambda_max<SEV>(g, uLt, pj[kk], aj[kk], bj[kk], uRt, pi, ai, bi) * ctn);
        }
        const LT dst = to_lt_up<LT>(dij);
        st_once(&d[e], dst);
        st_once(&d[et], dst);
      }
    }
  }
  // (an isolated node -- a padding row of a pack -- has den = scl = 0)
  if constexpr (IND == 0)
    alpha[i] = to_lt<LT>(den + scl > 0.0 ? fabs(num) / (den + 1e-2 * scl) : 0.0);
  else if constexpr (IND == 1) alpha[i] = LT(1);
  else alpha[i] = LT(0);
}

// FP32 evaluation (mixed-precision mode with FP32 arithmetic, entropy
// indicator, gamma = 7/5): the same quantities as visc_row with the
// velocities, pressures, |c_ij|, the fluxes and commutator terms of the
// indicator and lambda_max in FP32.  d_ij = lambda |c_ij| (1 + 2^-16) rounded
// up stays an upper bound of the FP64 value where lambda_max_f32 certifies
// its error; on the other entries (and for a padding row) lambda_max is
// evaluated in FP64 from the FP64 state, as in visc_row.
template <int DIM>
__device__ __forceinline__ float vel_pres_f(float gm1, const float *u, float *v, float &p) {
  const float ir = __builtin_amdgcn_rcpf(u[0]);
  float m2 = 0.0f;
#pragma unroll
  for (int k = 0; k < DIM; ++k) m2 += u[1 + k] * u[1 + k];
  const float eps = u[DIM + 1] - 0.5f * m2 * ir;
  p = gm1 * eps;
#pragma unroll
  for (int k = 0; k < DIM; ++k) v[k] = u[1 + k] * ir;
  return eps;
}

template <int DIM, typename LT>
__device__ __forceinline__ void visc_row_f32(const DevGraphT<LT> &G,
                                             const double *__restrict__ U,
                                             const double *__restrict__ aux,
                                             LT *__restrict__ d, LT *__restrict__ alpha,
                                             const Gas &g, uint32_t blk, int64_t i) {
  using X = Aux<DIM>;
  using C = Cfg<DIM, NS_CH_VISC>;
  constexpr int NC = C::NC;
  const int64_t N = G.N;
  if (i >= N) return;
  BoxNbr<DIM> jv = block_nbr<DIM>(G, blk, i);
  const float gm1 = (float)g.gm1;
  double ui[NC], vi[DIM], pi;
  load_state<NC>(U, N, i, ui);
  const double eps_i = vel_pres<DIM>(g, ui, vi, pi);  // FP64 (the fallback needs it)
  const double ai = aux[X::A * N + i], bi = aux[X::B * N + i];
  const bool wall_i = G.wall[i] != 0;
  // entropy variables of row i, formed in FP64 once per row
  float etap[NC], vif[DIM];
  {
    double m2 = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) m2 += ui[1 + k] * ui[1 + k];
    const double s = -aux[X::ETA * N + i] / ui[0];
    const double ie = 1.0 / eps_i;
    etap[0] = (float)(g.gamma - s - m2 / (2.0 * ui[0] * eps_i));
#pragma unroll
    for (int k = 0; k < DIM; ++k) {
      etap[1 + k] = (float)(ui[1 + k] * ie);
      vif[k] = (float)vi[k];
    }
    etap[NC - 1] = (float)(-ui[0] * ie);
  }
  const float pif = (float)pi, aif = (float)ai, bif = (float)bi;
  float num = 0.0f, den = 0.0f, scl = 0.0f;
#pragma unroll
  for (int ch = 0; ch < C::NCH; ++ch) {
    jv.fence();
    double c[C::CH][DIM], uj[C::CH][NC], aj[C::CH], bj[C::CH], etaj[C::CH];
    int32_t jc[C::CH];
#pragma unroll
    for (int kk = 0; kk < C::CH; ++kk) {
      const int k = ch * C::CH + kk;
      jc[kk] = jv[k];
      const int64_t js = jc[kk] >= 0 ? jc[kk] : i;
      jv.grad(k, c[kk]);
      aj[kk] = aux[X::A * N + js];
      bj[kk] = aux[X::B * N + js];
      load_state<NC>(U, N, js, uj[kk]);
      etaj[kk] = aux[X::ETA * N + js];
    }
#pragma unroll
    for (int kk = 0; kk < C::CH; ++kk) {
      const int k = ch * C::CH + kk;
      const int32_t j = jc[kk];
      if (j < 0) continue;
      float cf[DIM], ujf[NC], vjf[DIM], pjf;
#pragma unroll
      for (int q = 0; q < DIM; ++q) cf[q] = (float)c[kk][q];
#pragma unroll
      for (int q = 0; q < NC; ++q) ujf[q] = (float)uj[kk][q];
      vel_pres_f<DIM>(gm1, ujf, vjf, pjf);
      float c2 = 0.0f, vc = 0.0f;
#pragma unroll
      for (int q = 0; q < DIM; ++q) {
        c2 += cf[q] * cf[q];
        vc += vjf[q] * cf[q];
      }
      const float cn = __builtin_amdgcn_sqrtf(c2);
      {
        // commutator term of the indicator: eta_j (v_j.c) - eta'(U_i).f(U_j) c
        const float etajf = (float)etaj[kk];
        float t = etajf * vc;
        t -= etap[0] * (ujf[0] * vc);
#pragma unroll
        for (int q = 0; q < DIM; ++q) t -= etap[1 + q] * (ujf[1 + q] * vc + pjf * cf[q]);
        t -= etap[NC - 1] * (vc * (ujf[NC - 1] + pjf));
        num += t;
        den += fabsf(t);
        scl += cn * (float)aj[kk] * (ujf[0] + fabsf(etajf));
      }
      if (j > i) {
        const int64_t e = eidx<DIM>(k, i);
        const int kt = tslot<DIM>(k);
        const int64_t et = eidx<DIM>(kt, j);
        const float icn = __builtin_amdgcn_rcpf(cn);
        float uL = 0.0f, uR = 0.0f;
#pragma unroll
        for (int q = 0; q < DIM; ++q) {
          uL += vif[q] * cf[q];
          uR += vjf[q] * cf[q];
        }
        bool ok;
        const float lam = lambda_max_f32(g, uL * icn, pif, aif, bif, uR * icn, pjf,
                                         (float)aj[kk], (float)bj[kk], &ok);
        double dij = (double)lam * (double)cn * kLambdaInflate;
        double vj[DIM], pj;
        if (!ok || wall_i) vel_pres<DIM>(g, uj[kk], vj, pj);
        if (!ok) {  // FP64, as visc_row
          double c2d = 0.0;
#pragma unroll
          for (int q = 0; q < DIM; ++q) c2d += c[kk][q] * c[kk][q];
          const double cnd = fast_sqrt(c2d), icnd = fast_rcp(cnd);
          double uLd = 0.0, uRd = 0.0;
#pragma unroll
          for (int q = 0; q < DIM; ++q) {
            uLd += vi[q] * c[kk][q] * icnd;
            uRd += vj[q] * c[kk][q] * icnd;
          }
          dij = lambda_max<1>(g, uLd, pi, ai, bi, uRd, pj, aj[kk], bj[kk]) * cnd;
        }
        if (wall_i) {
          // both ends may be on the wall: c_ji != -c_ij, take both
          // directions (the transposed one in FP64: walls are a thin set)
          double ct[DIM];
          grad_transposed<DIM>(k, c[kk], ct);
          double ct2 = 0.0;
#pragma unroll
          for (int q = 0; q < DIM; ++q) ct2 += ct[q] * ct[q];
          const double ctn = fast_sqrt(ct2);
          const double ictn = fast_rcp(ctn);
          double uLt = 0.0, uRt = 0.0;
#pragma unroll
          for (int q = 0; q < DIM; ++q) {
            uLt += vj[q] * ct[q] * ictn;
            uRt += vi[q] * ct[q] * ictn;
          }
          dij = fmax(dij, lambda_max<1>(g, uLt, pj, aj[kk], bj[kk], uRt, pi, ai, bi) * ctn);
        }
        const LT dst = to_lt_up<LT>(dij);
        st_once(&d[e], dst);
        st_once(&d[et], dst);
      }
    }
  }
  alpha[i] = to_lt<LT>(den + scl > 0.0f ? fabsf(num) / (den + 1e-2f * scl) : 0.0f);
}

template <int DIM, typename LT>
__global__ __launch_bounds__(kBlock) void k_visc_f32(DevGraphT<LT> G,
                                                     const double *__restrict__ U,
                                                     const double *__restrict__ aux,
                                                     LT *__restrict__ d,
                                                     LT *__restrict__ alpha, Gas g) {
  visc_row_f32<DIM, LT>(G, U, aux, d, alpha, g, blockIdx.x, row_id());
}

template <int DIM, int IND, int SEV, typename LT>
__global__ __launch_bounds__(kBlock) void k_visc(DevGraphT<LT> G,
                                                 const double *__restrict__ U,
                                                 const double *__restrict__ aux,
                                                 LT *__restrict__ d,
                                                 LT *__restrict__ alpha,
                                                 Gas g) {
  visc_row<DIM, IND, SEV, LT>(G, U, aux, d, alpha, g, blockIdx.x, row_id());
}

// ---------------------------------------------------------------------------
// Time step: per-block min of m_i / (2 sum_{j != i} d_ij) = -m_i / (2 d_ii).
// (every thread of the workgroup calls it: it ends in a workgroup reduction)
template <int DIM, typename LT>
__device__ __forceinline__ void dt_partial_blk(const DevGraphT<LT> &G,
                                               const LT *__restrict__ d,
                                               double *__restrict__ partial, uint32_t blk,
                                               int64_t i) {
  using C = Cfg<DIM>;
  const int64_t N = G.N;
  double r = INFINITY;
  if (i < N) {
    double dsum = 0.0;
    BoxNbr<DIM> jv = block_nbr<DIM>(G, blk, i);
#pragma unroll
    for (int k = 0; k < C::W; ++k) {
      if (k == C::W / 2) continue;  // the diagonal
      const int64_t e = eidx<DIM>(k, i);
      const int32_t j = jv[k];
      const double v = d[e];  // absent entries hold 0
      if (j >= 0 && j != i) dsum += v;
    }
    r = G.mi[i] / (2.0 * dsum);
  }
  r = block_min(r);
  if (threadIdx.x == 0) partial[blk] = r;
}

template <int DIM, typename LT>
__global__ __launch_bounds__(kBlock) void k_dt_partial(DevGraphT<LT> G,
                                                       const LT *__restrict__ d,
                                                       double *__restrict__ partial) {
  dt_partial_blk<DIM, LT>(G, d, partial, blockIdx.x, row_id());
}

// One workgroup per member of a pack: the member's workgroups are
// [mblk[m], mblk[m+1]); min is exact, so tau equals the one-mesh value.
__global__ __launch_bounds__(1024) void k_dt_final_members(const double *__restrict__ partial,
                                                           const int32_t *__restrict__ mblk,
                                                           double cfl,
                                                           double *__restrict__ tau) {
  __shared__ double red[16];
  const int m = blockIdx.x;
  double v = INFINITY;
  for (int64_t b = mblk[m] + threadIdx.x; b < mblk[m + 1]; b += 1024) v = fmin(v, partial[b]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 16; ++w) v = fmin(v, red[w]);
    tau[m] = cfl * v;
  }
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
// Low-order update, bounds and high-order flux (stored divided by m_i).
// first: the lane that empties the limiter work lists of this stage
template <int DIM, typename LT>
__device__ __forceinline__ void lo_row(const DevGraphT<LT> &G, const StageArgsT<LT> &A,
                                       const Gas &g, uint32_t blk, int64_t i, bool first) {
  using X = Aux<DIM>;
  using C = Cfg<DIM, NS_CH_LO>;
  constexpr int NC = C::NC;
  const int64_t N = G.N;
  if (first) {
    A.qcnt[0] = 0;
    A.qcnt[1] = 0;
    if (A.drow) A.qcnt[2] = 0;
  }
  if (i >= N) return;
  const double *__restrict__ U = A.U;
  const double *__restrict__ aux = A.aux;
  const LT *__restrict__ alpha = A.alpha;
  const LT *__restrict__ dd = A.d;
  BoxNbr<DIM> jv = block_nbr<DIM>(G, blk, i);
  double ui[NC], vi[DIM], pi;
  load_state<NC>(U, N, i, ui);
  vel_pres<DIM>(g, ui, vi, pi);
  const double ali = alpha[i];
  const int mem = member(A, i);
  const double tau = A.tau[mem];
  double acc[NC], fh[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) { acc[q] = 0.0; fh[q] = 0.0; }
  double rmin = ui[0], rmax = ui[0], phimin = aux[X::PHI * N + i], dsum = 0.0;
  // sum_j (f(U_j) - f(U_i)) c_ij: the row's own flux enters once, against
  // the sum of c_ij over the off-diagonal entries (only its density
  // component is needed entry by entry, for the bar states)
  double csum[DIM];
#pragma unroll
  for (int k = 0; k < DIM; ++k) csum[k] = 0.0;
  double vci = 0.0;  // v_i . c_ij of the current entry
#pragma unroll
  for (int ch = 0; ch < C::NCH; ++ch) {
    jv.fence();
    double c[C::CH][DIM], uj[C::CH][NC], phij[C::CH], alj[C::CH], dij[C::CH];
    int32_t jc[C::CH];
#pragma unroll
    for (int kk = 0; kk < C::CH; ++kk) {
      const int k = ch * C::CH + kk;
      const int64_t e = eidx<DIM>(k, i);
      jc[kk] = jv[k];
      const int64_t js = jc[kk] >= 0 ? jc[kk] : i;
      jv.grad(k, c[kk]);
      load_state<NC>(U, N, js, uj[kk]);  // v and p follow from it
      phij[kk] = aux[X::PHI * N + js];
      alj[kk] = alpha[js];
      dij[kk] = ld_once(&dd[e]);
    }
#pragma unroll
    for (int kk = 0; kk < C::CH; ++kk) {
      const int32_t j = jc[kk];
      if (j < 0) continue;
      if (j == i) {
        double fci[NC];
        flux_dot<DIM>(ui, vi, pi, c[kk], fci);
#pragma unroll
        for (int q = 0; q < NC; ++q) fh[q] -= fci[q];
        continue;
      }
      vci = 0.0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) {
        vci += vi[k] * c[kk][k];
        csum[k] += c[kk][k];
      }
      double fcj[NC], vj[DIM], pj;
      vel_pres<DIM>(g, uj[kk], vj, pj);
      flux_dot<DIM>(uj[kk], vj, pj, c[kk], fcj);
      const double dk = dij[kk];
      // density of the bar state (eq. bar_state) for the local bounds
      const double rbar = 0.5 * (ui[0] + uj[kk][0]) - (fcj[0] - ui[0] * vci) * fast_rcp(2.0 * dk);
      rmin = fmin(rmin, rbar);
      rmax = fmax(rmax, rbar);
      phimin = fmin(phimin, phij[kk]);
      const double dH = 0.5 * (ali + alj[kk]) * dk;
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        const double du = uj[kk][q] - ui[q];
        acc[q] += dk * du - fcj[q];
        fh[q] += -fcj[q] + dH * du;
      }
      dsum += dk;
    }
  }
  {
    double fcs[NC];
    flux_dot<DIM>(ui, vi, pi, csum, fcs);
#pragma unroll
    for (int q = 0; q < NC; ++q) acc[q] += fcs[q];
  }
  const double rmi = G.rmi[i];
  const double tm = tau * rmi;
  double ul[NC];
  LT fs[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    ul[q] = ui[q] + tm * acc[q];
    fs[q] = to_lt<LT>(fh[q] * rmi);
  }
  store_state<NC>(A.UL, N, i, ul);
  if constexpr (DIM == 3) {
    // alpha_i beside F^H's fifth component: a neighbour's F^H and alpha come
    // in three 16-byte loads in the limiter sweeps
    LT f6[NC + 1];
#pragma unroll
    for (int q = 0; q < NC; ++q) f6[q] = fs[q];
    f6[NC] = alpha[i];
    store_state<NC + 1>(A.FH, N, i, f6);
  } else {
    store_state<NC>(A.FH, N, i, fs);
  }
  if (A.check_cfl && tau > G.mi[i] / (2.0 * dsum)) A.flags[4 * mem] = 1;
  if (A.check_low) {
    double m2 = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) m2 += ul[1 + k] * ul[1 + k];
    if (!(ul[0] > 0.0) || !(ul[NC - 1] - 0.5 * m2 / ul[0] > 0.0)) A.flags[4 * mem + 3] = 1;
  }
  const double r = G.rrel[i];
  const double bv[3] = {(1.0 - r) * rmin, (1.0 + r) * rmax, (1.0 - r) * phimin};
  store_state<3>(A.bnds, N, i, bv);
}

template <int DIM, typename LT>
__global__ __launch_bounds__(kBlock) void k_lo(DevGraphT<LT> G, StageArgsT<LT> A, Gas g) {
  const int64_t i = row_id();
  lo_row<DIM, LT>(G, A, g, blockIdx.x, i, i == 0);
}

// P_ij = tau/(m_i lambda_i) (b_ij F_j - b_ji F_i + (dH - d)(U_j - U_i)) with
// b_ij = -m_ij/m_j, b_ji = -m_ij/m_i (Sec. 3.3); with Fs = F^H/m stored:
// P_ij = tau (|I(i)|-1)/m_i (m_ij (Fs_i - Fs_j) + (dH - d)(U_j - U_i)).
template <int DIM>
struct RowCtx {
  static constexpr int NC = DIM + 2;
  double ui[NC], fi[NC];
  double ali, coef;
};

template <int DIM, typename LT>
__device__ __forceinline__ void load_row(const DevGraphT<LT> &G, const StageArgsT<LT> &A,
                                         int64_t i, double tau, RowCtx<DIM> &R) {
  constexpr int NC = DIM + 2;
  const int64_t N = G.N;
  load_state<NC>(A.U, N, i, R.ui);
  if constexpr (DIM == 3) {
    double f6[NC + 1];
    load_state<NC + 1>(A.FH, N, i, f6);  // F^H / m_i and alpha_i
#pragma unroll
    for (int q = 0; q < NC; ++q) R.fi[q] = f6[q];
    R.ali = f6[NC];
  } else {
    load_state<NC>(A.FH, N, i, R.fi);
    R.ali = A.alpha[i];
  }
  R.coef = tau * G.crm[i];
}

// Neighbour data entering P_ij, gathered unconditionally (absent entries
// read row i itself) so that a chunk's loads are in flight together.
template <int DIM>
struct PIn {
  static constexpr int NC = DIM + 2;
  double u[NC], f[NC], al, d, m;
};

template <int DIM, typename LT>
__device__ __forceinline__ void gather_P(const DevGraphT<LT> &G, const StageArgsT<LT> &A,
                                         int64_t e, int64_t js, double mij, PIn<DIM> &x) {
  constexpr int NC = DIM + 2;
  const int64_t N = G.N;
  load_state<NC>(A.U, N, js, x.u);
  if constexpr (DIM == 3) {
    double f6[NC + 1];
    load_state<NC + 1>(A.FH, N, js, f6);  // F^H / m_j and alpha_j
#pragma unroll
    for (int q = 0; q < NC; ++q) x.f[q] = f6[q];
    x.al = f6[NC];
  } else {
    load_state<NC>(A.FH, N, js, x.f);
    x.al = A.alpha[js];
  }
  x.d = ld_once(&A.d[e]);
  x.m = mij;
}

template <int DIM>
__device__ __forceinline__ void make_P(const RowCtx<DIM> &R, const PIn<DIM> &x,
                                       double *P) {
#pragma clang fp contract(off)  // the same bits in every kernel (k_lim2 MODE 4)
  constexpr int NC = DIM + 2;
  const double dH = 0.5 * (R.ali + x.al) * x.d;
#pragma unroll
  for (int q = 0; q < NC; ++q)
    P[q] = R.coef * (x.m * (R.fi[q] - x.f[q]) + (dH - x.d) * (x.u[q] - R.ui[q]));
}

template <int DIM, typename LT>
__device__ __forceinline__ void compute_P(const DevGraphT<LT> &G, const StageArgsT<LT> &A,
                                          const RowCtx<DIM> &R, int64_t e,
                                          int32_t j, double mij, double *P) {
  PIn<DIM> x;
  gather_P<DIM>(G, A, e, j, mij, x);
  make_P<DIM>(R, x, P);
}

template <int DIM, typename LT>
__device__ __forceinline__ void finish(const DevGraphT<LT> &G, const StageArgsT<LT> &A,
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
  if (!(w[0] > 0.0) || !(eps > 0.0)) A.flags[4 * member(A, i) + 1] = 1;
  store_state<NC>(A.out, N, i, w);
}

struct Bounds {
  double rmin, rmax, pmin, pmin5;
};

template <typename LT>
__device__ __forceinline__ Bounds load_bounds(const StageArgsT<LT> &A, int64_t N,
                                              int64_t i) {
  Bounds b;
  double bv[3];
  load_state<3>(A.bnds, N, i, bv);  // (rho_min, rho_max) in one load
  b.rmin = bv[0];
  b.rmax = bv[1];
  b.pmin = bv[2];
  const double p2 = b.pmin * b.pmin;
  b.pmin5 = p2 * p2 * b.pmin;
  return b;
}

// Limiter line search for every off-diagonal entry of the row.  The cheap
// part (density limit, entropy test at that limit and at 0) runs in the
// row sweep, which stores l = l_rho; entries whose entropy bound cuts inside
// (0, l_rho) are appended to the work list and their root is found by
// k_root.  In a sweep such entries are rare but scattered: solved in place,
// a few lanes would hold their whole wavefront for the length of a root
// search, and the root finder's registers would lower the sweep's occupancy.
template <int DIM, int SEV>
__device__ __forceinline__ int limit_fast(const Gas &g, const double *u,
                                          const double *P, const Bounds &b,
                                          double *l) {
#pragma clang fp contract(off)  // the same bits in every kernel (k_lim2 MODE 4)
  double lr;
  if (P[0] > 0.0) lr = (b.rmax - u[0]) / P[0];
  else if (P[0] < 0.0) lr = (b.rmin - u[0]) / P[0];
  else lr = 1.0;
  lr = fmin(fmax(lr, 0.0), 1.0);
  *l = lr;
  if (entropy_ok<DIM, SEV>(g, u, P, lr, b.pmin, b.pmin5)) return 0;
  if (!entropy_ok<DIM, SEV>(g, u, P, 0.0, b.pmin, b.pmin5)) { *l = 0.0; return 0; }
  return 1;  // root of psi in (0, lr) still to be found
}

template <int DIM, int SEV, typename LT>
__device__ __forceinline__ void lim1_row(const DevGraphT<LT> &G, const StageArgsT<LT> &A,
                                         const Gas &g, uint32_t blk, int64_t i) {
#pragma clang fp contract(off)  // the same bits as k_lim2 MODE 4
  using C = Cfg<DIM, NS_CH_LIM1>;
  constexpr int NC = C::NC;
  const int64_t N = G.N;
  if (i >= N) return;
  BoxNbr<DIM> jv = block_nbr<DIM>(G, blk, i);
  RowCtx<DIM> R;
  load_row<DIM>(G, A, i, A.tau[member(A, i)], R);
  double ul[NC];
  load_state<NC>(A.UL, N, i, ul);
  const Bounds b = load_bounds(A, N, i);
  LT *__restrict__ lt1 = A.lt1;
  uint32_t slow = 0;
#pragma unroll
  for (int ch = 0; ch < C::NCH; ++ch) {
    jv.fence();
    PIn<DIM> x[C::CH];
    int32_t jc[C::CH];
#pragma unroll
    for (int kk = 0; kk < C::CH; ++kk) {
      const int k = ch * C::CH + kk;
      jc[kk] = jv[k];
      if (k == C::W / 2) continue;  // the diagonal has no P
      gather_P<DIM>(G, A, eidx<DIM>(k, i), jc[kk] >= 0 ? jc[kk] : i, jv.mass(k), x[kk]);
    }
#pragma unroll
    for (int kk = 0; kk < C::CH; ++kk) {
      const int k = ch * C::CH + kk;
      if (jc[kk] < 0 || jc[kk] == i) continue;
      double P[NC], l;
      make_P<DIM>(R, x[kk], P);
      if (limit_fast<DIM, SEV>(g, ul, P, b, &l)) slow |= 1u << k;
      st_once(&lt1[eidx<DIM>(k, i)], to_lt_down<LT>(l));
    }
  }
  if (slow) {
    uint32_t t = atomicAdd(&A.qcnt[0], (uint32_t)__builtin_popcount(slow));
    while (slow) {
      const int k = __builtin_ctz(slow);
      slow &= slow - 1;
      A.q[t++] = (uint32_t)eidx<DIM>(k, i);
    }
  }
}

template <int DIM, int SEV, typename LT>
__global__ __launch_bounds__(kBlock) void k_lim1(DevGraphT<LT> G, StageArgsT<LT> A, Gas g) {
  lim1_row<DIM, SEV, LT>(G, A, g, blockIdx.x, row_id());
}

// MODE 0: convex, pass-1 update + pass-2 line search; 1: convex with one
// pass, final; 2: l = 1 (unlimited high order), final; 3: convex, pass-1
// update only (3D: the pass-2 search is k_lim2b, since both in one kernel
// need more registers than a SIMD lane has); 4: MODE 0 with the pass-1 line
// searches in the same sweep (2D, replaces k_lim1).
//
// MODE 4: for every entry the row runs both line searches of the pair --
// its own on P_ij from its U^L and bounds, and the neighbour's on P_ji from
// the neighbour's, with P_ji formed from the same operands in the same
// order as the neighbour's row forms it -- so the two rows obtain the same
// l_ij = min(l~_ij, l~_ji) without a sweep storing l~ in between.  The own
// search is still stored in lt1 (a deferred neighbour reads it).  Where
// either search of a pair needs the root of the entropy bound, both rows of
// the pair are deferred: the own entries go to the pass-1 work list as in
// k_lim1, the row to the deferred list, and k_lim2_rows completes it with
// MODE 0 once k_root has solved the list.
template <int DIM, int MODE, int SEV, typename LT>
__device__ __forceinline__ void lim2_row(const DevGraphT<LT> &G, const StageArgsT<LT> &A,
                                         const Gas &g, uint32_t blk, int64_t i) {
  // no fused multiply-adds of the compiler's choosing: MODE 0 and MODE 4
  // must give the same bits (the persistent steps run MODE 0 throughout)
#pragma clang fp contract(off)
  using C = Cfg<DIM, NS_CH_LIM2>;
  constexpr int NC = C::NC;
  const int64_t N = G.N;
  if (i >= N) return;
  const LT *__restrict__ lt1 = A.lt1;
  BoxNbr<DIM> colk = block_nbr<DIM>(G, blk, i);
  RowCtx<DIM> R;
  const double tau = A.tau[member(A, i)];
  load_row<DIM>(G, A, i, tau, R);
  const double lam = 1.0 / G.lfac[i];
  double u1[NC];
  load_state<NC>(A.UL, N, i, u1);
  constexpr bool BOTH = MODE == 4;  // both pass-1 searches of every pair here
  double ul[BOTH ? NC : 1];
  Bounds bi{};
  uint32_t slow1 = 0;
  bool defer = false;
  if constexpr (BOTH) {
#pragma unroll
    for (int q = 0; q < NC; ++q) ul[q] = u1[q];
    bi = load_bounds(A, N, i);
  }
  // 2D: the row's P_ij and l_ij stay for the pass-2 search: the P of the
  // first NS_LIM2_LDS off-diagonal slots in the lane's own LDS words (no
  // sharing between lanes, so no barrier), the rest in registers
  constexpr bool CACHE = DIM == 2 && (MODE == 0 || MODE == 4);
  constexpr int NLDS = CACHE ? NS_LIM2_LDS : 0;
  __shared__ double Ps[NLDS > 0 ? NLDS : 1][NC][kBlock];
  const int lane = threadIdx.x;
  double Pc[CACHE ? C::W : 1][NC];
  double lc[CACHE ? C::W : 1];
#pragma unroll
  for (int ch = 0; ch < C::NCH; ++ch) {
    // (the 2D cached form holds fewer registers without the fences)
    if constexpr (!CACHE) colk.fence();
    PIn<DIM> x[C::CH];
    double la[C::CH], lb[C::CH];
    double ulj[BOTH ? C::CH : 1][NC], cj[C::CH];
    Bounds bj[BOTH ? C::CH : 1];
    int32_t jc[C::CH];
#pragma unroll
    for (int kk = 0; kk < C::CH; ++kk) {
      const int k = ch * C::CH + kk;
      const int64_t e = eidx<DIM>(k, i);
      jc[kk] = colk[k];
      if (k == C::W / 2) continue;  // the diagonal has no P
      const int64_t js = jc[kk] >= 0 ? jc[kk] : i;
      gather_P<DIM>(G, A, e, js, colk.mass(k), x[kk]);
      if constexpr (BOTH) {
        load_state<NC>(A.UL, N, js, ulj[kk]);
        bj[kk] = load_bounds(A, N, js);
        cj[kk] = tau * G.crm[js];  // as load_row forms it
      } else if constexpr (MODE != 2) {
        la[kk] = lt1[e];
        lb[kk] = lt1[eidx<DIM>(tslot<DIM>(k), js)];
      }
    }
#pragma unroll
    for (int kk = 0; kk < C::CH; ++kk) {
      const int k = ch * C::CH + kk;
      if (jc[kk] < 0 || jc[kk] == i) continue;
      double P[NC];
      make_P<DIM>(R, x[kk], P);
      double l;
      if constexpr (BOTH) {
        double l1, l2;
        if (limit_fast<DIM, SEV>(g, ul, P, bi, &l1)) {
          slow1 |= 1u << k;
          defer = true;
        }
        st_once(&A.lt1[eidx<DIM>(k, i)], to_lt_down<LT>(l1));
        // the neighbour's search on P_ji, formed as its row forms it
        RowCtx<DIM> Rj;
        PIn<DIM> xi;
#pragma unroll
        for (int q = 0; q < NC; ++q) {
          Rj.ui[q] = x[kk].u[q];
          Rj.fi[q] = x[kk].f[q];
          xi.u[q] = R.ui[q];
          xi.f[q] = R.fi[q];
        }
        Rj.ali = x[kk].al;
        Rj.coef = cj[kk];
        xi.al = R.ali;
        xi.d = x[kk].d;
        xi.m = x[kk].m;
        double Pj[NC];
        make_P<DIM>(Rj, xi, Pj);
        if (limit_fast<DIM, SEV>(g, ulj[kk], Pj, bj[kk], &l2)) defer = true;
        // as stored and reloaded by the two-sweep form
        l = fmin((double)to_lt_down<LT>(l1), (double)to_lt_down<LT>(l2));
      } else {
        l = MODE != 2 ? fmin(la[kk], lb[kk]) : 1.0;
      }
#pragma unroll
      for (int q = 0; q < NC; ++q) u1[q] += lam * l * P[q];
      if constexpr (CACHE) {
        const int o = k < C::W / 2 ? k : k - 1;  // off-diagonal ordinal
        if (o < NLDS) {
#pragma unroll
          for (int q = 0; q < NC; ++q) Ps[o < NLDS ? o : 0][q][lane] = P[q];
        } else {
#pragma unroll
          for (int q = 0; q < NC; ++q) Pc[k][q] = P[q];
        }
        lc[k] = l;
      }
    }
  }
  if constexpr (BOTH) {
    if (slow1) {
      uint32_t t = atomicAdd(&A.qcnt[0], (uint32_t)__builtin_popcount(slow1));
      while (slow1) {
        const int k = __builtin_ctz(slow1);
        slow1 &= slow1 - 1;
        A.q[t++] = (uint32_t)eidx<DIM>(k, i);
      }
    }
    if (defer) {
      A.drow[atomicAdd(&A.qcnt[2], 1u)] = (uint32_t)i;
      return;
    }
  }
  if constexpr (MODE == 3) {
    store_state<NC>(A.U1, N, i, u1);
  } else if constexpr (MODE == 1 || MODE == 2) {
    finish<DIM>(G, A, i, u1);
  } else {
    store_state<NC>(A.U1, N, i, u1);
    const Bounds b = BOTH ? bi : load_bounds(A, N, i);
    LT *__restrict__ lt2 = A.lt2;
    uint32_t slow = 0;
    uint32_t nzm = 0;  // slots whose stored product may be nonzero (k_fin)
    if constexpr (!CACHE) {
      // reload the neighbour data rather than keep a whole row of it live
      asm volatile("" ::: "memory");
    }
#pragma unroll
    for (int ch = 0; ch < C::NCH; ++ch) {
      if constexpr (!CACHE) colk.fence();
      double P[C::CH][NC], l[C::CH];
      int32_t jc[C::CH];
      if constexpr (CACHE) {
#pragma unroll
        for (int kk = 0; kk < C::CH; ++kk) {
          const int k = ch * C::CH + kk;
          const int o = k < C::W / 2 ? k : k - 1;
          if (k != C::W / 2 && o < NLDS) {
#pragma unroll
            for (int q = 0; q < NC; ++q) P[kk][q] = Ps[o < NLDS ? o : 0][q][lane];
          } else {
#pragma unroll
            for (int q = 0; q < NC; ++q) P[kk][q] = Pc[k][q];
          }
          l[kk] = lc[k];
          jc[kk] = colk[k];
        }
      } else {
        // one chunk of gathers in flight at a time (bounds the registers)
        asm volatile("" ::: "memory");
        PIn<DIM> x[C::CH];
        double la[C::CH], lb[C::CH];
#pragma unroll
        for (int kk = 0; kk < C::CH; ++kk) {
          const int k = ch * C::CH + kk;
          const int64_t e = eidx<DIM>(k, i);
          jc[kk] = colk[k];
          if (k == C::W / 2) continue;  // the diagonal has no P
          const int64_t js = jc[kk] >= 0 ? jc[kk] : i;
          gather_P<DIM>(G, A, e, js, colk.mass(k), x[kk]);
          la[kk] = lt1[e];
          lb[kk] = lt1[eidx<DIM>(tslot<DIM>(k), js)];
        }
#pragma unroll
        for (int kk = 0; kk < C::CH; ++kk) {
          if (ch * C::CH + kk == C::W / 2) continue;
          make_P<DIM>(R, x[kk], P[kk]);
          l[kk] = fmin(la[kk], lb[kk]);
        }
      }
#pragma unroll
      for (int kk = 0; kk < C::CH; ++kk) {
        const int k = ch * C::CH + kk;
        if (jc[kk] < 0 || jc[kk] == i) continue;
        // s1 = 0 (pass 1 took the whole P): the stored product is 0 and a
        // zero direction never needs a root, so the search is skipped
        double l2 = 0.0;
        const double s1 = 1.0 - l[kk];
        if (s1 != 0.0) {
#pragma unroll
          for (int q = 0; q < NC; ++q) P[kk][q] *= s1;
          if (limit_fast<DIM, SEV>(g, u1, P[kk], b, &l2)) slow |= 1u << k;
          else l2 *= s1;
        }
        const LT sv = to_lt_down<LT>(l2);
        st_once(&lt2[eidx<DIM>(k, i)], sv);
        if (sv != LT(0) || ((slow >> k) & 1u)) nzm |= 1u << k;
      }
    }
    if constexpr (DIM == 2) A.nzm[i] = nzm;
    if (slow) {
      uint32_t *__restrict__ q2 = A.q2 ? A.q2 : A.q;
      uint32_t t = atomicAdd(&A.qcnt[1], (uint32_t)__builtin_popcount(slow));
      while (slow) {
        const int k = __builtin_ctz(slow);
        slow &= slow - 1;
        q2[t++] = (uint32_t)eidx<DIM>(k, i);
      }
    }
  }
}

template <int DIM, int MODE, int SEV, typename LT>
__global__ __launch_bounds__(kBlock) void k_lim2(DevGraphT<LT> G, StageArgsT<LT> A, Gas g) {
  lim2_row<DIM, MODE, SEV, LT>(G, A, g, blockIdx.x, row_id());
}

// The rows that MODE 4 deferred (A.drow, qcnt[2] of them), completed with
// MODE 0 after k_root<1>; grid-stride over the list.
template <int DIM, int SEV, typename LT>
__global__ __launch_bounds__(kBlock) void k_lim2_rows(DevGraphT<LT> G, StageArgsT<LT> A,
                                                      Gas g) {
  const uint32_t n = A.qcnt[2];
  for (uint32_t t = blockIdx.x * kBlock + threadIdx.x; t < n; t += gridDim.x * kBlock) {
    const int64_t i = A.drow[t];
    lim2_row<DIM, 0, SEV, LT>(G, A, g, (uint32_t)(i / kBlock), i);
  }
}

// 3D: at most 4 waves per SIMD.  The 3D pass-1 update needs 82 VGPRs and
// would run 5 waves, whose extra gathers evict neighbour rows from L2 before
// their reuse (1.8x the HBM traffic, 4.6 instead of 4.1 ms per 256^3
// launch).
template <int DIM, int MODE, int SEV, typename LT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_lim2_w4(
    DevGraphT<LT> G, StageArgsT<LT> A, Gas g) {
  lim2_row<DIM, MODE, SEV, LT>(G, A, g, blockIdx.x, row_id());
}

// Pass-2 line search on (1 - l_ij) P_ij from U^(1) (stored by k_lim2<3>).
template <int DIM, int SEV, typename LT>
__device__ __forceinline__ void lim2b_row(const DevGraphT<LT> &G, const StageArgsT<LT> &A,
                                          const Gas &g, uint32_t blk, int64_t i) {
  using C = Cfg<DIM, NS_CH_LIM2>;
  constexpr int NC = C::NC;
  const int64_t N = G.N;
  if (i >= N) return;
  const LT *__restrict__ lt1 = A.lt1;
  LT *__restrict__ lt2 = A.lt2;
  BoxNbr<DIM> jv = block_nbr<DIM>(G, blk, i);
  RowCtx<DIM> R;
  load_row<DIM>(G, A, i, A.tau[member(A, i)], R);
  double u1[NC];
  load_state<NC>(A.U1, N, i, u1);
  const Bounds b = load_bounds(A, N, i);
  uint32_t slow = 0;
#pragma unroll
  for (int ch = 0; ch < C::NCH; ++ch) {
    jv.fence();
    double la[C::CH], lb[C::CH];
    int32_t jc[C::CH];
#pragma unroll
    for (int kk = 0; kk < C::CH; ++kk) {
      const int k = ch * C::CH + kk;
      const int64_t e = eidx<DIM>(k, i);
      jc[kk] = jv[k];
      if (k == C::W / 2) continue;  // the diagonal
      const int64_t js = jc[kk] >= 0 ? jc[kk] : i;
      la[kk] = lt1[e];
      lb[kk] = lt1[eidx<DIM>(tslot<DIM>(k), js)];
    }
#pragma unroll
    for (int kk = 0; kk < C::CH; ++kk) {
      const int k = ch * C::CH + kk;
      if (jc[kk] < 0 || jc[kk] == i) continue;
      double P[NC], l2 = 0.0;
      const double s1 = 1.0 - fmin(la[kk], lb[kk]);
      // else the stored product is 0 (see k_lim2), and P_ij's inputs are
      // not gathered
      if (s1 != 0.0) {
        PIn<DIM> x;
        gather_P<DIM>(G, A, eidx<DIM>(k, i), jc[kk], jv.mass(k), x);
        make_P<DIM>(R, x, P);
#pragma unroll
        for (int q = 0; q < NC; ++q) P[q] *= s1;
        if (limit_fast<DIM, SEV>(g, u1, P, b, &l2)) slow |= 1u << k;
        else l2 *= s1;
      }
      st_once(&lt2[eidx<DIM>(k, i)], to_lt_down<LT>(l2));
    }
  }
  if (slow) {
    uint32_t *__restrict__ q2 = A.q2 ? A.q2 : A.q;
    uint32_t t = atomicAdd(&A.qcnt[1], (uint32_t)__builtin_popcount(slow));
    while (slow) {
      const int k = __builtin_ctz(slow);
      slow &= slow - 1;
      q2[t++] = (uint32_t)eidx<DIM>(k, i);
    }
  }
}

template <int DIM, int SEV, typename LT>
__global__ __launch_bounds__(kBlock) void k_lim2b(DevGraphT<LT> G, StageArgsT<LT> A, Gas g) {
  lim2b_row<DIM, SEV, LT>(G, A, g, blockIdx.x, row_id());
}

// Row of a sliced-ELL edge index (inverse of eidx in the row).
template <int DIM>
__device__ __forceinline__ int64_t edge_row(int64_t e) {
  constexpr int W = DIM == 2 ? 9 : 27;
  return ((e >> 6) / W) * 64 + (e & 63);
}

// Roots of the entropy bound for the work list of limiter pass PASS (1 or 2):
// one lane per listed entry, grid-stride over the list, so the rare root
// finder runs at full occupancy instead of stalling a row sweep's wavefront.
// The line search's density limit l_rho was stored in lt by the sweep.
// List entries start, start + stride, ... below the list length.
template <int DIM, int PASS, int SEV, typename LT>
__device__ __forceinline__ void root_range(const DevGraphT<LT> &G, const StageArgsT<LT> &A,
                                           const Gas &g, uint32_t start, uint32_t stride) {
  constexpr int NC = DIM + 2;
  const int64_t N = G.N;
  const uint32_t n = A.qcnt[PASS - 1];
  const uint32_t *__restrict__ q = PASS == 2 && A.q2 ? A.q2 : A.q;
  LT *__restrict__ lt = PASS == 1 ? A.lt1 : A.lt2;
  for (uint32_t t = start; t < n; t += stride) {
    const int64_t e = q[t];
    const int64_t i = edge_row<DIM>(e);
    const int k = (int)((e >> 6) % (DIM == 2 ? 9 : 27));
    const BoxNbr<DIM> nb = row_nbr<DIM>(G, i);
    const int32_t j = nb[k];
    RowCtx<DIM> R;
    load_row<DIM>(G, A, i, A.tau[member(A, i)], R);
    double u[NC], P[NC];
    load_state<NC>(PASS == 1 ? A.UL : A.U1, N, i, u);
    const Bounds b = load_bounds(A, N, i);
    compute_P<DIM>(G, A, R, e, j, nb.mass(k), P);
    double s1 = 1.0;
    if constexpr (PASS == 2) {
      s1 = 1.0 - fmin(A.lt1[e], A.lt1[eidx<DIM>(tslot<DIM>(k), j)]);
#pragma unroll
      for (int c = 0; c < NC; ++c) P[c] *= s1;
    }
    const double l = entropy_root_fast<DIM, SEV>(g, u, P, lt[e], b.pmin, b.pmin5);
    lt[e] = to_lt_down<LT>(PASS == 2 ? l * s1 : l);
  }
}

template <int DIM, int PASS, int SEV, typename LT>
__global__ __launch_bounds__(kBlock) void k_root(DevGraphT<LT> G, StageArgsT<LT> A, Gas g) {
  root_range<DIM, PASS, SEV, LT>(G, A, g, blockIdx.x * kBlock + threadIdx.x,
                                 gridDim.x * kBlock);
}

template <int DIM, typename LT>
__device__ __forceinline__ void fin_row(const DevGraphT<LT> &G, const StageArgsT<LT> &A,
                                        const Gas &g, uint32_t blk, int64_t i) {
  using C = Cfg<DIM, NS_CH_FIN>;
  constexpr int NC = C::NC;
  const int64_t N = G.N;
  if (i >= N) return;
  const LT *__restrict__ lt2 = A.lt2;
  BoxNbr<DIM> jv = block_nbr<DIM>(G, blk, i);
  double u2[NC];
  load_state<NC>(A.U1, N, i, u2);
  // lt2 holds l~'_ij (1 - l_ij) with l_ij the symmetric pass-1 limiter;
  // (1 - l_ij) >= 0 and equal at ij and ji, and rounding is monotone, so the
  // smaller stored product is min(l~'_ij, l~'_ji) (1 - l_ij) itself.  It is
  // 0 wherever pass 1 took the whole P_ij (most entries away from shocks).
  // 2D: only rows with such an entry, a few in a hundred, load their own
  // data and the P_ij of those entries.
  // 3D, where most rows behind the shock have such entries, keeps one
  // unrolled pass (the entry-by-entry loop doubled the sweep's time there).
  if constexpr (DIM == 3) {
    RowCtx<DIM> R;
    load_row<DIM>(G, A, i, A.tau[member(A, i)], R);
    const double lam = 1.0 / G.lfac[i];
#pragma unroll
    for (int ch = 0; ch < C::NCH; ++ch) {
      jv.fence();
      double l2a[C::CH], l2b[C::CH];
      int32_t jc[C::CH];
#pragma unroll
      for (int kk = 0; kk < C::CH; ++kk) {
        const int k = ch * C::CH + kk;
        const int64_t e = eidx<DIM>(k, i);
        jc[kk] = jv[k];
        if (k == C::W / 2) continue;  // the diagonal
        const int64_t js = jc[kk] >= 0 ? jc[kk] : i;
        l2a[kk] = lt2[e];
        l2b[kk] = lt2[eidx<DIM>(tslot<DIM>(k), js)];
      }
#pragma unroll
      for (int kk = 0; kk < C::CH; ++kk) {
        const int k = ch * C::CH + kk;
        if (jc[kk] < 0 || jc[kk] == i) continue;
        const double w = lam * fmin(l2a[kk], l2b[kk]);
        if (w == 0.0) continue;  // no contribution, no gather
        PIn<DIM> x;
        gather_P<DIM>(G, A, eidx<DIM>(k, i), jc[kk], jv.mass(k), x);
        double P[NC];
        make_P<DIM>(R, x, P);
#pragma unroll
        for (int q = 0; q < NC; ++q) u2[q] += w * P[q];
      }
    }
    finish<DIM>(G, A, i, u2);
    return;
  }
  // the row's slots whose stored product may be nonzero, from k_lim2 (an
  // entry needs its own product nonzero)
  uint32_t nz = A.nzm[i];
  if (nz) {
    RowCtx<DIM> R;
    load_row<DIM>(G, A, i, A.tau[member(A, i)], R);
    const double lam = 1.0 / G.lfac[i];
    while (nz) {  // in slot order, as the sum over the row
      const int k = __builtin_ctz(nz);
      nz &= nz - 1;
      const int32_t j = jv[k];
      const double la = lt2[eidx<DIM>(k, i)], lb = lt2[eidx<DIM>(tslot<DIM>(k), j)];
      const double w = lam * fmin(la, lb);
      if (w == 0.0) continue;
      PIn<DIM> x;
      gather_P<DIM>(G, A, eidx<DIM>(k, i), j, jv.mass(k), x);
      double P[NC];
      make_P<DIM>(R, x, P);
#pragma unroll
      for (int q = 0; q < NC; ++q) u2[q] += w * P[q];
    }
  }
  finish<DIM>(G, A, i, u2);
}

template <int DIM, typename LT>
__global__ __launch_bounds__(kBlock) void k_fin(DevGraphT<LT> G, StageArgsT<LT> A, Gas g) {
  fin_row<DIM, LT>(G, A, g, blockIdx.x, row_id());
}

template <int DIM, typename LT>
__global__ __launch_bounds__(kBlock) void k_combine_low(DevGraphT<LT> G, StageArgsT<LT> A) {
  constexpr int NC = DIM + 2;
  const int64_t i = row_id();
  if (i >= G.N) return;
  double u[NC];
  load_state<NC>(A.UL, G.N, i, u);
  finish<DIM>(G, A, i, u);
}

// Slip projection of list entry t (entries below end).
template <int DIM>
__device__ __forceinline__ void slip_one(int t, int end, const int32_t *__restrict__ idx,
                                         const double *__restrict__ nrm, int stride,
                                         int64_t N, double *__restrict__ U) {
  if (t >= end) return;
  const int64_t i = idx[t];
  double n[DIM], mn = 0.0;
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    n[k] = nrm[(int64_t)k * stride + t];
    mn += U[node_at(DIM + 2, 1 + k, i, N)] * n[k];
  }
#pragma unroll
  for (int k = 0; k < DIM; ++k) U[node_at(DIM + 2, 1 + k, i, N)] -= mn * n[k];
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_slip(int nslip,
                                                 const int32_t *__restrict__ idx,
                                                 const double *__restrict__ nrm,
                                                 int stride, int64_t N,
                                                 double *__restrict__ U) {
  slip_one<DIM>(blockIdx.x * kBlock + threadIdx.x, nslip, idx, nrm, stride, N, U);
}

__global__ __launch_bounds__(kBlock) void k_copy(const double2 *__restrict__ src,
                                                 double2 *__restrict__ dst,
                                                 int64_t n16) {
  const int64_t t = plain_id();
  if (t < n16) dst[t] = src[t];
}

__global__ __launch_bounds__(kBlock) void k_copy8(const double *__restrict__ src,
                                                  double *__restrict__ dst,
                                                  int64_t n8) {
  const int64_t t = plain_id();
  if (t < n8) dst[t] = src[t];
}

// Component-major rows (component c of row t at c*ns + t) to and from rows
// first .. first+count-1 of a node vector of N rows (node_layout.hpp).
template <int NC>
__global__ __launch_bounds__(kBlock) void k_nodes_from_cm(const double *__restrict__ src,
                                                          int64_t ns, double *__restrict__ dst,
                                                          int64_t N, int64_t first,
                                                          int64_t count) {
  const int64_t t = plain_id();
  if (t >= count) return;
#pragma unroll
  for (int c = 0; c < NC; ++c) dst[node_at(NC, c, first + t, N)] = src[c * ns + t];
}

template <int NC>
__global__ __launch_bounds__(kBlock) void k_nodes_to_cm(const double *__restrict__ src,
                                                        int64_t N, int64_t first,
                                                        int64_t count, double *__restrict__ dst,
                                                        int64_t ns) {
  const int64_t t = plain_id();
  if (t >= count) return;
#pragma unroll
  for (int c = 0; c < NC; ++c) dst[c * ns + t] = src[node_at(NC, c, first + t, N)];
}

__global__ void k_set_scalar(double *p, double v, int n) {
  const int t = blockIdx.x * 64 + threadIdx.x;
  if (t < n) p[t] = v;
}

__global__ void k_add_scalar(double *acc, const double *v, int n) {
  const int t = blockIdx.x * 64 + threadIdx.x;
  if (t < n) acc[t] += v[t];
}

__global__ void k_clear_flags(int *flags, int n) {
  const int t = blockIdx.x * 64 + threadIdx.x;
  if (t < 4 * n) flags[t] = (t & 3) == 2 ? INT_MAX : 0;
}

template <int DIM>
__global__ __launch_bounds__(kBlock) void k_check_state(int64_t N,
                                                        const double *__restrict__ U,
                                                        int *__restrict__ flags) {
  constexpr int NC = DIM + 2;
  const int64_t i = plain_id();
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

// ---------------------------------------------------------------------------
// Diagnostics (ns_stats): minimum density and internal energy of a state and
// the limiter activity of the last stage.  Rows are strided over a fixed grid
// so that the partial results need kStatsParts slots whatever N is.
struct MinArg {
  double v;
  int64_t i;
};
__device__ __forceinline__ MinArg min_arg(MinArg a, MinArg b) {
  // smaller value, ties to the smaller index (NaN never wins)
  return (b.v < a.v || (b.v == a.v && b.i < a.i)) ? b : a;
}
__device__ __forceinline__ MinArg shfl_min_arg(MinArg a, int off) {
  MinArg b;
  b.v = __shfl_xor(a.v, off);
  b.i = __shfl_xor(a.i, off);
  return min_arg(a, b);
}

// Block reduction of the stats tuple; thread 0 holds the result.
__device__ __forceinline__ void block_stats(MinArg &r, MinArg &e, double &c0, double &c1,
                                            double &c2) {
  __shared__ MinArg sr[kBlock / 64], se[kBlock / 64];
  __shared__ double sc[3][kBlock / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    r = shfl_min_arg(r, off);
    e = shfl_min_arg(e, off);
    c0 += __shfl_xor(c0, off);
    c1 += __shfl_xor(c1, off);
    c2 += __shfl_xor(c2, off);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    sr[wid] = r; se[wid] = e; sc[0][wid] = c0; sc[1][wid] = c1; sc[2][wid] = c2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / 64; ++w) {
      r = min_arg(r, sr[w]);
      e = min_arg(e, se[w]);
      c0 += sc[0][w]; c1 += sc[1][w]; c2 += sc[2][w];
    }
  }
}

// part[b*7 + ...] = min rho, its node, min eps, its node, off-diagonal
// entries, entries with l < 1 after pass 1, entries with l + l'(1 - l) < 1
// after pass 2 (counts as doubles: exact below 2^53).
template <int DIM, typename LT>
__global__ __launch_bounds__(kBlock) void k_stats_partial(DevGraphT<LT> G,
                                                          const double *__restrict__ U,
                                                          const LT *__restrict__ lt1,
                                                          const LT *__restrict__ lt2,
                                                          int mode, double *__restrict__ part) {
  constexpr int NC = DIM + 2, W = DIM == 2 ? 9 : 27;
  const int64_t N = G.N;
  MinArg r{INFINITY, INT64_MAX}, e{INFINITY, INT64_MAX};
  double cnt = 0.0, c1 = 0.0, c2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * kBlock) {
    double u[NC];
    load_state<NC>(U, N, i, u);
    double m2 = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) m2 += u[1 + k] * u[1 + k];
    r = min_arg(r, MinArg{u[0], i});
    e = min_arg(e, MinArg{u[NC - 1] - 0.5 * m2 / u[0], i});
    const BoxNbr<DIM> nb = row_nbr<DIM>(G, i);
    for (int k = 0; k < W; ++k) {
      const int32_t j = nb[k];
      if (j < 0 || j == i) continue;
      cnt += 1.0;
      if (mode == 0) continue;
      const int64_t ea = eidx<DIM>(k, i), eb = eidx<DIM>(tslot<DIM>(k), j);
      const double l = fmin((double)lt1[ea], (double)lt1[eb]);
      if (l < 1.0) c1 += 1.0;
      if (mode == 2 && l + fmin((double)lt2[ea], (double)lt2[eb]) < 1.0) c2 += 1.0;
    }
  }
  block_stats(r, e, cnt, c1, c2);
  if (threadIdx.x == 0) {
    double *o = part + 7 * (int64_t)blockIdx.x;
    o[0] = r.v; o[1] = (double)r.i; o[2] = e.v; o[3] = (double)e.i;
    o[4] = cnt; o[5] = c1; o[6] = c2;
  }
}

__global__ __launch_bounds__(kBlock) void k_stats_final(const double *__restrict__ part,
                                                        int nparts, double *__restrict__ out) {
  MinArg r{INFINITY, INT64_MAX}, e{INFINITY, INT64_MAX};
  double c0 = 0.0, c1 = 0.0, c2 = 0.0;
  for (int b = threadIdx.x; b < nparts; b += kBlock) {
    const double *o = part + 7 * (int64_t)b;
    r = min_arg(r, MinArg{o[0], (int64_t)o[1]});
    e = min_arg(e, MinArg{o[2], (int64_t)o[3]});
    c0 += o[4]; c1 += o[5]; c2 += o[6];
  }
  block_stats(r, e, c0, c1, c2);
  if (threadIdx.x == 0) {
    out[0] = r.v; out[1] = (double)r.i; out[2] = e.v; out[3] = (double)e.i;
    out[4] = c0; out[5] = c1; out[6] = c2;
  }
}

// ---------------------------------------------------------------------------
// Persistent steps (PersistArgsT).  The workgroups take items in sequence
// order, so every item a workgroup waits for was taken earlier by a running
// workgroup, and the earliest unfinished item never waits: the launch makes
// progress whatever the number of resident workgroups.  A member's items of
// one phase depend only on that member's earlier phases, so members move
// through a stage independently.  Completion is published with a release at
// device scope (the stores of the item reach the device-coherent level
// before the counter moves) and a wait ends with an acquire (no stale cached
// copy is read afterwards).

// The two state buffers other than c, ascending (k = 0, 1).
__device__ __forceinline__ int other_buf(int c, int k) {
  return k == 0 ? (c == 0 ? 1 : 0) : (c == 2 ? 1 : 2);
}

// tau = cfl min over the member's row blocks; the time advanced grows by it
// (every thread of the workgroup calls it).
__device__ __forceinline__ void dt_final_member(const double *__restrict__ partial,
                                                int32_t b0, int32_t b1, double cfl,
                                                double *tau, double *tacc) {
  double v = INFINITY;
  for (int64_t b = b0 + threadIdx.x; b < b1; b += kBlock) v = fmin(v, partial[b]);
  v = block_min(v);
  if (threadIdx.x == 0) {
    const double t = cfl * v;
    *tau = t;
    *tacc += t;
  }
}

template <typename LT>
__device__ __forceinline__ bool persist_stopped(const PersistArgsT<LT> &P) {
  return __hip_atomic_load(P.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

template <typename LT>
__device__ __forceinline__ void persist_raise(const PersistArgsT<LT> &P, int why) {
  atomicCAS(P.stop + 1, 0, why);
  atomicOr(P.stop + 2, 1 << why);
  __hip_atomic_store(P.stop, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename LT>
__device__ __forceinline__ bool persist_give_up(const PersistArgsT<LT> &P) {
  return P.give_up &&
         __hip_atomic_load(P.give_up, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0;
}

// Wave 0: waits until *ctr >= need (every lane polls the same word, so
// every branch is uniform over the wave) and returns the value it saw, or
// 0 if the launch stops first.  The counter is polled with relaxed loads (an
// acquire per poll would invalidate the caches the working workgroups read,
// on every poll of every waiting workgroup); the acquire follows once,
// after the wait.  The wait is bounded by wait_ticks of the wall clock and
// ends early when the launch is stopped or the give-up word is set (which
// then stops the launch).
template <typename LT>
__device__ uint32_t persist_wait(const PersistArgsT<LT> &P, const uint32_t *ctr,
                                 uint32_t need) {
  auto seen = [&] {
    return __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  };
  uint32_t v = seen();
  if (v < need) {
    const uint64_t t0 = wall_clock64();
    for (uint32_t it = 0;; ++it) {
      if (__builtin_amdgcn_readfirstlane(persist_stopped(P))) return 0;
      if ((it & 63u) == 0) {
        if (__builtin_amdgcn_readfirstlane(persist_give_up(P))) {
          if (threadIdx.x == 0) persist_raise(P, 2);
          return 0;
        }
        if (__builtin_amdgcn_readfirstlane(wall_clock64() - t0 >= P.wait_ticks)) {
          if (threadIdx.x == 0) persist_raise(P, 1);
          return 0;
        }
      }
      __builtin_amdgcn_s_sleep(8);
      v = seen();
      if (v >= need) break;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return v;
}

// The control path (ticket, wait, publication) runs on wave 0 with
// conditions uniform over the wave, and only the atomics themselves on lane
// 0: a barrier reached under a condition the compiler takes as divergent
// within a wave -- e.g. thread 0 alone on both sides of the loop's back
// edge -- lets the structurizer nest the loop so that the other lanes repeat
// the barriers and the item on their own.
//
// Cache maintenance at device scope (write-back before a completion is
// published, invalidation after a wait) is paid per phase, not per item:
// a workgroup keeps its completed items pending and publishes them (one
// release, one counter update) only before it has to wait or moves to
// another member, and it skips the wait and the acquire when an earlier
// wait already saw the member's counter at or above the item's need.  A
// workgroup never waits while it holds pending items, so every pending item
// is published before anything can depend on it in a wait.
template <int DIM, int SEV, typename LT>
__global__ __launch_bounds__(kBlock) void k_persist(DevGraphT<LT> G, PersistArgsT<LT> P,
                                                    Gas g) {
  constexpr int W = DIM == 2 ? 9 : 27;
  __shared__ uint32_t s_item, s_seen;
  __shared__ int s_go;
  const int tid = threadIdx.x;
  const bool wave0 = __builtin_amdgcn_readfirstlane(tid) == 0;
  const PersistPlan &pl = P.plan;
  // uniform state, identical in every wave: the member and counter value of
  // the last acquire; the member and number of the pending completions
  int acq_m = -1, pend_m = -1;
  uint32_t acq_v = 0, pend_n = 0;
  auto publish = [&] {
    if (pend_n == 0) return;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (wave0 && tid == 0)
      __hip_atomic_fetch_add(P.done + pend_m, pend_n, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    pend_n = 0;
  };
  for (;;) {
    if (wave0) {
      int go = 0;
      uint32_t t = 0;
      if (!__builtin_amdgcn_readfirstlane(persist_stopped(P))) {
        uint32_t mine = 0;
        if (tid == 0) mine = atomicAdd(P.ticket, 1u);
        t = __builtin_amdgcn_readfirstlane(mine);
        if (t < P.items) {
          // the give-up word is also read every 16 items, so that it stops
          // a launch whose waits all end at once
          if ((t & 15u) == 0 && __builtin_amdgcn_readfirstlane(persist_give_up(P))) {
            if (tid == 0) persist_raise(P, 2);
          } else {
            go = 1;
          }
        }
      }
      if (tid == 0) {
        s_item = t;
        s_go = go;
      }
    }
    __syncthreads();
    if (!__builtin_amdgcn_readfirstlane(s_go)) {
      publish();
      return;
    }
    const uint32_t t = __builtin_amdgcn_readfirstlane(s_item);
    // item -> step, phase, member, item within the member's phase
    const uint32_t step = t / P.items_step;
    const uint32_t u = t - step * P.items_step;
    int p = 0;
    while (p + 1 < pl.nph && pl.off[p + 1] <= u) ++p;
    const int ph = pl.phase[p], st = pl.stage[p];
    const int kind = persist_kind(ph);
    uint32_t r = u - (uint32_t)pl.off[p];
    int m = 0;
    if (kind == PK_ONE) {
      m = (int)r;
      r = 0;
    } else {
      // (the member tables are read-only: scalar loads, uniform results)
      const int32_t *cum = kind == PK_ROW ? P.mblk : kind == PK_ROOT ? P.rblk : P.sblk;
      int lo = 0, hi = P.A.nmem;  // largest m with cum[m] <= r
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if ((uint32_t)geo_ld(&cum[mid]) <= r) lo = mid;
        else hi = mid;
      }
      m = lo;
      r -= (uint32_t)geo_ld(&cum[m]);
    }
    const int32_t mb0 = geo_ld(&P.mblk[m]), mb1 = geo_ld(&P.mblk[m + 1]);
    const uint32_t nb = mb1 - mb0, nr = geo_ld(&P.rblk[m + 1]) - geo_ld(&P.rblk[m]),
                   ns = geo_ld(&P.sblk[m + 1]) - geo_ld(&P.sblk[m]);
    auto before = [&](int q) {
      return pl.pre[q][PK_ROW] * nb + pl.pre[q][PK_ROOT] * nr + pl.pre[q][PK_SLIP] * ns +
             (uint32_t)pl.pre[q][PK_ONE];
    };
    const uint32_t need = step * before(pl.nph) + before(p);
    if (m != pend_m) publish();
    if (m != acq_m || need > acq_v) {
      publish();
      if (wave0) {
        const uint32_t v = persist_wait(P, P.done + m, need);
        if (tid == 0) s_seen = v;
      }
      __syncthreads();  // (the acquire of wave 0 covers the workgroup's CU)
      const uint32_t v = __builtin_amdgcn_readfirstlane(s_seen);
      if (v < need) return;  // the launch stopped
      acq_m = m;
      acq_v = v;
    }
    // buffers of the stage (as the launch path rotates them)
    int c = P.cur;
    for (uint32_t k = 0; k < step; ++k) c = other_buf(c, 0);
    const int o1 = other_buf(c, 0), o2 = other_buf(c, 1);
    StageArgsT<LT> A = P.A;
    A.Un = P.S[c];
    if (st == 0) {
      A.U = P.S[c]; A.out = P.S[o1]; A.sa = 0.0; A.sb = 1.0; A.check_cfl = 0;
    } else if (st == 1) {
      A.U = P.S[o1]; A.out = P.S[o2]; A.sa = 0.75; A.sb = 0.25; A.check_cfl = 1;
    } else {
      A.U = P.S[o2]; A.out = P.S[o1]; A.sa = 1.0 / 3.0; A.sb = 2.0 / 3.0; A.check_cfl = 1;
    }
    // the member's own work lists: its slice of q and its two counters
    A.q = P.A.q + (int64_t)W * kBlock * mb0;
    A.q2 = A.q;  // root1 empties the list before lim2 fills it again
    A.drow = nullptr;
    A.qcnt = P.pcnt + 2 * m;
    const uint32_t blk = kind == PK_ROW ? (uint32_t)mb0 + r : 0u;
    const int64_t i = (int64_t)blk * kBlock + tid;
    switch (ph) {
      case PP_PRIM: prim_row<DIM, false>(G.N, A.U, A.aux, g, i); break;
      case PP_VISC: visc_row<DIM, 0, SEV, LT>(G, A.U, A.aux, A.d, A.alpha, g, blk, i); break;
      case PP_DTP: dt_partial_blk<DIM, LT>(G, A.d, A.partial, blk, i); break;
      case PP_DTF:
        dt_final_member(A.partial, mb0, mb1, P.cfl, A.tau + m, P.tacc + m);
        break;
      case PP_LO: lo_row<DIM, LT>(G, A, g, blk, i, r == 0 && tid == 0); break;
      case PP_LIM1: lim1_row<DIM, SEV, LT>(G, A, g, blk, i); break;
      case PP_ROOT1: root_range<DIM, 1, SEV, LT>(G, A, g, r * kBlock + tid, nr * kBlock); break;
      case PP_LIM2: lim2_row<DIM, DIM == 2 ? 0 : 3, SEV, LT>(G, A, g, blk, i); break;
      case PP_LIM2B:
        if constexpr (DIM == 3) lim2b_row<DIM, SEV, LT>(G, A, g, blk, i);
        break;
      case PP_ROOT2: root_range<DIM, 2, SEV, LT>(G, A, g, r * kBlock + tid, nr * kBlock); break;
      case PP_FIN: fin_row<DIM, LT>(G, A, g, blk, i); break;
      case PP_SLIP:
        slip_one<DIM>(geo_ld(&P.mslip[m]) + (int)(r * kBlock) + tid, geo_ld(&P.mslip[m + 1]),
                      P.slip_idx, P.slip_n, P.nslip, G.N, A.out);
        break;
      default: break;
    }
    pend_m = m;
    ++pend_n;
  }
}

__global__ void k_persist_reset(uint32_t *done, uint32_t *pcnt, uint32_t *ticket, int *stop,
                                int nmem, int run_start) {
  const int t = blockIdx.x * 64 + threadIdx.x;
  if (t < nmem) done[t] = 0;
  if (t < 2 * nmem) pcnt[t] = 0;
  if (t == 0) {
    *ticket = 0;
    if (run_start) stop[2] = 0;
    stop[0] = stop[2] != 0;  // a launch after one that gave up stops at once
    stop[1] = 0;
  }
}

inline dim3 grid_for(int64_t n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

template <int DIM, int SEV, typename LT>
void stage_impl(const Gas &gas, const DevGraphT<LT> &G, const StageArgsT<LT> &A,
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
  if (indicator == 0)
    NS_LAUNCH("prim", hipLaunchKernelGGL((k_prim<DIM, false>), grid, block, 0, s, G.N, A.U,
                                         A.aux, gas));
  else
    NS_LAUNCH("prim", hipLaunchKernelGGL((k_prim<DIM, true>), grid, block, 0, s, G.N, A.U,
                                         A.aux, gas));
  bool f32 = false;
  if constexpr (SEV == 1 && sizeof(LT) == 4) {
    if (indicator == 0 && A.fp32_eval) {
      f32 = true;
      NS_LAUNCH("visc", hipLaunchKernelGGL((k_visc_f32<DIM, LT>), grid, block, 0, s, G, A.U,
                                           A.aux, A.d, A.alpha, gas));
    }
  }
  if (f32) {
  } else if (indicator == 0)
    NS_LAUNCH("visc", hipLaunchKernelGGL((k_visc<DIM, 0, SEV, LT>), grid, block, 0, s, G,
                                         A.U, A.aux, A.d, A.alpha, gas));
  else if (indicator == 1)
    NS_LAUNCH("visc", hipLaunchKernelGGL((k_visc<DIM, 1, SEV, LT>), grid, block, 0, s, G,
                                         A.U, A.aux, A.d, A.alpha, gas));
  else
    NS_LAUNCH("visc", hipLaunchKernelGGL((k_visc<DIM, 2, SEV, LT>), grid, block, 0, s, G,
                                         A.U, A.aux, A.d, A.alpha, gas));
  if (auto_dt) {
    NS_LAUNCH("dt_partial", hipLaunchKernelGGL((k_dt_partial<DIM, LT>), grid, block, 0, s,
                                               G, A.d, A.partial));
    if (A.seg)
      NS_LAUNCH("dt_final", hipLaunchKernelGGL(k_dt_final_members, dim3((unsigned)A.nmem),
                                               dim3(1024), 0, s, A.partial, A.mblk, cfl,
                                               A.tau));
    else
      NS_LAUNCH("dt_final", hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(1024), 0, s,
                                               A.partial, (int64_t)grid.x, cfl, A.tau));
  }
  NS_LAUNCH("lo", hipLaunchKernelGGL((k_lo<DIM, LT>), grid, block, 0, s, G, A, gas));
  if (limiter == 1) {
    NS_LAUNCH("combine", hipLaunchKernelGGL((k_combine_low<DIM, LT>), grid, block, 0, s,
                                            G, A));
  } else if (limiter == 2) {
    NS_LAUNCH("lim2", hipLaunchKernelGGL((k_lim2<DIM, 2, SEV, LT>), grid, block, 0, s, G, A,
                                         gas));
  } else {
    // the work lists hold a small fraction of the edges (~1.5% of them in the
    // 3D shock tube); up to 4M lanes cover a list without striding, and
    // blocks past its end exit at once
    const dim3 rgrid(std::min<unsigned>(grid.x, 16384u));
    bool merged = false;
    if constexpr (DIM == 2) {
      if (passes != 1 && A.drow && A.q2) {
        // both pass-1 searches, the update and the pass-2 search in one
        // sweep; the deferred rows after the pass-1 roots
        merged = true;
        NS_LAUNCH("lim12", hipLaunchKernelGGL((k_lim2<DIM, 4, SEV, LT>), grid, block, 0, s,
                                              G, A, gas));
        NS_LAUNCH("root1", hipLaunchKernelGGL((k_root<DIM, 1, SEV, LT>), rgrid, block, 0, s,
                                              G, A, gas));
        NS_LAUNCH("lim2d", hipLaunchKernelGGL((k_lim2_rows<DIM, SEV, LT>), rgrid, block, 0, s,
                                              G, A, gas));
        NS_LAUNCH("root2", hipLaunchKernelGGL((k_root<DIM, 2, SEV, LT>), rgrid, block, 0, s,
                                              G, A, gas));
        NS_LAUNCH("fin", hipLaunchKernelGGL((k_fin<DIM, LT>), grid, block, 0, s, G, A, gas));
      }
    }
    if (!merged) {
    NS_LAUNCH("lim1", hipLaunchKernelGGL((k_lim1<DIM, SEV, LT>), grid, block, 0, s, G, A, gas));
    NS_LAUNCH("root1", hipLaunchKernelGGL((k_root<DIM, 1, SEV, LT>), rgrid, block, 0, s, G,
                                          A, gas));
    if (passes == 1) {
      NS_LAUNCH("lim2", hipLaunchKernelGGL((k_lim2<DIM, 1, SEV, LT>), grid, block, 0, s, G,
                                           A, gas));
    } else {
      if constexpr (DIM == 2) {
        NS_LAUNCH("lim2", hipLaunchKernelGGL((k_lim2<DIM, 0, SEV, LT>), grid, block, 0, s,
                                             G, A, gas));
      } else {
        NS_LAUNCH("lim2", hipLaunchKernelGGL((k_lim2_w4<DIM, 3, SEV, LT>), grid, block, 0, s,
                                             G, A, gas));
        NS_LAUNCH("lim2b", hipLaunchKernelGGL((k_lim2b<DIM, SEV, LT>), grid, block, 0, s,
                                              G, A, gas));
      }
      NS_LAUNCH("root2", hipLaunchKernelGGL((k_root<DIM, 2, SEV, LT>), rgrid, block, 0, s, G,
                                            A, gas));
      NS_LAUNCH("fin", hipLaunchKernelGGL((k_fin<DIM, LT>), grid, block, 0, s, G, A, gas));
    }
    }
  }
#undef NS_LAUNCH
}

template <int DIM, int SEV, typename LT>
void dt_impl(const Gas &gas, const DevGraphT<LT> &G, const StageArgsT<LT> &A, double cfl,
             hipStream_t s, void (*before)(void *, const char *),
             void (*after)(void *), void *prof) {
  const dim3 grid = grid_for(G.N), block(kBlock);
  before(prof, "prim");
  hipLaunchKernelGGL((k_prim<DIM, true>), grid, block, 0, s, G.N, A.U, A.aux, gas);
  after(prof);
  before(prof, "visc_dt");
  hipLaunchKernelGGL((k_visc<DIM, 2, SEV, LT>), grid, block, 0, s, G, A.U, A.aux, A.d,
                     A.alpha, gas);
  after(prof);
  before(prof, "dt_partial");
  hipLaunchKernelGGL((k_dt_partial<DIM, LT>), grid, block, 0, s, G, A.d, A.partial);
  after(prof);
  before(prof, "dt_final");
  if (A.seg)
    hipLaunchKernelGGL(k_dt_final_members, dim3((unsigned)A.nmem), dim3(1024), 0, s,
                       A.partial, A.mblk, cfl, A.tau);
  else
    hipLaunchKernelGGL(k_dt_final, dim3(1), dim3(1024), 0, s, A.partial, (int64_t)grid.x,
                       cfl, A.tau);
  after(prof);
}

}  // namespace

template <typename LT>
void launch_dt_only(int dim, const Gas &gas, const DevGraphT<LT> &g,
                    const StageArgsT<LT> &a, double cfl, hipStream_t s,
                    void (*before)(void *, const char *), void (*after)(void *),
                    void *prof) {
  if (dim == 2) {
    if (gas.seven) dt_impl<2, 1, LT>(gas, g, a, cfl, s, before, after, prof);
    else dt_impl<2, 0, LT>(gas, g, a, cfl, s, before, after, prof);
  } else {
    if (gas.seven) dt_impl<3, 1, LT>(gas, g, a, cfl, s, before, after, prof);
    else dt_impl<3, 0, LT>(gas, g, a, cfl, s, before, after, prof);
  }
}

template <typename LT>
void launch_stage(int dim, const Gas &gas, const DevGraphT<LT> &g,
                  const StageArgsT<LT> &a, int indicator, int limiter, int passes,
                  bool auto_dt, double cfl, hipStream_t s,
                  void (*before)(void *, const char *), void (*after)(void *),
                  void *prof) {
  auto run = [&](auto impl) {
    impl(gas, g, a, indicator, limiter, passes, auto_dt, cfl, s, before, after, prof);
  };
  if (dim == 2) {
    if (gas.seven) run(stage_impl<2, 1, LT>);
    else run(stage_impl<2, 0, LT>);
  } else {
    if (gas.seven) run(stage_impl<3, 1, LT>);
    else run(stage_impl<3, 0, LT>);
  }
}

template void launch_stage<double>(int, const Gas &, const DevGraphT<double> &,
                                   const StageArgsT<double> &, int, int, int, bool,
                                   double, hipStream_t, void (*)(void *, const char *),
                                   void (*)(void *), void *);
template void launch_stage<float>(int, const Gas &, const DevGraphT<float> &,
                                  const StageArgsT<float> &, int, int, int, bool,
                                  double, hipStream_t, void (*)(void *, const char *),
                                  void (*)(void *), void *);
template void launch_dt_only<double>(int, const Gas &, const DevGraphT<double> &,
                                     const StageArgsT<double> &, double, hipStream_t,
                                     void (*)(void *, const char *), void (*)(void *),
                                     void *);
template void launch_dt_only<float>(int, const Gas &, const DevGraphT<float> &,
                                    const StageArgsT<float> &, double, hipStream_t,
                                    void (*)(void *, const char *), void (*)(void *),
                                    void *);

void launch_slip(int dim, int64_t N, int nslip, const int32_t *idx,
                 const double *nrm, double *U, hipStream_t s, int stride) {
  if (nslip <= 0) return;
  if (stride < 0) stride = nslip;
  const dim3 grid((unsigned)((nslip + kBlock - 1) / kBlock)), block(kBlock);
  if (dim == 2)
    hipLaunchKernelGGL(k_slip<2>, grid, block, 0, s, nslip, idx, nrm, stride, N, U);
  else
    hipLaunchKernelGGL(k_slip<3>, grid, block, 0, s, nslip, idx, nrm, stride, N, U);
}

void launch_set_scalar(double *p, double v, hipStream_t s, int n) {
  hipLaunchKernelGGL(k_set_scalar, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, p, v, n);
}

void launch_add_scalar(double *acc, const double *v, hipStream_t s, int n) {
  hipLaunchKernelGGL(k_add_scalar, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, acc, v,
                     n);
}

void launch_copy(const void *src, void *dst, int64_t n16, int word,
                 hipStream_t s) {
  if (word == 8)
    hipLaunchKernelGGL(k_copy8, grid_for(2 * n16), dim3(kBlock), 0, s,
                       static_cast<const double *>(src), static_cast<double *>(dst),
                       2 * n16);
  else
    hipLaunchKernelGGL(k_copy, grid_for(n16), dim3(kBlock), 0, s,
                       static_cast<const double2 *>(src),
                       static_cast<double2 *>(dst), n16);
}

void launch_nodes_from_cm(int nc, const double *src, int64_t ns, double *dst, int64_t N,
                          int64_t first, int64_t count, hipStream_t s) {
  if (count <= 0) return;
  if (nc == 4)
    hipLaunchKernelGGL(k_nodes_from_cm<4>, grid_for(count), dim3(kBlock), 0, s, src, ns, dst,
                       N, first, count);
  else
    hipLaunchKernelGGL(k_nodes_from_cm<5>, grid_for(count), dim3(kBlock), 0, s, src, ns, dst,
                       N, first, count);
}

void launch_nodes_to_cm(int nc, const double *src, int64_t N, int64_t first, int64_t count,
                        double *dst, int64_t ns, hipStream_t s) {
  if (count <= 0) return;
  if (nc == 4)
    hipLaunchKernelGGL(k_nodes_to_cm<4>, grid_for(count), dim3(kBlock), 0, s, src, N, first,
                       count, dst, ns);
  else
    hipLaunchKernelGGL(k_nodes_to_cm<5>, grid_for(count), dim3(kBlock), 0, s, src, N, first,
                       count, dst, ns);
}

void persist_plan(int dim, int64_t rows_tot, int64_t roots_tot, int64_t slips_tot,
                  int nmem, PersistPlan *pl) {
  int n = 0;
  auto add = [&](int ph, int st) {
    pl->phase[n] = (int8_t)ph;
    pl->stage[n] = (int8_t)st;
    ++n;
  };
  for (int st = 0; st < 3; ++st) {
    add(PP_PRIM, st);
    add(PP_VISC, st);
    if (st == 0) {  // the CFL time step of the step
      add(PP_DTP, st);
      add(PP_DTF, st);
    }
    add(PP_LO, st);
    add(PP_LIM1, st);
    add(PP_ROOT1, st);
    add(PP_LIM2, st);
    if (dim == 3) add(PP_LIM2B, st);
    add(PP_ROOT2, st);
    add(PP_FIN, st);
    add(PP_SLIP, st);
  }
  pl->nph = n;
  int16_t c[4] = {0, 0, 0, 0};
  int64_t off = 0;
  for (int p = 0; p <= n; ++p) {
    for (int k = 0; k < 4; ++k) pl->pre[p][k] = c[k];
    pl->off[p] = off;
    if (p == n) break;
    const int kind = persist_kind(pl->phase[p]);
    ++c[kind];
    off += kind == PK_ROW ? rows_tot : kind == PK_ROOT ? roots_tot
           : kind == PK_SLIP ? slips_tot : nmem;
  }
}

namespace {
template <typename F>
const void *persist_kernel(int dim, bool seven, F pick) {
  return dim == 2 ? (seven ? pick(std::integral_constant<int, 2>{}, std::integral_constant<int, 1>{})
                           : pick(std::integral_constant<int, 2>{}, std::integral_constant<int, 0>{}))
                  : (seven ? pick(std::integral_constant<int, 3>{}, std::integral_constant<int, 1>{})
                           : pick(std::integral_constant<int, 3>{}, std::integral_constant<int, 0>{}));
}
template <typename LT>
const void *persist_kernel_lt(int dim, bool seven) {
  return persist_kernel(dim, seven, [](auto d, auto sev) {
    return (const void *)k_persist<decltype(d)::value, decltype(sev)::value, LT>;
  });
}
}  // namespace

int persist_grid(int dim, bool seven, bool fp32) {
  const void *k = fp32 ? persist_kernel_lt<float>(dim, seven)
                       : persist_kernel_lt<double>(dim, seven);
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, kBlock, 0) != hipSuccess) return 0;
  return std::max(per, 1) * cus;
}

template <typename LT>
void launch_persistent(int dim, const Gas &gas, const DevGraphT<LT> &g,
                       const PersistArgsT<LT> &p, int grid, hipStream_t s) {
  const dim3 gr((unsigned)grid), bl(kBlock);
  if (dim == 2) {
    if (gas.seven) hipLaunchKernelGGL((k_persist<2, 1, LT>), gr, bl, 0, s, g, p, gas);
    else hipLaunchKernelGGL((k_persist<2, 0, LT>), gr, bl, 0, s, g, p, gas);
  } else {
    if (gas.seven) hipLaunchKernelGGL((k_persist<3, 1, LT>), gr, bl, 0, s, g, p, gas);
    else hipLaunchKernelGGL((k_persist<3, 0, LT>), gr, bl, 0, s, g, p, gas);
  }
}
template void launch_persistent<double>(int, const Gas &, const DevGraphT<double> &,
                                        const PersistArgsT<double> &, int, hipStream_t);
template void launch_persistent<float>(int, const Gas &, const DevGraphT<float> &,
                                       const PersistArgsT<float> &, int, hipStream_t);

void launch_persist_reset(uint32_t *done, uint32_t *pcnt, uint32_t *ticket, int *stop,
                          int nmem, bool run_start, hipStream_t s) {
  hipLaunchKernelGGL(k_persist_reset, dim3((unsigned)((2 * nmem + 63) / 64)), dim3(64), 0, s,
                     done, pcnt, ticket, stop, nmem, run_start ? 1 : 0);
}

void launch_clear_flags(int *flags, hipStream_t s, int n) {
  hipLaunchKernelGGL(k_clear_flags, dim3((unsigned)((4 * n + 63) / 64)), dim3(64), 0, s,
                     flags, n);
}

template <typename LT>
int launch_stats(int dim, const DevGraphT<LT> &g, const double *U, const LT *lt1,
                 const LT *lt2, int mode, double *part, double *out, hipStream_t s) {
  const int nparts = (int)std::min<int64_t>((g.N + kBlock - 1) / kBlock, kStatsParts);
  if (dim == 2)
    hipLaunchKernelGGL((k_stats_partial<2, LT>), dim3(nparts), dim3(kBlock), 0, s, g, U, lt1,
                       lt2, mode, part);
  else
    hipLaunchKernelGGL((k_stats_partial<3, LT>), dim3(nparts), dim3(kBlock), 0, s, g, U, lt1,
                       lt2, mode, part);
  hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(kBlock), 0, s, part, nparts, out);
  return nparts;
}
template int launch_stats<double>(int, const DevGraphT<double> &, const double *,
                                  const double *, const double *, int, double *, double *,
                                  hipStream_t);
template int launch_stats<float>(int, const DevGraphT<float> &, const double *, const float *,
                                 const float *, int, double *, double *, hipStream_t);

void launch_check_state(int dim, int64_t N, const double *U, int *flags,
                        hipStream_t s) {
  const dim3 grid = grid_for(N), block(kBlock);
  if (dim == 2)
    hipLaunchKernelGGL(k_check_state<2>, grid, block, 0, s, N, U, flags);
  else
    hipLaunchKernelGGL(k_check_state<3>, grid, block, 0, s, N, U, flags);
}

}  // namespace ns
