// par_ops.hpp -- the matrix-free Q1 operators of the parabolic step on a
// uniform box mesh, for one lane per node: neighbour indexing, the
// pre-summed interior stencil and the cell-by-cell element matrix at wall
// nodes (element tables of element.hpp), templated on the value type (FP64
// for the CG, FP32 for the multigrid V-cycle).
#pragma once

#include "par_kernels.hpp"

namespace ns {
namespace pops {

template <int DIM> struct P {
  static constexpr int S = DIM == 2 ? 9 : 27;  // neighbourhood slots
  static constexpr int L = 1 << DIM;           // nodes per cell
  static constexpr int C = S / 2;              // slot of the node itself
};

__device__ __forceinline__ void decode(const ParGrid &G, int64_t i, int64_t c[3]) {
  c[0] = i % G.n[0];
  const int64_t t = i / G.n[0];
  c[1] = t % G.n[1];
  c[2] = t / G.n[1];
}

// node at offset (slot s: o_d = (s / 3^d) % 3 - 1) from c, or -1 outside a
// wall-bounded direction
template <int DIM>
__device__ __forceinline__ int64_t nb_index(const ParGrid &G, const int64_t c[3],
                                            int s) {
  int64_t idx = 0, stride = 1;
  int m = 1;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    int64_t a = c[d] + (s / m) % 3 - 1;
    m *= 3;
    if (G.per[d]) {
      a = a < 0 ? a + G.n[d] : (a >= G.n[d] ? a - G.n[d] : a);
    } else if (a < 0 || a >= G.n[d]) {
      return -1;
    }
    idx += a * stride;
    stride *= G.n[d];
  }
  return idx;
}

// does the cell in which node c is local node a exist?
template <int DIM>
__device__ __forceinline__ bool cell_exists(const ParGrid &G, const int64_t c[3],
                                            int a) {
  bool ok = true;
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int64_t lo = c[d] - ((a >> d) & 1);
    if (!G.per[d] && (lo < 0 || lo > G.n[d] - 2)) ok = false;
  }
  return ok;
}

// neighbourhood slot of local node b of the cell in which the centre is a
template <int DIM>
__host__ __device__ constexpr int slot_of(int a, int b) {
  int s = 0, m = 1;
  for (int d = 0; d < DIM; ++d) {
    s += (((b >> d) & 1) - ((a >> d) & 1) + 1) * m;
    m *= 3;
  }
  return s;
}

// offsets into the element table (element.hpp, Q1Tables::packed)
template <int DIM> struct TabOff {
  static constexpr int L = 1 << DIM, S = DIM == 2 ? 9 : 27;
  static constexpr int heat = DIM * DIM * L * L;
  static constexpr int phi = heat + L * L;
  static constexpr int dphi = phi + L * L;
  static constexpr int w = dphi + L * L * DIM;
  static constexpr int sst = w + 1;
  static constexpr int sht = sst + S * DIM * DIM;
};

// all 2^dim cells of the node exist (no wall face through it)
template <int DIM>
__device__ __forceinline__ bool interior(const ParGrid &G, const int64_t c[3]) {
  bool in = true;
#pragma unroll
  for (int d = 0; d < DIM; ++d)
    if (!G.per[d] && (c[d] == 0 || c[d] == G.n[d] - 1)) in = false;
  return in;
}

// acc_k = (operator row of the node applied to x), without the mass term:
// at interior nodes by the pre-summed 3^dim-point stencil, at wall nodes
// cell by cell with the element matrix (NC = dim: stress, NC = 1: heat)
template <int DIM, int NC, typename T = double>
__device__ __forceinline__ void op_apply(const ParGrid &G, const T *__restrict__ tab,
                                         const T *__restrict__ x,
                                         const int64_t c[3], T (&acc)[NC]) {
  using O = TabOff<DIM>;
  constexpr int L = O::L, S = O::S;
  const int64_t N = G.N;
#pragma unroll
  for (int k = 0; k < NC; ++k) acc[k] = T(0);
  if (interior<DIM>(G, c)) {
    const T *__restrict__ st = tab + (NC > 1 ? O::sst : O::sht);
    // a plane of 3^(dim-1) neighbours at a time (all 27 gathers of the 3D
    // stencil in flight at once would cut the occupancy to 2 waves)
#pragma unroll 9
    for (int s = 0; s < S; ++s) {
      const int64_t j = nb_index<DIM>(G, c, s);
      T xj[NC];
#pragma unroll
      for (int l = 0; l < NC; ++l) xj[l] = x[l * N + j];
#pragma unroll
      for (int k = 0; k < NC; ++k)
#pragma unroll
        for (int l = 0; l < NC; ++l) acc[k] += st[(s * NC + k) * NC + l] * xj[l];
    }
  } else {
    const T *__restrict__ E = tab + (NC > 1 ? 0 : O::heat);
    for (int a = 0; a < L; ++a) {
      if (!cell_exists<DIM>(G, c, a)) continue;
      for (int b = 0; b < L; ++b) {
        const int64_t j = nb_index<DIM>(G, c, slot_of<DIM>(a, b));
        T xj[NC];
#pragma unroll
        for (int l = 0; l < NC; ++l) xj[l] = x[l * N + j];
#pragma unroll
        for (int k = 0; k < NC; ++k)
#pragma unroll
          for (int l = 0; l < NC; ++l)
            acc[k] += E[((k * NC + l) * L + a) * L + b] * xj[l];
      }
    }
  }
}

// diagonal entry E^kk_aa summed over the node's cells
template <int DIM, int NC, typename T = double>
__device__ __forceinline__ T op_diag(const ParGrid &G, const T *__restrict__ E,
                                     const int64_t c[3], int k) {
  constexpr int L = P<DIM>::L;
  T d = T(0);
#pragma unroll
  for (int a = 0; a < L; ++a)
    if (cell_exists<DIM>(G, c, a)) d += E[((k * NC + k) * L + a) * L + a];
  return d;
}

}  // namespace pops
}  // namespace ns
