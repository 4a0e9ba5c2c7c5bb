// box_nbr.hpp -- column index and coefficients m_ij, c_ij of every entry of
// the Q1 stencil graph of a uniform box mesh, derived from the row index
// instead of loaded.
//
// The nodes of a box mesh are numbered lexicographically (x fastest) and the
// neighbour in slot k = (dx+1) + 3(dy+1) + 9(dz+1) is the node at offset
// (dx,dy,dz), wrapped in a periodic direction and absent beyond a wall.  The
// transposed entry (j,i) of (i,j) is therefore in slot W-1-k of row j.
// m_ij and c_ij (Sec. 2.2) are tensor products of 1D factors that depend
// only on the offset, the mesh size and whether the node is at a wall end
// along each direction; they are formed here in the order of the graph
// builder (graph.hpp), so they equal its values bit for bit.  The row sweeps
// compute all of them instead of reading (2 + dim) arrays per entry.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace ns {

// One box mesh inside the row numbering of a solver: rows base .. base+nn-1
// are its nodes; rows from base+nn up to the next mesh (padding rows of a
// pack) are isolated nodes whose only entry is the diagonal one.
struct BoxGeom {
  // 1D mass factors along d: diagonal of an interior node (2h/3), diagonal
  // at a wall end (h/3), off-diagonal (h/6)
  double m_inner[3], m_end[3], m_off[3];
  int32_t base;
  int32_t nn;
  int32_t n[3];  // nodes per direction (n[2] = 1 in 2D)
  int32_t per;   // bit d set: direction d is periodic
};

// Reads of the mesh geometry.  On the device they go through the constant
// address space: the geometry is never written by a kernel, and its
// addresses are uniform over a workgroup, so they become scalar loads even
// in kernels that also store to global memory (where a plain load could
// alias a store and would have to be a vector load).
template <typename T>
__host__ __forceinline__ T geo_ld(const T *p) {
  return *p;
}
template <typename T>
__device__ __forceinline__ T geo_ld(const T *p) {
  return *(const __attribute__((address_space(4))) T *)p;
}

// Per lane only the row, the ends of the mesh it lies on and the absent
// directions; the steps between neighbours are the same for all rows of a
// mesh (scalar registers when the mesh is uniform over the wavefront).
template <int DIM>
struct BoxNbr {
  const BoxGeom *g;
  int32_t i;
  uint32_t ends;  // bit 2d: row on the low end along d; bit 2d+1: high end
  uint32_t bad;   // bits of `ends` without a neighbour (walls); all bits
                  // for an isolated (padding) row
  int32_t stride[3], wrap[3];  // step to the next node along d; step across
                               // the periodic seam, (n_d - 1) stride_d

  __host__ __device__ __forceinline__ BoxNbr(const BoxGeom *geo, int64_t row)
      : g(geo), i((int32_t)row), ends(0), bad(0) {
    const uint32_t li = (uint32_t)(row - geo_ld(&g->base));
    const bool iso = li >= (uint32_t)geo_ld(&g->nn);
    uint32_t a[3] = {0, 0, 0};
    if (!iso) {
      const uint32_t n0 = (uint32_t)geo_ld(&g->n[0]);
      const uint32_t t = li / n0;
      a[0] = li - t * n0;
      if constexpr (DIM == 3) {
        const uint32_t n1 = (uint32_t)geo_ld(&g->n[1]);
        a[2] = t / n1;
        a[1] = t - a[2] * n1;
      } else {
        a[1] = t;
      }
    }
    int32_t st = 1;
    uint32_t wall = 0;
    const int32_t per = geo_ld(&g->per);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      stride[d] = st;
      wrap[d] = 0;
      if (d >= DIM) continue;
      const int32_t n = geo_ld(&g->n[d]);
      wrap[d] = (n - 1) * st;
      if (a[d] == 0) ends |= 1u << (2 * d);
      if ((int32_t)a[d] == n - 1) ends |= 2u << (2 * d);
      if (!((per >> d) & 1)) wall |= 3u << (2 * d);
      st *= n;
    }
    bad = iso ? 0x3fu : (ends & wall);
  }

  // Column of slot k, -1 if the entry is absent.  With k known at compile
  // time (unrolled loops) the offsets fold away.
  __host__ __device__ __forceinline__ int32_t operator[](int k) const {
    const int o[3] = {k % 3 - 1, (k / 3) % 3 - 1, DIM == 3 ? k / 9 - 1 : 0};
    int32_t j = i;
    uint32_t m = 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      if (o[d] < 0) {
        j += (ends >> (2 * d)) & 1u ? wrap[d] : -stride[d];
        m |= 1u << (2 * d);
      } else if (o[d] > 0) {
        j += (ends >> (2 * d)) & 2u ? -wrap[d] : stride[d];
        m |= 2u << (2 * d);
      }
    }
    return (bad & m) ? -1 : j;
  }

  // Called where a chunk of a row's entries starts: the columns and
  // coefficients of later chunks depend on no load, and without it the
  // compiler computes all of them ahead and keeps them live (over 200
  // registers in 3D).  Emits no instruction.
  __device__ __forceinline__ void fence() {
    asm volatile("" : "+v"(i), "+v"(ends), "+v"(bad));
  }

  // An isolated row has both ends along x set in `bad`, which no mesh node
  // has (every direction has at least 2 nodes).
  __host__ __device__ __forceinline__ bool isolated() const { return (bad & 3u) == 3u; }

  // 1D factors of slot k along d: mass factor and gradient factor (+-1/2 off
  // the diagonal; on it -1/2 at a low wall end, +1/2 at a high one, else 0).
  __host__ __device__ __forceinline__ void factors(int k, double *f, double *c1) const {
    const int o[3] = {k % 3 - 1, (k / 3) % 3 - 1, DIM == 3 ? k / 9 - 1 : 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      if (o[d] != 0) {
        f[d] = geo_ld(&g->m_off[d]);
        c1[d] = o[d] < 0 ? -0.5 : 0.5;
      } else {
        const uint32_t w = (bad >> (2 * d)) & 3u;
        f[d] = w ? geo_ld(&g->m_end[d]) : geo_ld(&g->m_inner[d]);
        c1[d] = w == 1u ? -0.5 : (w == 2u ? 0.5 : 0.0);
      }
    }
  }

  // m_ij of slot k: the product of the mass factors (1 on the diagonal of an
  // isolated row).  Meaningful where the entry is present.
  __host__ __device__ __forceinline__ double mass(int k) const {
    double f[3], c1[3];
    factors(k, f, c1);
    double m = 1.0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) m *= f[d];
    return isolated() ? (k == (DIM == 2 ? 4 : 13) ? 1.0 : 0.0) : m;
  }

  // c_ij of slot k: component e is the gradient factor along e times the
  // mass factors of the other directions (0 on an isolated row).
  __host__ __device__ __forceinline__ void grad(int k, double *c) const {
    double f[3], c1[3];
    factors(k, f, c1);
    const bool iso = isolated();
#pragma unroll
    for (int e = 0; e < DIM; ++e) {
      double v = c1[e];
#pragma unroll
      for (int d = 0; d < DIM; ++d)
        if (d != e) v *= f[d];
      c[e] = iso ? 0.0 : v;
    }
  }
};

// c_ji from c_ij for the entry in slot k: the offset is reversed, the nodes
// share their wall ends along the directions the offset does not move, so
// the components along moved directions change sign and the others stay
// (exact: the products only differ in the sign of one factor).
template <int DIM>
__host__ __device__ __forceinline__ void grad_transposed(int k, const double *c, double *ct) {
  const int o[3] = {k % 3 - 1, (k / 3) % 3 - 1, DIM == 3 ? k / 9 - 1 : 0};
#pragma unroll
  for (int e = 0; e < DIM; ++e) ct[e] = o[e] != 0 ? -c[e] : c[e];
}

// Slot of the transposed entry: the opposite offset.
template <int DIM>
__host__ __device__ __forceinline__ constexpr int tslot(int k) {
  return (DIM == 2 ? 9 : 27) - 1 - k;
}

}  // namespace ns
