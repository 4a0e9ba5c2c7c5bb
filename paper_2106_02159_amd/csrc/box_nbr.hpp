// box_nbr.hpp -- column index of every entry of the Q1 stencil graph of a
// uniform box mesh, derived from the row index instead of loaded.
//
// The nodes of a box mesh are numbered lexicographically (x fastest) and the
// neighbour in slot k = (dx+1) + 3(dy+1) + 9(dz+1) is the node at offset
// (dx,dy,dz), wrapped in a periodic direction and absent beyond a wall.  The
// transposed entry (j,i) of (i,j) is therefore in slot W-1-k of row j.  The
// row sweeps compute both instead of reading an index array per entry: 4+1
// bytes per entry less to move, and a row's neighbour gathers no longer wait
// for the index loads.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace ns {

// One box mesh inside the row numbering of a solver: rows base .. base+nn-1
// are its nodes; rows from base+nn up to the next mesh (padding rows of a
// pack) are isolated nodes whose only entry is the diagonal one.
struct BoxGeom {
  int32_t base;
  int32_t nn;
  int32_t n[3];  // nodes per direction (n[2] = 1 in 2D)
  int32_t per;   // bit d set: direction d is periodic
};

// Per lane only the row, the ends of the mesh it lies on and the absent
// directions; the steps between neighbours are the same for all rows of a
// mesh (scalar registers when the mesh is uniform over the wavefront).
template <int DIM>
struct BoxNbr {
  int32_t i;
  uint32_t ends;  // bit 2d: row on the low end along d; bit 2d+1: high end
  uint32_t bad;   // bits of `ends` without a neighbour (walls); all bits
                  // for an isolated (padding) row
  int32_t stride[3], wrap[3];  // step to the next node along d; step across
                               // the periodic seam, (n_d - 1) stride_d

  __host__ __device__ __forceinline__ BoxNbr(const BoxGeom &g, int64_t row)
      : i((int32_t)row), ends(0), bad(0) {
    const uint32_t li = (uint32_t)(row - g.base);
    const bool iso = li >= (uint32_t)g.nn;
    uint32_t a[3] = {0, 0, 0};
    if (!iso) {
      const uint32_t t = li / (uint32_t)g.n[0];
      a[0] = li - t * (uint32_t)g.n[0];
      if constexpr (DIM == 3) {
        a[2] = t / (uint32_t)g.n[1];
        a[1] = t - a[2] * (uint32_t)g.n[1];
      } else {
        a[1] = t;
      }
    }
    int32_t st = 1;
    uint32_t wall = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      stride[d] = st;
      wrap[d] = 0;
      if (d >= DIM) continue;
      const int32_t n = g.n[d];
      wrap[d] = (n - 1) * st;
      if (a[d] == 0) ends |= 1u << (2 * d);
      if ((int32_t)a[d] == n - 1) ends |= 2u << (2 * d);
      if (!((g.per >> d) & 1)) wall |= 3u << (2 * d);
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
};

// Slot of the transposed entry: the opposite offset.
template <int DIM>
__host__ __device__ __forceinline__ constexpr int tslot(int k) {
  return (DIM == 2 ? 9 : 27) - 1 - k;
}

}  // namespace ns
