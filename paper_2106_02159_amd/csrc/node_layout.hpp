// node_layout.hpp -- where the components of a node vector (a state, U^L,
// F^H, U^(1): K = dim + 2 components per node) sit in device memory.
//
// Components are stored in pairs: components 2p and 2p+1 of node i are
// neighbours, at 2pN + 2i and 2pN + 2i + 1, so that one 16-byte load (8 bytes
// in FP32) brings both and the lanes of a wavefront reading consecutive nodes
// read one contiguous run.  With K odd the last component is alone, at
// (K-1)N + i.  The array holds K*N entries, as a component-major one would.
//
// The row sweeps gather the state of every neighbour of their row; such a
// gather costs ceil(K/2) load instructions here instead of K, and on these
// sweeps the cost per load instruction, not the bytes, is what the gathers
// are bound by (a 9-point gather of 8 doubles per neighbour: 0.63 ms with
// 8-byte loads, 0.46 ms with 16-byte loads of the same bytes, at 4096^2).
// The C interface keeps component-major arrays (component c of node i at
// cN + i); ns_api converts at the boundary.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace ns {

// Offset of component c of node i in a K-component node vector of N nodes.
__host__ __device__ __forceinline__ constexpr int64_t node_at(int K, int c, int64_t i,
                                                              int64_t N) {
  return (int64_t)(c & ~1) * N + ((c | 1) < K ? 2 * i + (c & 1) : i);
}

}  // namespace ns
