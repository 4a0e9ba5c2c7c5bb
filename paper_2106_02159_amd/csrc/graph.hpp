// graph.hpp -- closed-form Q1 stencil graph of a uniform box mesh.
//
// The quantities of Sec. 2.2 (m_i, m_ij, c_ij) and the boundary integrals of
// eq. unit_normal_vector are tensor products of 1D factors on a uniform
// mesh, so they are written here in closed form rather than assembled by
// quadrature.  1D factors with mesh size h for node a and neighbour offset o:
//   mass      m1(a, 0) = 2h/3 (h/3 at a wall end),  m1(a, +-1) = h/6
//   gradient  c1(a, +-1) = +-1/2, c1(a, 0) = 0 (-1/2 at the low wall end,
//             +1/2 at the high wall end)
//   lumped    ml(a) = h (h/2 at a wall end)
//   boundary  bn1(a) = -1 at the low wall end, +1 at the high end, else 0.
// Multi-D: m_ij = prod_d m1_d, c_ij[e] = c1_e prod_{d != e} m1_d,
// m_i = prod_d ml_d, int phi_i n_e = bn1_e prod_{d != e} ml_d.  The products
// are formed in the same order for (i,j) and (j,i), so c_ij = -c_ji holds
// bit for bit whenever one of the two nodes is interior.
//
// Storage is slot-major ELL: entry (slot k, node i) at k*N + i, W = 3^dim
// slots, slot k <-> offset (dx,dy,dz) with k = (dx+1) + 3(dy+1) + 9(dz+1).
#pragma once

#include <cstdint>

namespace ns {

struct MeshGraph {
  int dim = 0;
  int64_t n[3] = {1, 1, 1};
  int periodic[3] = {0, 0, 0};
  double lo[3] = {0, 0, 0};
  double hi[3] = {0, 0, 0};
  double h[3] = {1, 1, 1};
  int64_t N = 0;
  int W = 0;          // 3^dim
  int64_t nnz = 0;    // valid entries

  // 1D factors
  bool wall_lo(int d, int64_t a) const { return !periodic[d] && a == 0; }
  bool wall_hi(int d, int64_t a) const { return !periodic[d] && a == n[d] - 1; }
  // neighbour index along d, or -1 outside a wall-bounded direction
  int64_t nb1(int d, int64_t a, int o) const;
  double m1(int d, int64_t a, int o) const;
  // the three values of m1 along d: diagonal of an interior node, diagonal
  // at a wall end, off-diagonal
  void m1_values(int d, double *inner, double *end, double *off) const;
  double c1(int d, int64_t a, int o) const;
  double ml(int d, int64_t a) const;
  double bn1(int d, int64_t a) const;

  void coords(int64_t i, int64_t a[3]) const;
  void slot_offset(int k, int o[3]) const;
  bool on_wall(int64_t i) const;

  // One ELL slot for all nodes: col (-1 if missing), transpose slot, m_ij
  // and the dim components of c_ij.  Any output may be null.
  void fill_slot(int k, int32_t *col, uint8_t *trk, double *mij,
                 double *const *cij) const;
  void fill_nodes(double *mi, double *bnd /* dim*N */, uint8_t *wall) const;
};

int build_mesh_graph(int dim, const int64_t *n, const double *lo,
                     const double *hi, const int *periodic, MeshGraph *g,
                     const char **why);

}  // namespace ns
