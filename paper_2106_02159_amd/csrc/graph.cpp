// graph.cpp -- closed-form Q1 stencil graph (see graph.hpp).
#include "graph.hpp"

#include <cmath>

namespace ns {

int64_t MeshGraph::nb1(int d, int64_t a, int o) const {
  const int64_t b = a + o;
  if (periodic[d]) return (b + n[d]) % n[d];
  if (b < 0 || b >= n[d]) return -1;
  return b;
}

void MeshGraph::m1_values(int d, double *inner, double *end, double *off) const {
  *inner = 2.0 * h[d] / 3.0;
  *end = h[d] / 3.0;
  *off = h[d] / 6.0;
}

double MeshGraph::m1(int d, int64_t a, int o) const {
  double inner, end, off;
  m1_values(d, &inner, &end, &off);
  if (o != 0) return off;
  if (wall_lo(d, a) || wall_hi(d, a)) return end;
  return inner;
}

double MeshGraph::c1(int d, int64_t a, int o) const {
  if (o == 1) return 0.5;
  if (o == -1) return -0.5;
  // o == 0: int phi_a phi_a' = [phi_a^2 / 2] over the support
  double v = 0.0;
  if (wall_lo(d, a)) v -= 0.5;
  if (wall_hi(d, a)) v += 0.5;
  return v;
}

double MeshGraph::ml(int d, int64_t a) const {
  if (wall_lo(d, a) || wall_hi(d, a)) return 0.5 * h[d];
  return h[d];
}

double MeshGraph::bn1(int d, int64_t a) const {
  double v = 0.0;
  if (wall_lo(d, a)) v -= 1.0;
  if (wall_hi(d, a)) v += 1.0;
  return v;
}

void MeshGraph::coords(int64_t i, int64_t a[3]) const {
  a[0] = i % n[0];
  a[1] = (i / n[0]) % n[1];
  a[2] = i / (n[0] * n[1]);
}

void MeshGraph::slot_offset(int k, int o[3]) const {
  o[0] = k % 3 - 1;
  o[1] = (k / 3) % 3 - 1;
  o[2] = k / 9 - 1;
  if (dim == 2) o[2] = 0;
}

bool MeshGraph::on_wall(int64_t i) const {
  int64_t a[3];
  coords(i, a);
  for (int d = 0; d < dim; ++d)
    if (wall_lo(d, a[d]) || wall_hi(d, a[d])) return true;
  return false;
}

void MeshGraph::fill_slot(int k, int32_t *col, uint8_t *trk, double *mij,
                          double *const *cij) const {
  int o[3];
  slot_offset(k, o);
  const int kt = W - 1 - k;  // slot of the opposite offset
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    int64_t a[3], b[3];
    coords(i, a);
    bool ok = true;
    for (int d = 0; d < 3; ++d) {
      if (d < dim) {
        b[d] = nb1(d, a[d], o[d]);
        if (b[d] < 0) ok = false;
      } else {
        b[d] = 0;
      }
    }
    if (!ok) {
      if (col) col[i] = -1;
      if (trk) trk[i] = 0;
      if (mij) mij[i] = 0.0;
      if (cij)
        for (int e = 0; e < dim; ++e) cij[e][i] = 0.0;
      continue;
    }
    const int64_t j = b[0] + n[0] * (b[1] + n[1] * b[2]);
    if (col) col[i] = (int32_t)j;
    if (trk) trk[i] = (uint8_t)kt;
    if (mij) {
      double m = 1.0;
      for (int d = 0; d < dim; ++d) m *= m1(d, a[d], o[d]);
      mij[i] = m;
    }
    if (cij) {
      for (int e = 0; e < dim; ++e) {
        double c = c1(e, a[e], o[e]);
        for (int d = 0; d < dim; ++d)
          if (d != e) c *= m1(d, a[d], o[d]);
        cij[e][i] = c;
      }
    }
  }
}

void MeshGraph::fill_nodes(double *mi, double *bnd, uint8_t *wall) const {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < N; ++i) {
    int64_t a[3];
    coords(i, a);
    if (mi) {
      double m = 1.0;
      for (int d = 0; d < dim; ++d) m *= ml(d, a[d]);
      mi[i] = m;
    }
    if (bnd) {
      for (int e = 0; e < dim; ++e) {
        double v = bn1(e, a[e]);
        for (int d = 0; d < dim; ++d)
          if (d != e) v *= ml(d, a[d]);
        bnd[(int64_t)e * N + i] = v;
      }
    }
    if (wall) wall[i] = on_wall(i) ? 1 : 0;
  }
}

int build_mesh_graph(int dim, const int64_t *n, const double *lo,
                     const double *hi, const int *periodic, MeshGraph *g,
                     const char **why) {
  if (dim != 2 && dim != 3) { *why = "dim must be 2 or 3"; return -1; }
  g->dim = dim;
  g->W = dim == 2 ? 9 : 27;
  int64_t N = 1;
  for (int d = 0; d < 3; ++d) {
    if (d < dim) {
      g->n[d] = n[d];
      g->periodic[d] = periodic[d] ? 1 : 0;
      g->lo[d] = lo[d];
      g->hi[d] = hi[d];
      if (g->periodic[d] ? n[d] < 3 : n[d] < 2) {
        *why = "too few nodes (periodic directions need n >= 3, walls n >= 2)";
        return -1;
      }
      if (!(hi[d] > lo[d]) || !std::isfinite(hi[d] - lo[d])) {
        *why = "box must have lo < hi";
        return -1;
      }
      g->h[d] = (hi[d] - lo[d]) / (double)(g->periodic[d] ? n[d] : n[d] - 1);
    } else {
      g->n[d] = 1; g->periodic[d] = 0; g->lo[d] = 0; g->hi[d] = 0; g->h[d] = 1;
    }
    N *= g->n[d];
    if (N > 2147483647LL) { *why = "more than 2^31-1 nodes"; return -1; }
  }
  g->N = N;
  // valid entries: product over directions of the 1D row lengths summed
  int64_t nnz = 1;
  for (int d = 0; d < dim; ++d) {
    const int64_t m = g->n[d];
    nnz *= g->periodic[d] ? 3 * m : 3 * m - 2;
  }
  g->nnz = nnz;
  return 0;
}

}  // namespace ns
