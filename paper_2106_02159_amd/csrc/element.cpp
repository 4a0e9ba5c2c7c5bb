// element.cpp -- closed-form Q1 element matrices (see element.hpp).
#include "element.hpp"

#include <cmath>

namespace ns {

namespace {

double mass1(double h, int s, int t) { return s == t ? h / 3.0 : h / 6.0; }
double stiff1(double h, int s, int t) { return s == t ? 1.0 / h : -1.0 / h; }
double deriv1(int s) { return s ? 0.5 : -0.5; }

// S^pq_ab = int d_p phi_a d_q phi_b over the cell
double S(int dim, const double *h, int p, int q, int a, int b) {
  double v = 1.0;
  for (int c = 0; c < dim; ++c) {
    const int ac = (a >> c) & 1, bc = (b >> c) & 1;
    if (p == q && c == p) v *= stiff1(h[c], ac, bc);
    else if (p != q && c == p) v *= deriv1(ac);
    else if (p != q && c == q) v *= deriv1(bc);
    else v *= mass1(h[c], ac, bc);
  }
  return v;
}

}  // namespace

void build_interior_stencils(Q1Tables *t);

void build_q1_tables(int dim, const double *h, double mu, double lambda,
                     double kappa_over_cv, Q1Tables *t) {
  const int n = 1 << dim;
  t->dim = dim;
  t->nloc = n;
  t->stress.assign((size_t)dim * dim * n * n, 0.0);
  t->heat.assign((size_t)n * n, 0.0);
  const double lam23 = lambda - 2.0 / 3.0 * mu;
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      double lap = 0.0;
      for (int c = 0; c < dim; ++c) lap += S(dim, h, c, c, a, b);
      t->heat[(size_t)a * n + b] = kappa_over_cv * lap;
      for (int k = 0; k < dim; ++k)
        for (int l = 0; l < dim; ++l) {
          double v = mu * S(dim, h, l, k, a, b) + lam23 * S(dim, h, k, l, a, b);
          if (k == l) v += mu * lap;
          t->stress[(((size_t)k * dim + l) * n + a) * n + b] = v;
        }
    }
  // Gauss points 1/2 -+ 1/(2 sqrt 3) on [0,1] per direction
  const double g[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  double vol = 1.0;
  for (int c = 0; c < dim; ++c) vol *= h[c];
  t->w = vol / n;
  t->phi.assign((size_t)n * n, 0.0);
  t->dphi.assign((size_t)n * n * dim, 0.0);
  for (int q = 0; q < n; ++q)
    for (int a = 0; a < n; ++a) {
      double f = 1.0;
      for (int c = 0; c < dim; ++c) {
        const double x = g[(q >> c) & 1];
        f *= ((a >> c) & 1) ? x : 1.0 - x;
      }
      t->phi[(size_t)q * n + a] = f;
      for (int p = 0; p < dim; ++p) {
        double d = (((a >> p) & 1) ? 1.0 : -1.0) / h[p];
        for (int c = 0; c < dim; ++c) {
          if (c == p) continue;
          const double x = g[(q >> c) & 1];
          d *= ((a >> c) & 1) ? x : 1.0 - x;
        }
        t->dphi[((size_t)q * n + a) * dim + p] = d;
      }
    }
  build_interior_stencils(t);
}

namespace {
// neighbourhood slot of local node b seen from local node a of the same cell
int slot_of(int dim, int a, int b) {
  int s = 0, m = 1;
  for (int d = 0; d < dim; ++d) {
    s += (((b >> d) & 1) - ((a >> d) & 1) + 1) * m;
    m *= 3;
  }
  return s;
}
}  // namespace

void build_interior_stencils(Q1Tables *t) {
  const int dim = t->dim, n = t->nloc;
  int S = 1;
  for (int d = 0; d < dim; ++d) S *= 3;
  t->stencil_stress.assign((size_t)S * dim * dim, 0.0);
  t->stencil_heat.assign((size_t)S, 0.0);
  // node i is local node a of one of its 2^dim cells; b runs over that cell
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      const int s = slot_of(dim, a, b);
      t->stencil_heat[s] += t->heat[(size_t)a * n + b];
      for (int k = 0; k < dim; ++k)
        for (int l = 0; l < dim; ++l)
          t->stencil_stress[((size_t)s * dim + k) * dim + l] +=
              t->stress[(((size_t)k * dim + l) * n + a) * n + b];
    }
}

std::vector<double> Q1Tables::packed() const {
  std::vector<double> v;
  v.reserve(off_w() + 1);
  v.insert(v.end(), stress.begin(), stress.end());
  v.insert(v.end(), heat.begin(), heat.end());
  v.insert(v.end(), phi.begin(), phi.end());
  v.insert(v.end(), dphi.begin(), dphi.end());
  v.push_back(w);
  v.insert(v.end(), stencil_stress.begin(), stencil_stress.end());
  v.insert(v.end(), stencil_heat.begin(), stencil_heat.end());
  return v;
}

}  // namespace ns
