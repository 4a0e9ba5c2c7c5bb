// element.hpp -- closed-form Q1 element matrices of the parabolic operators
// on a uniform box cell, and the tensor Gauss rule used for the dissipation.
//
// On a box cell with sizes h_d the integrals of products of Q1 shape
// functions and their derivatives are products of 1D factors (local node
// a has bit a_d = 0 / 1 at the low / high end of direction d):
//   int phi_s phi_t     = h/3 (s == t), h/6 (s != t)
//   int phi_s' phi_t'   = 1/h (s == t), -1/h (s != t)
//   int phi_s' phi_t    = -1/2 (s = 0), +1/2 (s = 1)      (any t)
// so that S^pq_ab = int d_p phi_a d_q phi_b is
//   p == q:  K(p) * prod_{c != p} M(c)
//   p != q:  D_p(a_p) D_q(b_q) * prod_{c != p,q} M(c).
// The stress form a(v, w) = int sigma(v) : eps(w), sigma = 2 mu eps(v) +
// (lambda - 2/3 mu) div(v) I, gives for trial phi_b e_l and test phi_a e_k
//   E^kl_ab = mu (delta_kl sum_c S^cc_ab + S^lk_ab) + (lambda - 2/3 mu) S^kl_ab
// and the heat form b(e, w) = (kappa/cv) int grad e . grad w gives
//   L_ab = (kappa/cv) sum_c S^cc_ab.
#pragma once

#include <cstddef>
#include <vector>

namespace ns {

struct Q1Tables {
  int dim = 0, nloc = 0;
  // stress[((k*dim + l)*nloc + a)*nloc + b] = E^kl_ab
  std::vector<double> stress;
  // heat[a*nloc + b] = L_ab
  std::vector<double> heat;
  // Gauss rule with 2 points per direction on the cell: weight w (equal for
  // all points), phi[q*nloc + a], dphi[(q*nloc + a)*dim + p]
  double w = 0.0;
  std::vector<double> phi, dphi;
  // The operators' rows at a node all of whose 2^dim cells exist, summed
  // over the cells: stencil_stress[(s*dim + k)*dim + l] couples component k
  // of the node with component l of its neighbour in slot s (offset
  // o_d = (s / 3^d) % 3 - 1), stencil_heat[s] likewise.
  std::vector<double> stencil_stress, stencil_heat;

  // layout of the single device table:
  // stress | heat | phi | dphi | w | stencil_stress | stencil_heat
  std::size_t off_heat() const { return stress.size(); }
  std::size_t off_phi() const { return off_heat() + heat.size(); }
  std::size_t off_dphi() const { return off_phi() + phi.size(); }
  std::size_t off_w() const { return off_dphi() + dphi.size(); }
  std::size_t off_sst() const { return off_w() + 1; }
  std::size_t off_sht() const { return off_sst() + stencil_stress.size(); }
  std::vector<double> packed() const;
};

void build_q1_tables(int dim, const double *h, double mu, double lambda,
                     double kappa_over_cv, Q1Tables *t);

}  // namespace ns
