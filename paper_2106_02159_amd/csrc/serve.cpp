// serve.cpp -- continuous batching of independent simulations on one GPU.
//
// Each request is a uniform-mesh Euler problem (mesh, initial state, number
// of SSPRK(3,3) steps with the CFL time step).  Requests wait in a FIFO queue
// and are admitted, in order, whenever their device footprint fits in the
// server's memory budget beside the running ones (and the number of running
// units is below the limit).  A unit is either one request with its own
// solver, or -- for meshes of at most half the pack size -- a pack: the
// consecutive queued requests with the same step count whose rows fit in
// one pack, advanced by the same kernel launches (ns_pack_*), each with its
// own time step.  Each unit runs on its own HIP stream.  Its steps are
// enqueued in small chunks, at most `depth` chunks in flight, without host
// synchronization: every progress call tops up each running unit by one
// chunk (round robin), so the running units advance together -- a small
// request is never queued behind the whole run of a large one on a hardware
// queue -- and their kernels overlap on the device.  ns_server_progress also
// collects finished units (copying their states to host memory and freeing
// their device memory, which lets the next queued requests in) and admits
// new ones; it never blocks on the device.  Each request's result depends
// only on its own input: the kernels are deterministic, requests share no
// device data, and a pack member's result is bit-identical to its own
// solver's.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <future>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/ns.h"
#include "device.hpp"

namespace {

double now_s() {
  using clk = std::chrono::steady_clock;
  return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

enum { QUEUED = 0, RUNNING = 1, FINISHED = 2 };

struct Request {
  int64_t id = 0;
  ns_mesh_desc mesh{};
  std::vector<double> u0;
  int steps = 0;
  int state = QUEUED;
  ns_graph *g = nullptr;
  int64_t N = 0, rows = 0;  // nodes; rows in a pack (N rounded up to 256)
  int dim = 0;
  int64_t bytes = 0;        // footprint of its own solver
  double t_submit = 0, t_admit = 0, t_finish = 0;
  double t_sim = 0.0;
  int status = NS_OK;
  std::string error;
  std::vector<double> out;
};

// One request with its own solver, or a pack of several.  The solver or
// pack is created and given its states in a worker thread (graph set-up
// and uploads take host time in proportion to the mesh), while the
// progress calls keep the running units fed.
struct Unit {
  std::vector<Request *> mem;
  ns_solver *s = nullptr;
  ns_pack *k = nullptr;
  int steps = 0, enqueued = 0;
  int64_t bytes = 0;
  std::future<int> ready;  // set-up in a worker thread, until collected
  bool preparing = false;
  std::string err;         // set-up failure
};

}  // namespace

struct ns_server {
  ns_server_params prm{};
  int device = 0;  // the creating thread's device, for the set-up threads
  std::deque<Request *> queue;
  std::vector<Unit *> running;
  std::map<int64_t, std::unique_ptr<Request>> all;
  int64_t used = 0;
  int64_t next_id = 1;
  ns_server_stats st{};
  std::string err = "no error";
};

namespace {

void release_graph(Request *r) {
  if (r->g) ns_graph_destroy(r->g);
  r->g = nullptr;
}

void release(ns_server *sv, Unit *u) {
  if (u->s) ns_solver_destroy(u->s);
  if (u->k) ns_pack_destroy(u->k);
  u->s = nullptr;
  u->k = nullptr;
  for (Request *r : u->mem) release_graph(r);
  sv->used -= u->bytes;
}

const char *unit_error(const Unit *u) {
  return u->k ? ns_pack_error(u->k) : u->s ? ns_last_error(u->s) : ns_create_error();
}

// rows of a unit: its mesh, or its members padded to whole workgroups
int64_t unit_rows(const Unit *u) {
  if (u->mem.size() == 1) return u->mem[0]->N;
  int64_t n = 0;
  for (const Request *r : u->mem) n += r->rows;
  return n;
}

// Wait limit of the persistent launches: far above any chunk's run time, so
// that it only ends a launch that can no longer progress.
constexpr double kPersistWaitS = 10.0;

// enqueue the next chunk of steps: one persistent launch for a unit of at
// most persistent_rows rows, else the captured step graphs
int top_up(ns_server *sv, Unit *u) {
  const int k = std::min(sv->prm.chunk, u->steps - u->enqueued);
  const bool pers = unit_rows(u) <= sv->prm.persistent_rows;
  int rc;
  if (pers)
    rc = u->k ? ns_pack_step_cfl_persistent(u->k, k, kPersistWaitS)
              : ns_step_cfl_persistent(u->s, k, kPersistWaitS);
  else
    rc = u->k ? ns_pack_step_cfl_async(u->k, k) : ns_step_cfl_async(u->s, k);
  if (rc == NS_OK) u->enqueued += k;
  return rc;
}

int inflight(Unit *u, int *n) {
  return u->k ? ns_pack_inflight(u->k, n) : ns_inflight(u->s, n);
}

// Worker thread: create the unit's solver or pack and set the states.
int prepare(const ns_params prm, int device, Unit *u) {
  ns::use_device(device);
  int rc;
  if (u->mem.size() == 1) {
    Request *r = u->mem[0];
    rc = ns_solver_create(r->g, &prm, nullptr, &u->s);
    if (rc == NS_OK) rc = ns_set_state(u->s, r->u0.data(), 0);
  } else {
    std::vector<const ns_graph *> gs;
    for (Request *r : u->mem) gs.push_back(r->g);
    rc = ns_pack_create(gs.data(), (int)gs.size(), &prm, nullptr, &u->k);
    for (size_t m = 0; rc == NS_OK && m < u->mem.size(); ++m)
      rc = ns_pack_set_state(u->k, (int)m, u->mem[m]->u0.data());
  }
  if (rc != NS_OK) u->err = unit_error(u);
  return rc;
}

// Main thread, once the set-up is done: enqueue the first chunk.
int start(ns_server *sv, Unit *u) {
  u->preparing = false;
  int rc = u->ready.get();
  if (rc == NS_OK) {
    rc = top_up(sv, u);
    if (rc != NS_OK) u->err = unit_error(u);
  }
  for (Request *r : u->mem) {
    if (rc != NS_OK) r->error = u->err;
    std::vector<double>().swap(r->u0);
  }
  return rc;
}

void finish_request(ns_server *sv, Request *r, int status) {
  r->status = status;
  r->t_finish = now_s();
  r->state = FINISHED;
  sv->st.finished += 1;
}

// all steps done (rc NS_OK) or the unit failed (rc): collect its requests
void finish(ns_server *sv, Unit *u, int rc) {
  const size_t n = u->mem.size();
  std::vector<int> st(n, rc);
  std::vector<double> t(n, 0.0);
  if (rc == NS_OK) {
    if (u->k) {
      rc = ns_pack_finish(u->k, st.data(), t.data());
      if (rc != NS_OK) std::fill(st.begin(), st.end(), rc);
    } else {
      st[0] = ns_async_finish(u->s, &t[0]);
    }
  }
  for (size_t m = 0; m < n; ++m) {
    Request *r = u->mem[m];
    r->t_sim = t[m];
    int s = st[m];
    if (s == NS_OK || s == NS_ECFL || s == NS_EBOUNDS) {  // (not NS_EABORT)
      r->out.resize((size_t)(r->dim + 2) * r->N);
      const int rg = u->k ? ns_pack_get_state(u->k, (int)m, r->out.data())
                          : ns_get_state(u->s, r->out.data(), 0);
      if (s == NS_OK) s = rg;
    }
    if (s != NS_OK && r->error.empty()) r->error = u->err.empty() ? unit_error(u) : u->err;
    finish_request(sv, r, s);
  }
  release(sv, u);
  delete u;
}

// The unit to admit next: the queue head alone, or the head and the
// consecutive queued requests with its step count that fit in a pack (and
// in the memory left).  Empty if the head does not fit.
Unit *next_unit(ns_server *sv) {
  Request *h = sv->queue.front();
  const int64_t free_bytes = sv->prm.mem_bytes - sv->used;
  const int64_t cap = sv->prm.pack_nodes;
  std::vector<Request *> mem{h};
  if (cap > 0 && h->rows * 2 <= cap) {
    int64_t rows = h->rows;
    for (size_t q = 1; q < sv->queue.size() && (int)mem.size() < sv->prm.pack_max; ++q) {
      Request *r = sv->queue[q];
      if (r->steps != h->steps || r->dim != h->dim || r->rows * 2 > cap ||
          rows + r->rows > cap)
        break;
      mem.push_back(r);
      rows += r->rows;
    }
  }
  // shrink to the memory left
  while (!mem.empty()) {
    int64_t b = 0;
    if (mem.size() == 1) {
      b = mem[0]->bytes;
    } else {
      std::vector<const ns_graph *> gs;
      for (Request *r : mem) gs.push_back(r->g);
      if (ns_pack_footprint(gs.data(), (int)gs.size(), &sv->prm.solver, &b) != NS_OK)
        b = INT64_MAX;
    }
    if (b <= free_bytes) {
      Unit *u = new Unit;
      u->mem = mem;
      u->steps = h->steps;
      u->bytes = b;
      return u;
    }
    mem.pop_back();
  }
  return nullptr;
}

}  // namespace

extern "C" {

int ns_server_create(const ns_server_params *p, ns_server **out) {
  if (!p || !out || p->mem_bytes <= 0 || p->max_running < 1 || p->chunk < 1 ||
      p->depth < 1 || p->pack_nodes < 0 || (p->pack_nodes > 0 && p->pack_max < 2) ||
      p->persistent_rows < 0)
    return NS_EINVAL;
  // persistent launches run the entropy indicator and two-pass convex limiting
  if (p->persistent_rows > 0 &&
      (p->solver.indicator != NS_IND_ENTROPY || p->solver.limiter != NS_LIM_CONVEX ||
       p->solver.passes != 2))
    return NS_EINVAL;
  ns_server *sv = new (std::nothrow) ns_server;
  if (!sv) return NS_ENOMEM;
  sv->prm = *p;
  sv->device = ns::current_device();
  *out = sv;
  return NS_OK;
}

void ns_server_destroy(ns_server *sv) {
  if (!sv) return;
  for (Unit *u : sv->running) {
    if (u->preparing) u->ready.wait();
    release(sv, u);  // waits for the unit's stream
    delete u;
  }
  for (auto &kv : sv->all) release_graph(kv.second.get());
  delete sv;
}

int ns_server_submit(ns_server *sv, const ns_mesh_desc *mesh, const double *U0,
                     int steps, int64_t *id) {
  if (!sv || !mesh || !U0 || !id || steps < 0) return NS_EINVAL;
  auto r = std::make_unique<Request>();
  r->mesh = *mesh;
  int rc = ns_graph_create(mesh, &r->g);
  if (rc != NS_OK) {
    sv->err = ns_create_error();
    return rc;
  }
  int64_t N = 0;
  int dim = 0;
  ns_graph_info(r->g, &N, nullptr, &dim, nullptr);
  rc = ns_solver_footprint(r->g, &sv->prm.solver, &r->bytes);
  if (rc != NS_OK) {
    ns_graph_destroy(r->g);
    return rc;
  }
  if (r->bytes > sv->prm.mem_bytes) {
    ns_graph_destroy(r->g);
    sv->err = "the request needs more device memory than the server's budget";
    return NS_ENOMEM;
  }
  // an inadmissible state is refused here, so that it never shares a pack
  for (int64_t i = 0; i < N; ++i) {
    const double rho = U0[i], E = U0[(dim + 1) * N + i];
    double m2 = 0.0;
    bool ok = std::isfinite(rho) && std::isfinite(E);
    for (int d = 0; d < dim; ++d) {
      const double mk = U0[(1 + d) * N + i];
      ok = ok && std::isfinite(mk);
      m2 += mk * mk;
    }
    if (!ok || !(rho > 0.0) || !(E - 0.5 * m2 / rho > 0.0)) {
      ns_graph_destroy(r->g);
      sv->err = "initial state not admissible at node " + std::to_string(i);
      return NS_ENOTADMISSIBLE;
    }
  }
  r->u0.assign(U0, U0 + (size_t)(dim + 2) * N);
  r->N = N;
  r->dim = dim;
  r->rows = (N + 255) / 256 * 256;
  r->steps = steps;
  r->id = sv->next_id++;
  r->t_submit = now_s();
  *id = r->id;
  sv->queue.push_back(r.get());
  sv->all[r->id] = std::move(r);
  sv->st.submitted += 1;
  return NS_OK;
}

int ns_server_progress(ns_server *sv, int *n_finished) {
  if (!sv) return NS_EINVAL;
  const int64_t before = sv->st.finished;
  // top up running units by one chunk each; collect finished ones
  for (size_t k = 0; k < sv->running.size();) {
    Unit *u = sv->running[k];
    int n = 0;
    int rc = NS_OK;
    if (u->preparing) {
      if (u->ready.wait_for(std::chrono::seconds(0)) != std::future_status::ready) {
        ++k;
        continue;
      }
      const double t0 = now_s();
      rc = start(sv, u);
      sv->st.host_admit_s += now_s() - t0;
      if (rc == NS_OK) {
        ++k;
        continue;
      }
    }
    if (rc == NS_OK) rc = inflight(u, &n);
    if (rc == NS_OK && u->enqueued < u->steps) {
      if (n < sv->prm.depth) {
        const double t0 = now_s();
        rc = top_up(sv, u);
        sv->st.host_topup_s += now_s() - t0;
      }
      if (rc == NS_OK) {
        ++k;
        continue;
      }
    }
    if (rc == NS_OK && n > 0) {
      ++k;
      continue;
    }
    sv->running.erase(sv->running.begin() + k);
    const double t0 = now_s();
    finish(sv, u, rc);
    sv->st.host_finish_s += now_s() - t0;
  }
  // admit queued requests, in order, while they fit
  while (!sv->queue.empty() && (int)sv->running.size() < sv->prm.max_running) {
    Unit *u = next_unit(sv);
    if (!u) break;
    for (size_t m = 0; m < u->mem.size(); ++m) sv->queue.pop_front();
    sv->used += u->bytes;
    sv->st.units += 1;
    const double t0 = now_s();
    for (Request *r : u->mem) {
      r->t_admit = t0;
      r->state = RUNNING;
    }
    u->ready = std::async(std::launch::async, prepare, sv->prm.solver, sv->device, u);
    u->preparing = true;
    sv->st.host_admit_s += now_s() - t0;
    sv->running.push_back(u);
    int64_t nreq = 0;
    for (Unit *v : sv->running) nreq += (int64_t)v->mem.size();
    sv->st.peak_running = std::max(sv->st.peak_running, nreq);
    sv->st.peak_bytes = std::max(sv->st.peak_bytes, sv->used);
  }
  if (n_finished) *n_finished = (int)(sv->st.finished - before);
  return NS_OK;
}

int ns_server_request(ns_server *sv, int64_t id, ns_request_info *info) {
  if (!sv || !info) return NS_EINVAL;
  auto it = sv->all.find(id);
  if (it == sv->all.end()) return NS_EINVAL;
  const Request *r = it->second.get();
  info->state = r->state;
  info->status = r->status;
  info->steps = r->steps;
  info->bytes = r->bytes;
  info->t_submit = r->t_submit;
  info->t_admit = r->t_admit;
  info->t_finish = r->t_finish;
  info->t_sim = r->t_sim;
  info->n_nodes = 1;
  for (int d = 0; d < r->mesh.dim; ++d) info->n_nodes *= r->mesh.n[d];
  return NS_OK;
}

int ns_server_result(ns_server *sv, int64_t id, double *U) {
  if (!sv || !U) return NS_EINVAL;
  auto it = sv->all.find(id);
  if (it == sv->all.end()) return NS_EINVAL;
  Request *r = it->second.get();
  if (r->state != FINISHED) return NS_ESTATE;
  std::copy(r->out.begin(), r->out.end(), U);
  const int status = r->status;
  sv->all.erase(it);
  return status;
}

int ns_server_stats_get(const ns_server *sv, ns_server_stats *out) {
  if (!sv || !out) return NS_EINVAL;
  *out = sv->st;
  out->queued = (int64_t)sv->queue.size();
  out->running = 0;
  for (const Unit *u : sv->running) out->running += (int64_t)u->mem.size();
  out->bytes_in_use = sv->used;
  return NS_OK;
}

const char *ns_server_error(const ns_server *sv, int64_t id) {
  if (!sv) return "null server";
  auto it = sv->all.find(id);
  if (it == sv->all.end()) return sv->err.c_str();
  return it->second->error.c_str();
}

}  // extern "C"
