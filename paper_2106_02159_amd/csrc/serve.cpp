// serve.cpp -- continuous batching of independent simulations on one GPU.
//
// Each request is a uniform-mesh Euler problem (mesh, initial state, number
// of SSPRK(3,3) steps with the CFL time step).  Requests wait in a FIFO queue
// and are admitted, in order, whenever their device footprint fits in the
// server's memory budget beside the running ones (and the number of running
// requests is below the limit).  An admitted request gets its own solver on
// its own HIP stream.  Its steps are enqueued in small chunks, at most
// `depth` chunks in flight, without host synchronization: every progress
// call tops up each running request by one chunk (round robin), so the
// running requests advance together -- a small request is never queued
// behind the whole run of a large one on a hardware queue -- and their
// kernels overlap on the device.  ns_server_progress also collects finished
// requests (copying their states to host memory and freeing their device
// memory, which lets the next queued requests in) and admits new ones; it
// never blocks on the device.  Each request's result depends only on its own
// input: the kernels are deterministic and requests share no device data.
#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/ns.h"

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
  int enqueued = 0;  // steps enqueued so far
  int state = QUEUED;
  ns_graph *g = nullptr;
  ns_solver *s = nullptr;
  int64_t bytes = 0;
  double t_submit = 0, t_admit = 0, t_finish = 0;
  double t_sim = 0.0;
  int status = NS_OK;
  std::string error;
  std::vector<double> out;
};

}  // namespace

struct ns_server {
  ns_server_params prm{};
  std::deque<Request *> queue;
  std::vector<Request *> running;
  std::map<int64_t, std::unique_ptr<Request>> all;
  int64_t used = 0;
  int64_t next_id = 1;
  ns_server_stats st{};
  std::string err = "no error";
};

namespace {

void release(ns_server *sv, Request *r) {
  if (r->s) ns_solver_destroy(r->s);
  if (r->g) ns_graph_destroy(r->g);
  r->s = nullptr;
  r->g = nullptr;
  sv->used -= r->bytes;
}

// enqueue the next chunk of steps
int top_up(ns_server *sv, Request *r) {
  const int k = std::min(sv->prm.chunk, r->steps - r->enqueued);
  const int rc = ns_step_cfl_async(r->s, k);
  if (rc == NS_OK) r->enqueued += k;
  return rc;
}

// admit the request at the head of the queue: solver, state, first chunk
int admit(ns_server *sv, Request *r) {
  int rc = ns_solver_create(r->g, &sv->prm.solver, nullptr, &r->s);
  if (rc == NS_OK) rc = ns_set_state(r->s, r->u0.data(), 0);
  if (rc == NS_OK) rc = top_up(sv, r);
  if (rc != NS_OK) {
    r->error = r->s ? ns_last_error(r->s) : ns_create_error();
    return rc;
  }
  r->t_admit = now_s();
  r->state = RUNNING;
  std::vector<double>().swap(r->u0);
  return NS_OK;
}

void finish(ns_server *sv, Request *r, int status) {
  r->status = status;
  r->t_finish = now_s();
  r->state = FINISHED;
  release(sv, r);
  sv->st.finished += 1;
}

}  // namespace

extern "C" {

int ns_server_create(const ns_server_params *p, ns_server **out) {
  if (!p || !out || p->mem_bytes <= 0 || p->max_running < 1 || p->chunk < 1 ||
      p->depth < 1)
    return NS_EINVAL;
  ns_server *sv = new (std::nothrow) ns_server;
  if (!sv) return NS_ENOMEM;
  sv->prm = *p;
  *out = sv;
  return NS_OK;
}

void ns_server_destroy(ns_server *sv) {
  if (!sv) return;
  for (auto &kv : sv->all) {
    Request *r = kv.second.get();
    if (r->state == RUNNING) {
      double t;
      (void)ns_async_finish(r->s, &t);
    }
    release(sv, r);
  }
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
  r->u0.assign(U0, U0 + (size_t)(dim + 2) * N);
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
  int nf = 0;
  // top up running requests by one chunk each; collect finished ones
  for (size_t k = 0; k < sv->running.size();) {
    Request *r = sv->running[k];
    int inflight = 0;
    int rc = ns_inflight(r->s, &inflight);
    if (rc == NS_OK && r->enqueued < r->steps) {
      if (inflight < sv->prm.depth) rc = top_up(sv, r);
      if (rc == NS_OK) {
        ++k;
        continue;
      }
    }
    if (rc == NS_OK && inflight > 0) {
      ++k;
      continue;
    }
    if (rc == NS_OK) rc = ns_async_finish(r->s, &r->t_sim);
    if (rc == NS_OK || rc == NS_ECFL || rc == NS_EBOUNDS) {
      int64_t N = 0;
      int dim = 0;
      ns_graph_info(r->g, &N, nullptr, &dim, nullptr);
      r->out.resize((size_t)(dim + 2) * N);
      const int rg = ns_get_state(r->s, r->out.data(), 0);
      if (rc == NS_OK) rc = rg;
    }
    if (rc != NS_OK) r->error = ns_last_error(r->s);
    finish(sv, r, rc);
    sv->running.erase(sv->running.begin() + k);
    ++nf;
  }
  // admit queued requests, in order, while they fit
  while (!sv->queue.empty() && (int)sv->running.size() < sv->prm.max_running) {
    Request *r = sv->queue.front();
    if (sv->used + r->bytes > sv->prm.mem_bytes) break;
    sv->queue.pop_front();
    sv->used += r->bytes;
    const int rc = admit(sv, r);
    if (rc != NS_OK) {
      finish(sv, r, rc);
      ++nf;
      continue;
    }
    sv->running.push_back(r);
    sv->st.peak_running = std::max<int64_t>(sv->st.peak_running, (int64_t)sv->running.size());
    sv->st.peak_bytes = std::max(sv->st.peak_bytes, sv->used);
  }
  if (n_finished) *n_finished = nf;
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
  out->running = (int64_t)sv->running.size();
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
