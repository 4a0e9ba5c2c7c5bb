// ns_api.hip -- implementation of the C ABI declared in include/ns.h.
//
// Host side: graph construction (closed form, graph.cpp), device allocation,
// state transfer and validation, the SSPRK(3,3) driver (Sec. 4.1, eq.
// SPPRK33) with a device-resident time step, and per-kernel event timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/ns.h"
#include "element.hpp"
#include "graph.hpp"
#include "hyp_kernels.hpp"
#include "device.hpp"
#include "par_kernels.hpp"

struct ns_graph {
  ns::MeshGraph mg;
};

namespace {

thread_local std::string g_create_error = "no error";

struct Profiler {
  bool on = false;
  hipStream_t stream = nullptr;
  std::vector<std::string> names;
  std::map<std::string, int> ids;
  std::vector<int64_t> launches;
  std::vector<double> total_ms;
  struct Pending { int id; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pool;
  int cur_id = -1;
  hipEvent_t cur_a = nullptr, cur_b = nullptr;

  void reset() {
    flush();
    names.clear(); ids.clear(); launches.clear(); total_ms.clear();
  }
  void flush() {
    for (auto &p : pending) {
      (void)hipEventSynchronize(p.b);
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess && p.id >= 0) {
        total_ms[p.id] += ms;
        launches[p.id] += 1;
      }
      pool.emplace_back(p.a, p.b);
    }
    pending.clear();
  }
  void destroy() {
    flush();
    for (auto &e : pool) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    pool.clear();
  }
  static void before(void *self, const char *name) {
    Profiler *P = static_cast<Profiler *>(self);
    if (!P->on) return;
    auto it = P->ids.find(name);
    int id;
    if (it == P->ids.end()) {
      id = (int)P->names.size();
      P->ids[name] = id;
      P->names.emplace_back(name);
      P->launches.push_back(0);
      P->total_ms.push_back(0.0);
    } else {
      id = it->second;
    }
    if (P->pool.empty()) {
      hipEvent_t a, b;
      (void)hipEventCreate(&a);
      (void)hipEventCreate(&b);
      P->pool.emplace_back(a, b);
    }
    P->cur_a = P->pool.back().first;
    P->cur_b = P->pool.back().second;
    P->pool.pop_back();
    P->cur_id = id;
    (void)hipEventRecord(P->cur_a, P->stream);
  }
  static void after(void *self) {
    Profiler *P = static_cast<Profiler *>(self);
    if (!P->on) return;
    (void)hipEventRecord(P->cur_b, P->stream);
    P->pending.push_back({P->cur_id, P->cur_a, P->cur_b});
    if (P->pending.size() > 8192) P->flush();
  }
};

}  // namespace

struct ns_solver {
  ns::MeshGraph mg;
  ns_params prm{};
  ns::Gas gas{};
  int dim = 0, nc = 0;
  int64_t N = 0;
  int64_t Np = 0;  // N rounded up to the 64-row slices of the edge arrays
  int W = 0;
  // a pack of several meshes (ns_pack): members, the first row of each (a
  // multiple of kBlock; the rows up to the next member are isolated padding
  // nodes), their node counts and slip-list ranges; seg and mblk on the
  // device (see StageArgsT)
  int nmem = 1;
  bool pack = false;
  std::vector<ns::MeshGraph> mgs;
  std::vector<int64_t> mbase, mslip;
  std::vector<char> mset;
  int32_t *seg = nullptr, *mblk = nullptr;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;  // the HIP device current at creation
  std::vector<void *> allocs;
  int64_t bytes = 0;
  // graph on the device: one box geometry per mesh (the kernels derive the
  // column indices, m_ij and c_ij from it) and the per-node data
  ns::BoxGeom *geo = nullptr;
  // mixed precision: FP32 storage of alpha, d_ij, F^H and the limiter
  // coefficients (the FP64 arrays stay null)
  bool mixed = false;
  // NS_PREC_MIXED_FP32: the graph viscosity sweep evaluates in FP32, U^L is
  // re-checked in FP64 every stage; redo_fp64 while a synchronous step is
  // redone in FP64 arithmetic after a failed re-check (fp64_redo counts them)
  bool fp32_eval = false, redo_fp64 = false;
  int fp64_redo = 0;
  float *alphaf = nullptr, *df = nullptr, *FHf = nullptr, *lt1f = nullptr,
        *lt2f = nullptr;
  double *mi = nullptr, *rmi = nullptr, *lfac = nullptr, *crm = nullptr, *rrel = nullptr;
  uint8_t *wall = nullptr;
  int nslip = 0;
  int32_t *slip_idx = nullptr;
  double *slip_n = nullptr;
  // non-reflecting nodes (ns_set_boundary): index, unit normal (dim x nnr),
  // far-field state (nc x nnr), method
  int nnr = 0, nr_method = 0;
  // multigrid preconditioner of the parabolic CG (NS_PC_GMG): levels on the
  // device (their buffers), z vector of the CG
  std::vector<ns::MGLevel> mgl;
  double *mg_z = nullptr;
  // adaptive CFL step in progress: CFL number of its time step, U^L checks
  bool adaptive = false;
  double cfl_now = 0.0;
  int32_t *nr_idx = nullptr;
  double *nr_n = nullptr, *nr_ud = nullptr;
  // state and scratch
  double *S[3] = {nullptr, nullptr, nullptr};
  int cur = 0;
  bool has_state = false;
  double *aux = nullptr, *alpha = nullptr, *d = nullptr, *UL = nullptr,
         *FH = nullptr, *bnds = nullptr, *lt1 = nullptr, *lt2 = nullptr,
         *U1 = nullptr, *partial = nullptr, *tau = nullptr;
  int *flags = nullptr;
  uint32_t *q = nullptr, *qcnt = nullptr;
  uint32_t *nzm = nullptr;  // 2D: slots with a pass-2 weight, per row
  // host copies of device scalars (pageable: no pinned allocation, whose
  // release would synchronize the whole device)
  int hflags[4] = {0, 0, 0, 0};
  double *tacc = nullptr;  // device: time advanced by the asynchronous steps
  // one event per ns_step_cfl_async call still running, oldest first, and
  // a pool of finished ones for reuse
  std::deque<hipEvent_t> inflight;
  std::vector<hipEvent_t> ev_pool;
  // asynchronous CFL steps: one step (plus the time accumulation) from start
  // buffer S[b], captured as a graph on its first use and replayed after;
  // graphs_off once a capture failed (then kernels are launched one by one)
  hipGraphExec_t step_graph[3] = {nullptr, nullptr, nullptr};
  bool graphs_off = false;
  bool async_open = false;
  double htau[1] = {0.0};
  int last_out = 1;        // buffer holding the last stage output
  bool stage_ran = false;  // a stage has run: its limiter arrays hold data
  // persistent steps (ns_step_cfl_persistent): per member (nmem + 1
  // entries) the first row block, work-list slice, slip slice and slip
  // entry; list counters, completion counters, ticket, stop words; the
  // give-up word (pinned host memory, shared pool) and the launch width
  int32_t *pmblk = nullptr, *prblk = nullptr, *psblk = nullptr, *pmslip = nullptr;
  uint32_t *pcnt = nullptr, *pdone = nullptr, *pticket = nullptr;
  int *pstop = nullptr;
  int64_t rows_tot = 0, roots_tot = 0, slips_tot = 0;
  int *give_up = nullptr;
  int pgrid = 0;
  int hpstop[4] = {0, 0, 0, 0};
  // parabolic step (allocated by ns_set_viscous)
  bool viscous = false;
  ns_viscous vprm{};
  ns::ParBufs pb{};
  double *ptab = nullptr;
  double *backup = nullptr;       // nc*N: state at the start of a Strang step
  ns::CGState hcg[1] = {};
  double hscal[4] = {0, 0, 0, 0};
  ns_par_info pinfo{};
  std::string err = "no error";
  Profiler prof;

  ns::DevGraph devgraph() const {
    ns::DevGraph g;
    g.N = N; g.W = W; g.geo = geo; g.seg = seg;
    g.mi = mi; g.rmi = rmi; g.lfac = lfac; g.crm = crm; g.rrel = rrel; g.wall = wall;
    return g;
  }
  ns::DevGraphT<float> devgraph32() const {
    ns::DevGraphT<float> g;
    g.N = N; g.W = W; g.geo = geo; g.seg = seg;
    g.mi = mi; g.rmi = rmi; g.lfac = lfac; g.crm = crm; g.rrel = rrel; g.wall = wall;
    return g;
  }
  ns::StageArgsT<float> args32(int in, int out, double sa, double sb, int check) const {
    const ns::StageArgs a = args(in, out, sa, sb, check);
    ns::StageArgsT<float> b;
    b.U = a.U; b.Un = a.Un; b.out = a.out; b.aux = a.aux; b.UL = a.UL; b.bnds = a.bnds;
    b.U1 = a.U1; b.partial = a.partial; b.tau = a.tau; b.flags = a.flags;
    b.sa = a.sa; b.sb = a.sb; b.check_cfl = a.check_cfl; b.q = a.q; b.qcnt = a.qcnt;
    b.q2 = a.q2; b.drow = a.drow; b.nzm = a.nzm;
    b.seg = a.seg; b.mblk = a.mblk; b.nmem = a.nmem; b.check_low = a.check_low;
    b.alpha = alphaf; b.d = df; b.FH = FHf; b.lt1 = lt1f; b.lt2 = lt2f;
    b.fp32_eval = fp32_eval && !redo_fp64;
    return b;
  }
  ns::StageArgs args(int in, int out, double sa, double sb, int check) const {
    ns::StageArgs a;
    a.U = S[in]; a.Un = S[cur]; a.out = S[out];
    a.aux = aux; a.alpha = alpha; a.d = d; a.UL = UL; a.FH = FH; a.bnds = bnds;
    a.lt1 = lt1; a.lt2 = lt2; a.U1 = U1; a.partial = partial; a.tau = tau;
    a.flags = flags; a.sa = sa; a.sb = sb; a.check_cfl = adaptive ? 0 : check;
    a.check_low = adaptive || fp32_eval ? 1 : 0;
    a.q = q; a.qcnt = qcnt;
    a.q2 = q + (int64_t)W * Np;  // the pass-2 list and the deferred rows
    a.drow = q + 2 * (int64_t)W * Np;
    a.nzm = nzm;
    a.seg = seg; a.mblk = mblk; a.nmem = nmem;
    return a;
  }
  int fail(int code, const std::string &msg) { err = msg; return code; }
  int hipfail(hipError_t e, const char *what) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    return NS_EHIP;
  }
  // Device memory is stream-ordered (hipMallocAsync / hipFreeAsync on the
  // solver's stream): creating and destroying solvers while others run, as
  // the server does, never waits for the whole device.
  template <typename T> hipError_t alloc(T **p, size_t count) {
    void *q = nullptr;
    hipError_t e = hipMallocAsync(&q, count * sizeof(T) > 0 ? count * sizeof(T) : 1,
                                  stream);
    if (e != hipSuccess) return e;
    allocs.push_back(q);
    bytes += (int64_t)(count * sizeof(T));
    *p = static_cast<T *>(q);
    return hipSuccess;
  }
  // frees one allocation made by alloc (stream-ordered)
  template <typename T> void free_one(T *&p, size_t count) {
    if (!p) return;
    auto it = std::find(allocs.begin(), allocs.end(), (void *)p);
    if (it != allocs.end()) {
      allocs.erase(it);
      bytes -= (int64_t)(count * sizeof(T));
      (void)hipFreeAsync(p, stream);
    }
    p = nullptr;
  }
};

namespace {

// Host transfers of node vectors (states): the device holds them in the
// paired layout of node_layout.hpp, the interface component-major.  Rows
// first .. first+count-1 of the device vector dst (N rows, nc components)
// from the component-major host array src (component c of row t at
// c*ns + t): interleaved on the host, then one copy per component pair.
// Synchronises the stream (the host buffer is released on return).
hipError_t upload_nodes(double *dst, int64_t N, int nc, int64_t first, int64_t count,
                        const double *src, int64_t ns, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  std::vector<double> tmp((size_t)nc * count);
  for (int c = 0; c < nc; ++c)
    for (int64_t t = 0; t < count; ++t)
      tmp[ns::node_at(nc, c, t, count)] = src[c * ns + t];
  hipError_t e = hipSuccess;
  for (int c = 0; c < nc && e == hipSuccess; c += 2) {
    const int64_t w = c + 1 < nc ? 2 : 1;  // components in this block
    e = hipMemcpyAsync(dst + ns::node_at(nc, c, first, N), tmp.data() + c * count,
                       w * count * sizeof(double), hipMemcpyHostToDevice, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e;
}

// The reverse: rows first .. first+count-1 of the device vector src into
// the component-major host array dst (component c of row t at c*ns + t).
hipError_t download_nodes(const double *src, int64_t N, int nc, int64_t first,
                          int64_t count, double *dst, int64_t ns, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  std::vector<double> tmp((size_t)nc * count);
  hipError_t e = hipSuccess;
  for (int c = 0; c < nc && e == hipSuccess; c += 2) {
    const int64_t w = c + 1 < nc ? 2 : 1;
    e = hipMemcpyAsync(tmp.data() + c * count, src + ns::node_at(nc, c, first, N),
                       w * count * sizeof(double), hipMemcpyDeviceToHost, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return e;
  for (int c = 0; c < nc; ++c)
    for (int64_t t = 0; t < count; ++t)
      dst[c * ns + t] = tmp[ns::node_at(nc, c, t, count)];
  return hipSuccess;
}

// Give-up words of the persistent steps: one int per solver in pinned host
// memory, which the host writes and the kernel polls across the bus.  One
// block of slots is allocated per process and kept until it ends (releasing
// pinned memory would wait for the whole device); solvers take a slot on
// their first persistent step and return it when destroyed.
constexpr int kGiveUpSlots = 1024;
std::mutex g_give_up_mu;
int *g_give_up_host = nullptr;  // the slots as the host writes them
int *g_give_up_dev = nullptr;   // the same slots as kernels address them
std::vector<int> g_give_up_free;

int *take_give_up_word() {
  std::lock_guard<std::mutex> lk(g_give_up_mu);
  if (!g_give_up_host) {
    void *p = nullptr;
    if (hipHostMalloc(&p, kGiveUpSlots * sizeof(int),
                      hipHostMallocMapped | hipHostMallocPortable | hipHostMallocCoherent) !=
        hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    void *d = nullptr;
    if (hipHostGetDevicePointer(&d, p, 0) != hipSuccess) {
      (void)hipGetLastError();
      (void)hipHostFree(p);
      return nullptr;
    }
    g_give_up_host = static_cast<int *>(p);
    g_give_up_dev = static_cast<int *>(d);
    for (int k = kGiveUpSlots - 1; k >= 0; --k) g_give_up_free.push_back(k);
  }
  if (g_give_up_free.empty()) return nullptr;
  const int k = g_give_up_free.back();
  g_give_up_free.pop_back();
  __atomic_store_n(g_give_up_host + k, 0, __ATOMIC_SEQ_CST);
  return g_give_up_host + k;
}

// The device address of a host slot.
const int *give_up_device(const int *w) {
  return w ? g_give_up_dev + (w - g_give_up_host) : nullptr;
}

void return_give_up_word(int *w) {
  if (!w) return;
  std::lock_guard<std::mutex> lk(g_give_up_mu);
  g_give_up_free.push_back((int)(w - g_give_up_host));
}

void release(ns_solver *s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  return_give_up_word(s->give_up);
  s->give_up = nullptr;
  s->prof.destroy();
  for (void *p : s->allocs) (void)hipFreeAsync(p, s->stream);
  s->allocs.clear();

  for (hipGraphExec_t &g : s->step_graph) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
  for (hipEvent_t ev : s->inflight) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : s->ev_pool) (void)hipEventDestroy(ev);
  s->inflight.clear();
  s->ev_pool.clear();
  if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
}

int others(int cur, int k) {  // k-th (0/1) buffer index different from cur
  int r[2], n = 0;
  for (int b = 0; b < 3; ++b)
    if (b != cur) r[n++] = b;
  return r[k];
}

int read_flags(ns_solver *s) {
  hipError_t e = hipMemcpyAsync(s->hflags, s->flags, 4 * sizeof(int),
                                hipMemcpyDeviceToHost, s->stream);
  if (e != hipSuccess) return s->hipfail(e, "flag readback");
  e = hipMemcpyAsync(s->htau, s->tau, sizeof(double), hipMemcpyDeviceToHost,
                     s->stream);
  if (e != hipSuccess) return s->hipfail(e, "dt readback");
  e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return s->hipfail(e, "stream synchronize");
  e = hipGetLastError();
  if (e != hipSuccess) return s->hipfail(e, "kernel launch");
  return NS_OK;
}

void run_stage(ns_solver *s, int in, int out, double sa, double sb, int check,
               bool auto_dt) {
  s->stage_ran = true;
  if (s->mixed)
    ns::launch_stage(s->dim, s->gas, s->devgraph32(), s->args32(in, out, sa, sb, check),
                     s->prm.indicator, s->prm.limiter, s->prm.passes, auto_dt,
                     s->adaptive ? s->cfl_now : s->prm.cfl, s->stream, &Profiler::before,
                     &Profiler::after,
                     &s->prof);
  else
    ns::launch_stage(s->dim, s->gas, s->devgraph(), s->args(in, out, sa, sb, check),
                     s->prm.indicator, s->prm.limiter, s->prm.passes, auto_dt,
                     s->adaptive ? s->cfl_now : s->prm.cfl, s->stream, &Profiler::before,
                     &Profiler::after,
                     &s->prof);
}

// Boundary post-processing of a stage result (Sec. 4.3): the non-reflecting
// nodes first, then the slip projection (a node in both sets keeps no normal
// momentum through its slip faces).
void run_slip(ns_solver *s, int buf) {
  if (s->nnr > 0) {
    Profiler::before(&s->prof, "nonreflecting");
    ns::launch_nonreflecting(s->dim, s->gas, s->nr_method, s->nnr, s->nr_idx, s->nr_n,
                             s->nr_ud, s->N, s->S[buf], s->flags, s->stream);
    Profiler::after(&s->prof);
  }
  Profiler::before(&s->prof, "slip");
  ns::launch_slip(s->dim, s->N, s->nslip, s->slip_idx, s->slip_n, s->S[buf],
                  s->stream);
  Profiler::after(&s->prof);
}

// One SSPRK(3,3) step; dt either given (auto_dt false) or computed in stage 1.
// Enqueues one SSPRK(3,3) step from S[cur] into S[o1] (eq. SPPRK33; dt given
// or computed in the first stage); the status flags are not cleared.
int ssprk3_enqueue(ns_solver *s, double dt, bool auto_dt) {
  const int o1 = others(s->cur, 0), o2 = others(s->cur, 1);
  if (!auto_dt) ns::launch_set_scalar(s->tau, dt, s->stream);
  // w1 = E(u^n)
  run_stage(s, s->cur, o1, 0.0, 1.0, auto_dt ? 0 : 1, auto_dt);
  run_slip(s, o1);
  // w2 = 3/4 u^n + 1/4 E(w1)
  run_stage(s, o1, o2, 0.75, 0.25, 1, false);
  run_slip(s, o2);
  // u^{n+1} = 1/3 u^n + 2/3 E(w2)
  run_stage(s, o2, o1, 1.0 / 3.0, 2.0 / 3.0, 1, false);
  run_slip(s, o1);
  s->last_out = o1;
  return o1;
}

int ssprk3(ns_solver *s, double dt, bool auto_dt, double *dt_out) {
  if (!s->has_state) return s->fail(NS_ESTATE, "no state set");
  ns::launch_clear_flags(s->flags, s->stream);
  int o1 = ssprk3_enqueue(s, dt, auto_dt);
  int rc = read_flags(s);
  if (rc != NS_OK) return rc;
  if (s->fp32_eval && (s->hflags[3] || s->hflags[1])) {
    // the FP64 re-check found an inadmissible U^L (or stage result) in some
    // row: the step again from the unchanged S[cur], in FP64 arithmetic
    ++s->fp64_redo;
    s->redo_fp64 = true;
    ns::launch_clear_flags(s->flags, s->stream);
    o1 = ssprk3_enqueue(s, dt, auto_dt);
    s->redo_fp64 = false;
    rc = read_flags(s);
    if (rc != NS_OK) return rc;
  }
  if (dt_out) *dt_out = *s->htau;
  if (s->hflags[0]) {
    char buf[160];
    snprintf(buf, sizeof buf, "dt = %.17g exceeds the stage CFL limit", *s->htau);
    return s->fail(NS_ECFL, buf);
  }
  if (s->hflags[1]) return s->fail(NS_EBOUNDS, "a stage produced an inadmissible state");
  s->cur = o1;
  return NS_OK;
}

ns::ParGrid par_grid(const ns_solver *s) {
  ns::ParGrid g;
  g.N = s->N;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = s->mg.n[d];
    g.per[d] = d < s->dim ? s->mg.periodic[d] : 0;
  }
  return g;
}

// Conjugate gradients on the device: start, then batches of iterations
// with one status readback per batch.
int run_cg(ns_solver *s, int ncomp, double cdt, const char *label, int *iters) {
  const ns::ParGrid g = par_grid(s);
  const bool mg = s->vprm.precond == NS_PC_GMG && !s->mgl.empty();
  const int nlev = (int)s->mgl.size(), deg = 3, cdeg = 12;
  Profiler::before(&s->prof, label);
  if (mg) {
    ns::mg_setup(s->dim, ncomp, s->mgl.data(), nlev, s->pb.rm, cdt, s->stream);
    ns::par_cg_start_mg(s->dim, ncomp, g, s->pb, s->mg_z, cdt, s->vprm.cg_rtol,
                        s->vprm.cg_maxit, s->mgl.data(), nlev, deg, cdeg, s->stream);
  } else {
    ns::par_cg_start(s->dim, ncomp, g, s->pb, cdt, s->vprm.cg_rtol, s->vprm.cg_maxit,
                     s->stream);
  }
  Profiler::after(&s->prof);
  int launched = 0, batch = 2;
  for (;;) {
    Profiler::before(&s->prof, label);
    if (mg)
      ns::par_cg_iterate_mg(s->dim, ncomp, g, s->pb, s->mg_z, cdt, batch, s->mgl.data(), nlev,
                            deg, cdeg, s->stream);
    else
      ns::par_cg_iterate(s->dim, ncomp, g, s->pb, cdt, batch, s->stream);
    Profiler::after(&s->prof);
    launched += batch;
    hipError_t e = hipMemcpyAsync(s->hcg, s->pb.cg, sizeof(ns::CGState),
                                  hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return s->hipfail(e, "parabolic CG");
    if (s->hcg->done || launched > s->vprm.cg_maxit) break;
    batch = std::min(2 * batch, 16);
  }
  *iters = s->hcg->it;
  const bool ok = s->hcg->bb == 0.0 || s->hcg->rr <= s->hcg->rtol2 * s->hcg->bb;
  if (!ok) {
    char buf[160];
    snprintf(buf, sizeof buf, "%s: CG did not converge in %d iterations (|r|/|b| = %.3g)",
             label, s->hcg->it, std::sqrt(s->hcg->rr / s->hcg->bb));
    return s->fail(NS_ECG, buf);
  }
  return NS_OK;
}

// Parabolic step of size dt from S[in] into S[out] (the parabolic-step
// algorithm of the appendix); S[in] is not modified.
int par_step(ns_solver *s, double dt, int in, int out) {
  const ns::ParGrid g = par_grid(s);
  const ns::ParBufs &B = s->pb;
  const double *U = s->S[in];
  double *O = s->S[out];
  const int dim = s->dim;
  s->pinfo = ns_par_info{};
  ns::launch_clear_flags(s->flags, s->stream);
  Profiler::before(&s->prof, "par_prep");
  ns::par_prep(dim, g, B, U, dt, s->stream);
  Profiler::after(&s->prof);
  // Step 1: velocity (Crank-Nicolson, no-slip rows eliminated)
  int rc = run_cg(s, dim, 0.5 * dt, "cg_velocity", &s->pinfo.it_v);
  if (rc != NS_OK) return rc;
  Profiler::before(&s->prof, "par_velocity");
  ns::par_velocity_done(dim, g, B, U, O, s->vprm.mu, s->vprm.lambda, s->stream);
  Profiler::after(&s->prof);
  // Step 2: internal energy (Crank-Nicolson, source dt/2 m K)
  Profiler::before(&s->prof, "par_energy_setup");
  ns::par_energy_setup(dim, g, B, 0.5 * dt, 0.5 * dt, s->stream);
  Profiler::after(&s->prof);
  rc = run_cg(s, 1, 0.5 * dt, "cg_energy", &s->pinfo.it_e);
  if (rc != NS_OK) return rc;
  Profiler::before(&s->prof, "par_energy_high");
  ns::par_energy_high(dim, g, B, s->stream);
  Profiler::after(&s->prof);
  hipError_t e = hipMemcpyAsync(s->hscal, B.scal, sizeof(double), hipMemcpyDeviceToHost,
                                s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return s->hipfail(e, "parabolic step");
  s->pinfo.min_eH = s->hscal[0];
  // Step 3: limiting when the internal energy is not positive (or forced)
  if (s->vprm.fct == NS_FCT_ALWAYS || !(s->hscal[0] > 0.0)) {
    s->pinfo.fct = 1;
    Profiler::before(&s->prof, "par_energy_setup");
    ns::par_energy_setup(dim, g, B, dt, dt, s->stream);
    Profiler::after(&s->prof);
    rc = run_cg(s, 1, dt, "cg_low", &s->pinfo.it_l);
    if (rc != NS_OK) return rc;
    Profiler::before(&s->prof, "par_fct");
    ns::par_fct(dim, g, B, dt, s->stream);
    Profiler::after(&s->prof);
  }
  Profiler::before(&s->prof, "par_finish");
  ns::par_finish(dim, g, B, U, B.eH, O, s->stream);
  Profiler::after(&s->prof);
  rc = read_flags(s);
  if (rc != NS_OK) return rc;
  if (s->hflags[1])
    return s->fail(NS_EBOUNDS, "the parabolic step produced a non-positive internal energy");
  return NS_OK;
}

int strang(ns_solver *s, double tau, bool auto_dt, double *tau_out) {
  if (!s->has_state) return s->fail(NS_ESTATE, "no state set");
  if (!s->viscous) return s->fail(NS_ESTATE, "ns_set_viscous has not been called");
  const size_t bytes = (size_t)s->nc * s->N * sizeof(double);
  hipError_t e = hipMemcpyAsync(s->backup, s->S[s->cur], bytes, hipMemcpyDeviceToDevice,
                                s->stream);
  if (e != hipSuccess) return s->hipfail(e, "state backup");
  double t = tau;
  int rc = ssprk3(s, tau, auto_dt, &t);
  if (rc != NS_OK) return rc;  // the hyperbolic step left the state unchanged
  if (tau_out) *tau_out = t;
  const int o = others(s->cur, 0);
  rc = par_step(s, 2.0 * t, s->cur, o);
  if (rc == NS_OK) {
    s->cur = o;
    rc = ssprk3(s, t, false, nullptr);
  }
  if (rc != NS_OK) {
    e = hipMemcpyAsync(s->S[s->cur], s->backup, bytes, hipMemcpyDeviceToDevice,
                       s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return s->hipfail(e, "state restore");
  }
  return rc;
}

}  // namespace

extern "C" {

const char *ns_strerror(int code) {
  switch (code) {
    case NS_OK: return "ok";
    case NS_EINVAL: return "invalid argument";
    case NS_ENOMEM: return "out of memory";
    case NS_EHIP: return "HIP runtime error";
    case NS_ENOTADMISSIBLE: return "state not admissible";
    case NS_ECFL: return "time step above the CFL limit";
    case NS_EBOUNDS: return "inadmissible state produced";
    case NS_ESTATE: return "no state set";
    case NS_ECG: return "CG did not converge";
    default: return "unknown status";
  }
}

const char *ns_create_error(void) { return g_create_error.c_str(); }

int ns_graph_create(const ns_mesh_desc *mesh, ns_graph **out) {
  if (!mesh || !out) { g_create_error = "null argument"; return NS_EINVAL; }
  ns_graph *g = new (std::nothrow) ns_graph;
  if (!g) { g_create_error = "host allocation"; return NS_ENOMEM; }
  const char *why = "";
  if (ns::build_mesh_graph(mesh->dim, mesh->n, mesh->lo, mesh->hi,
                           mesh->periodic, &g->mg, &why) != 0) {
    g_create_error = why;
    delete g;
    return NS_EINVAL;
  }
  *out = g;
  return NS_OK;
}

void ns_graph_destroy(ns_graph *g) { delete g; }

int ns_graph_info(const ns_graph *g, int64_t *n_nodes, int64_t *nnz, int *dim,
                  int *width) {
  if (!g) return NS_EINVAL;
  if (n_nodes) *n_nodes = g->mg.N;
  if (nnz) *nnz = g->mg.nnz;
  if (dim) *dim = g->mg.dim;
  if (width) *width = g->mg.W;
  return NS_OK;
}

int ns_graph_export(const ns_graph *g, int32_t *col, double *mij, double *cij,
                    double *mi, double *bnd) {
  if (!g) return NS_EINVAL;
  const ns::MeshGraph &m = g->mg;
  const int64_t N = m.N;
  for (int k = 0; k < m.W; ++k) {
    double *cp[3] = {nullptr, nullptr, nullptr};
    if (cij)
      for (int e = 0; e < m.dim; ++e) cp[e] = cij + ((int64_t)e * m.W + k) * N;
    m.fill_slot(k, col ? col + (int64_t)k * N : nullptr, nullptr,
                mij ? mij + (int64_t)k * N : nullptr, cij ? cp : nullptr);
  }
  if (mi || bnd) m.fill_nodes(mi, bnd, nullptr);
  return NS_OK;
}

extern "C++" {
namespace {
// Geometry of a box mesh placed at row `base`: sizes, periodic flags and
// the graph builder's own 1D mass factors.
ns::BoxGeom box_geom(const ns::MeshGraph &m, int64_t base) {
  ns::BoxGeom b{};
  b.base = (int32_t)base;
  b.nn = (int32_t)m.N;
  b.per = 0;
  for (int d = 0; d < 3; ++d) {
    b.n[d] = d < m.dim ? (int32_t)m.n[d] : 1;
    if (d < m.dim && m.periodic[d]) b.per |= 1 << d;
    b.m_inner[d] = b.m_end[d] = b.m_off[d] = 1.0;
    if (d < m.dim) m.m1_values(d, &b.m_inner[d], &b.m_end[d], &b.m_off[d]);
  }
  return b;
}

template <int DIM>
void stencil_rows(const ns::BoxGeom &geo, int64_t rows, int32_t *col, double *mij,
                  double *cij) {
  constexpr int W = DIM == 2 ? 9 : 27;
  for (int64_t r = 0; r < rows; ++r) {
    const ns::BoxNbr<DIM> nb(&geo, geo.base + r);
    for (int k = 0; k < W; ++k) {
      if (col) col[k * rows + r] = nb[k];
      if (mij) mij[k * rows + r] = nb.mass(k);
      if (cij) {
        double c[3];
        nb.grad(k, c);
        for (int e = 0; e < DIM; ++e) cij[((int64_t)e * W + k) * rows + r] = c[e];
      }
    }
  }
}
}  // namespace
}  // extern "C++"

int ns_graph_stencil(const ns_graph *g, int64_t base, int64_t rows, int32_t *col,
                     double *mij, double *cij) {
  if (!g) return NS_EINVAL;
  const ns::MeshGraph &m = g->mg;
  if (rows < m.N || base < 0 || base + rows > INT32_MAX) return NS_EINVAL;
  const ns::BoxGeom geo = box_geom(m, base);
  if (m.dim == 2) stencil_rows<2>(geo, rows, col, mij, cij);
  else stencil_rows<3>(geo, rows, col, mij, cij);
  return NS_OK;
}

extern "C++" {
namespace ns {
int current_device() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return dev;
}
void use_device(int device) {
  if (hipSetDevice(device) != hipSuccess) (void)hipGetLastError();
}
}  // namespace ns
}  // extern "C++"

namespace {
// Rows of a solver: one mesh (N nodes, edge slices padded to 64 rows) or a
// pack (each member's rows start at a workgroup boundary).
struct Layout {
  std::vector<const ns::MeshGraph *> mgs;
  std::vector<int64_t> base;
  int64_t N = 0, Np = 0;
  bool pack = false;
};

Layout one_mesh(const ns::MeshGraph &m) {
  Layout L;
  L.mgs = {&m};
  L.base = {0};
  L.N = m.N;
  L.Np = (m.N + 63) / 64 * 64;
  return L;
}

Layout packed(const ns::MeshGraph *const *m, int count) {
  Layout L;
  L.pack = true;
  for (int r = 0; r < count; ++r) {
    L.mgs.push_back(m[r]);
    L.base.push_back(L.N);
    L.N += (m[r]->N + ns::kBlock - 1) / ns::kBlock * ns::kBlock;
  }
  L.Np = L.N;
  return L;
}

int64_t slip_count(const ns::MeshGraph &m) {
  int64_t interior = 1;
  for (int d = 0; d < m.dim; ++d)
    interior *= m.periodic[d] ? m.n[d] : std::max<int64_t>(m.n[d] - 2, 0);
  return m.N - interior;
}

int64_t footprint(const Layout &Lt, const ns_params *p) {
  const ns::MeshGraph &m = *Lt.mgs[0];
  const int64_t N = Lt.N, Np = Lt.Np, W = m.W, dim = m.dim, nc = dim + 2;
  const int64_t L = p->precision != NS_PREC_FP64 ? 4 : 8;
  const int64_t nblocks = (N + ns::kBlock - 1) / ns::kBlock;
  const int64_t nm = (int64_t)Lt.mgs.size();
  int64_t nslip = 0;
  for (const ns::MeshGraph *g : Lt.mgs) nslip += slip_count(*g);
  int64_t b = 0;
  b += nm * (int64_t)sizeof(ns::BoxGeom);             // box geometry
  b += 5 * N * 8 + N;                                // m_i, 1/m_i, lfac, lfac/m_i, r_i, wall
  b += 3 * nc * N * 8 + (dim + 5) * N * 8;           // states, aux
  b += N * L + W * Np * L + nc * N * 8 + (nc + (dim == 3)) * N * L;  // alpha, d, U^L, F^H
  b += 3 * N * 8 + 2 * W * Np * L + nc * N * 8;      // bounds, l~ (2), U^(1)
  b += N * 4;                                        // pass-2 weight mask
  b += nblocks * 8 + nm * (8 + 4 * 4 + 8);           // partial, tau, flags, time
  b += (2 * W * Np + Np) * 4 + 4 * 4;                // root work lists, deferred rows
  b += nslip * 4 + dim * nslip * 8;                  // slip list
  if (Lt.pack) b += nblocks * 4 + (nm + 1) * 4;      // member of each workgroup
  b += 4 * (nm + 1) * 4 + 3 * nm * 4 + 4 + 4 * 4;    // persistent-step tables
  return b;
}
}  // namespace

int ns_solver_footprint(const ns_graph *g, const ns_params *p, int64_t *bytes) {
  if (!g || !p || !bytes) return NS_EINVAL;
  *bytes = footprint(one_mesh(g->mg), p);
  return NS_OK;
}

namespace {
// Keep memory freed by hipFreeAsync in the device's default pool instead of
// returning it to the GPU kernel driver, so that solvers created after
// others were destroyed reuse it without new allocations from the system.
// (solvers may be created from several threads: once per device)
void keep_pool_memory() {
  static std::mutex mu;
  static std::vector<int> done;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  std::lock_guard<std::mutex> lock(mu);
  if (std::find(done.begin(), done.end(), dev) != done.end()) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  (void)hipGetLastError();
  done.push_back(dev);
}
}  // namespace

namespace {
int create_impl(const Layout &Lt, const ns_params *p, void *stream, ns_solver **out) {
  if (!(p->gamma > 1.0 && p->gamma <= 5.0 / 3.0 + 1e-12) ||
      !(p->cfl > 0.0 && p->cfl <= 1.0) || p->indicator < 0 || p->indicator > 2 ||
      p->limiter < 0 || p->limiter > 2 || (p->passes != 1 && p->passes != 2) ||
      !(p->relax >= 0.0) || !std::isfinite(p->relax) ||
      (p->precision != NS_PREC_FP64 && p->precision != NS_PREC_MIXED &&
       p->precision != NS_PREC_MIXED_FP32)) {
    g_create_error = "invalid parameters (need 1 < gamma <= 5/3, 0 < cfl <= 1, "
                     "indicator/limiter in range, passes 1 or 2, relax >= 0, "
                     "precision NS_PREC_FP64, NS_PREC_MIXED or NS_PREC_MIXED_FP32)";
    return NS_EINVAL;
  }
  const ns::MeshGraph &m0 = *Lt.mgs[0];
  if ((int64_t)m0.W * Lt.Np > (int64_t)UINT32_MAX) {
    g_create_error = "mesh too large: edge indices must fit in 32 bits";
    return NS_EINVAL;
  }
  ns_solver *s = new (std::nothrow) ns_solver;
  if (!s) { g_create_error = "host allocation"; return NS_ENOMEM; }
  keep_pool_memory();
  s->mg = m0;
  s->prm = *p;
  s->mixed = p->precision != NS_PREC_FP64;
  s->fp32_eval = p->precision == NS_PREC_MIXED_FP32;
  s->dim = m0.dim;
  s->nc = s->dim + 2;
  s->N = Lt.N;
  s->Np = Lt.Np;
  s->W = m0.W;
  s->pack = Lt.pack;
  s->nmem = (int)Lt.mgs.size();
  for (const ns::MeshGraph *g : Lt.mgs) s->mgs.push_back(*g);
  s->mbase = Lt.base;
  s->mset.assign(s->nmem, 0);
  const double gm = p->gamma;
  s->gas.gamma = gm;
  s->gas.gm1 = gm - 1.0;
  s->gas.ex = (gm - 1.0) / (2.0 * gm);
  s->gas.inv_ex = 2.0 * gm / (gm - 1.0);
  s->gas.cg = (gm + 1.0) / (2.0 * gm);
  s->gas.lgm1 = std::log(gm - 1.0);
  s->gas.seven = gm == 1.4 ? 1 : 0;

  auto bail = [&](int code, const std::string &msg) {
    g_create_error = msg;
    release(s);
    delete s;
    return code;
  };
  hipError_t e;
  if (stream) {
    s->stream = static_cast<hipStream_t>(stream);
  } else {
    e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(NS_EHIP, "hipStreamCreate failed");
    s->own_stream = true;
  }
  s->prof.stream = s->stream;
  s->device = ns::current_device();
  const int64_t N = s->N, W = s->W, nc = s->nc, dim = s->dim, Np = s->Np;
  const int64_t nblocks = (N + ns::kBlock - 1) / ns::kBlock;
#define NS_ALLOC(ptr, count)                                                \
  do {                                                                      \
    e = s->alloc(&(ptr), (size_t)(count));                                  \
    if (e != hipSuccess) {                                                  \
      (void)hipGetLastError();                                              \
      return bail(NS_ENOMEM, std::string("device allocation of ") + #ptr + \
                                 " failed: " + hipGetErrorString(e));       \
    }                                                                       \
  } while (0)
  NS_ALLOC(s->geo, s->nmem);
  NS_ALLOC(s->mi, N);
  NS_ALLOC(s->rmi, N);
  NS_ALLOC(s->lfac, N);
  NS_ALLOC(s->crm, N);
  NS_ALLOC(s->rrel, N);
  NS_ALLOC(s->wall, N);
  for (int b = 0; b < 3; ++b) NS_ALLOC(s->S[b], nc * N);
  NS_ALLOC(s->aux, (dim + 5) * N);
  if (s->mixed) {
    NS_ALLOC(s->alphaf, N);
    NS_ALLOC(s->df, W * Np);
    NS_ALLOC(s->FHf, (nc + (dim == 3)) * N);  // 3D: alpha beside F^H
    NS_ALLOC(s->lt1f, W * Np);
    NS_ALLOC(s->lt2f, W * Np);
  } else {
    NS_ALLOC(s->alpha, N);
    NS_ALLOC(s->d, W * Np);
    NS_ALLOC(s->FH, (nc + (dim == 3)) * N);
    NS_ALLOC(s->lt1, W * Np);
    NS_ALLOC(s->lt2, W * Np);
  }
  NS_ALLOC(s->UL, nc * N);
  NS_ALLOC(s->bnds, 3 * N);
  NS_ALLOC(s->U1, nc * N);
  NS_ALLOC(s->nzm, N);
  NS_ALLOC(s->partial, nblocks);
  NS_ALLOC(s->tau, s->nmem);
  NS_ALLOC(s->flags, 4 * s->nmem);
  NS_ALLOC(s->tacc, s->nmem);
  if (s->pack) {
    NS_ALLOC(s->seg, nblocks);
    NS_ALLOC(s->mblk, s->nmem + 1);
  }
  // limiter root work list, large enough for every edge
  NS_ALLOC(s->q, 2 * W * Np + Np);  // pass-1 and pass-2 lists, deferred rows
  NS_ALLOC(s->qcnt, 4);
  NS_ALLOC(s->pmblk, s->nmem + 1);
  NS_ALLOC(s->prblk, s->nmem + 1);
  NS_ALLOC(s->psblk, s->nmem + 1);
  NS_ALLOC(s->pmslip, s->nmem + 1);
  NS_ALLOC(s->pcnt, 2 * s->nmem);
  NS_ALLOC(s->pdone, s->nmem);
  NS_ALLOC(s->pticket, 1);
  NS_ALLOC(s->pstop, 4);
  // the uploads below are synchronous copies: the stream-ordered allocations
  // must have completed
  e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return bail(NS_EHIP, "stream synchronize");

  // --- the graph: one box geometry per mesh (the kernels derive the column
  // indices, m_ij and c_ij of every entry from it); |I(i)| per row from the
  // graph builder's columns
  {
    const int nm = s->nmem;
    auto mend = [&](int r) { return r + 1 < nm ? Lt.base[r + 1] : N; };
    std::vector<int> cnt(N, 0);
    std::vector<ns::BoxGeom> geo(nm);
    for (int r = 0; r < nm; ++r) {
      const ns::MeshGraph &m = *Lt.mgs[r];
      const int64_t b0 = Lt.base[r], Nr = m.N;
      geo[r] = box_geom(m, b0);
      std::vector<int32_t> col(Nr);
      for (int k = 0; k < W; ++k) {
        m.fill_slot(k, col.data(), nullptr, nullptr, nullptr);
        for (int64_t i = 0; i < Nr; ++i) cnt[b0 + i] += col[i] >= 0;
      }
      // padding rows of a pack: isolated nodes (only the diagonal entry)
      for (int64_t i = b0 + Nr; i < mend(r); ++i) cnt[i] = 1;
    }
    e = hipMemcpyAsync(s->geo, geo.data(), nm * sizeof(ns::BoxGeom), hipMemcpyHostToDevice,
                       s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return bail(NS_EHIP, "graph upload failed");
    // node data; padding rows: m_i = 1, |I(i)| - 1 := 1, r_i = 0, no wall
    std::vector<double> mi(N, 1.0), rmi(N, 1.0), lfac(N, 1.0), crm(N, 1.0), rrel(N, 0.0);
    std::vector<uint8_t> wall(N, 0);
    std::vector<int32_t> sidx;
    std::vector<double> nrm;  // unit normals of the slip nodes, node by node
    s->mslip.assign(1, 0);
    for (int r = 0; r < nm; ++r) {
      const ns::MeshGraph &m = *Lt.mgs[r];
      const int64_t b0 = Lt.base[r], Nr = m.N;
      std::vector<double> mr(Nr), bnd((size_t)dim * Nr);
      std::vector<uint8_t> wr(Nr);
      m.fill_nodes(mr.data(), bnd.data(), wr.data());
      double vol = 0.0;
      for (int64_t i = 0; i < Nr; ++i) vol += mr[i];
      for (int64_t i = 0; i < Nr; ++i) {
        mi[b0 + i] = mr[i];
        rmi[b0 + i] = 1.0 / mr[i];
        lfac[b0 + i] = (double)(cnt[b0 + i] - 1);
        crm[b0 + i] = lfac[b0 + i] * rmi[b0 + i];
        rrel[b0 + i] = p->relax * std::pow(mr[i] / vol, 1.5 / dim);
        wall[b0 + i] = wr[i];
        if (!wr[i]) continue;
        sidx.push_back((int32_t)(b0 + i));
        double nn = 0.0, v[3];
        for (int q = 0; q < dim; ++q) { v[q] = bnd[(size_t)q * Nr + i]; nn += v[q] * v[q]; }
        nn = std::sqrt(nn);
        for (int q = 0; q < dim; ++q) nrm.push_back(v[q] / nn);
      }
      s->mslip.push_back((int64_t)sidx.size());
    }
    s->nslip = (int)sidx.size();
    std::vector<double> snrm((size_t)dim * s->nslip);
    for (int t = 0; t < s->nslip; ++t)
      for (int q = 0; q < dim; ++q) snrm[(size_t)q * s->nslip + t] = nrm[(size_t)t * dim + q];
    NS_ALLOC(s->slip_idx, s->nslip);
    NS_ALLOC(s->slip_n, dim * s->nslip);
    // member of every workgroup, workgroup offsets of the members
    std::vector<int32_t> hseg, hmblk;
    if (s->pack) {
      hseg.resize(nblocks);
      for (int r = 0; r < nm; ++r) {
        hmblk.push_back((int32_t)(Lt.base[r] / ns::kBlock));
        for (int64_t b = Lt.base[r] / ns::kBlock; b < mend(r) / ns::kBlock; ++b) hseg[b] = r;
      }
      hmblk.push_back((int32_t)nblocks);
    }
    // persistent steps: per member its row blocks, its work-list slices (one
    // per 8 row blocks: the lists hold a small fraction of the edges) and
    // its slip slices (256 entries each), as running sums
    std::vector<int32_t> pmb(nm + 1), prb(nm + 1), psb(nm + 1), pms(nm + 1);
    for (int r = 0; r <= nm; ++r) {
      pmb[r] = s->pack ? hmblk[r] : (r == 0 ? 0 : (int32_t)nblocks);
      pms[r] = (int32_t)s->mslip[r];
    }
    prb[0] = psb[0] = 0;
    for (int r = 0; r < nm; ++r) {
      const int32_t nb = pmb[r + 1] - pmb[r], ns = pms[r + 1] - pms[r];
      prb[r + 1] = prb[r] + std::max<int32_t>(1, nb / 8);
      psb[r + 1] = psb[r] + (ns + ns::kBlock - 1) / ns::kBlock;
    }
    s->rows_tot = pmb[nm];
    s->roots_tot = prb[nm];
    s->slips_tot = psb[nm];
    struct { void *dst; const void *src; size_t n; } ups[] = {
        {s->pmblk, pmb.data(), pmb.size() * sizeof(int32_t)},
        {s->prblk, prb.data(), prb.size() * sizeof(int32_t)},
        {s->psblk, psb.data(), psb.size() * sizeof(int32_t)},
        {s->pmslip, pms.data(), pms.size() * sizeof(int32_t)},
        {s->mi, mi.data(), N * sizeof(double)},
        {s->rmi, rmi.data(), N * sizeof(double)},
        {s->lfac, lfac.data(), N * sizeof(double)},
        {s->crm, crm.data(), N * sizeof(double)},
        {s->rrel, rrel.data(), N * sizeof(double)},
        {s->wall, wall.data(), (size_t)N},
        {s->slip_idx, sidx.data(), sidx.size() * sizeof(int32_t)},
        {s->slip_n, snrm.data(), snrm.size() * sizeof(double)},
        {s->seg, hseg.data(), hseg.size() * sizeof(int32_t)},
        {s->mblk, hmblk.data(), hmblk.size() * sizeof(int32_t)}};
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return bail(NS_EHIP, "stream synchronize");
    for (auto &u : ups) {
      if (u.n == 0) continue;
      e = hipMemcpyAsync(u.dst, u.src, u.n, hipMemcpyHostToDevice, s->stream);
      if (e != hipSuccess) return bail(NS_EHIP, "graph upload failed");
    }
    // the host arrays go out of scope below
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return bail(NS_EHIP, "graph upload failed");
    // padding rows of a pack hold a constant admissible state in every
    // state buffer (they have no neighbours, so the steps keep it)
    if (s->pack) {
      std::vector<double> pad((size_t)nc * ns::kBlock, 0.0);
      for (int t = 0; t < ns::kBlock; ++t) {
        pad[t] = 1.0;
        pad[(size_t)(nc - 1) * ns::kBlock + t] = 1.0;
      }
      for (int r = 0; r < nm; ++r) {
        const int64_t first = Lt.base[r] + Lt.mgs[r]->N, count = mend(r) - first;
        if (count <= 0) continue;
        for (int b = 0; b < 3 && e == hipSuccess; ++b)
          e = upload_nodes(s->S[b], N, nc, first, count, pad.data(), ns::kBlock, s->stream);
      }
      if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
      if (e != hipSuccess) return bail(NS_EHIP, "padding upload failed");
    }
  }
  // zero the scratch edge arrays once: entries never written stay zero
  for (void *z : {(void *)s->d, (void *)s->lt1, (void *)s->lt2, (void *)s->df,
                  (void *)s->lt1f, (void *)s->lt2f}) {
    if (!z) continue;
    e = hipMemsetAsync(z, 0, (size_t)W * Np * (s->mixed ? sizeof(float) : sizeof(double)),
                       s->stream);
    if (e != hipSuccess) return bail(NS_EHIP, "memset failed");
  }
  e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return bail(NS_EHIP, hipGetErrorString(e));
#undef NS_ALLOC
  *out = s;
  return NS_OK;
}
}  // namespace

int ns_solver_create(const ns_graph *g, const ns_params *p, void *stream,
                     ns_solver **out) {
  if (!g || !p || !out) { g_create_error = "null argument"; return NS_EINVAL; }
  return create_impl(one_mesh(g->mg), p, stream, out);
}

void ns_solver_destroy(ns_solver *s) {
  release(s);
  delete s;
}

int ns_set_state(ns_solver *s, const double *U, int flags) {
  if (!s || !U) return NS_EINVAL;
  const int tgt = others(s->cur, 0);
  hipError_t e = hipSuccess;
  if (flags & NS_ON_DEVICE) {
    ns::launch_nodes_from_cm(s->nc, U, s->N, s->S[tgt], s->N, 0, s->N, s->stream);
    e = hipGetLastError();
  } else {
    e = upload_nodes(s->S[tgt], s->N, s->nc, 0, s->N, U, s->N, s->stream);
  }
  if (e != hipSuccess) return s->hipfail(e, "state upload");
  ns::launch_clear_flags(s->flags, s->stream);
  ns::launch_check_state(s->dim, s->N, s->S[tgt], s->flags, s->stream);
  int rc = read_flags(s);
  if (rc != NS_OK) return rc;
  if (s->hflags[1]) {
    char buf[128];
    snprintf(buf, sizeof buf, "state not admissible at node %d", s->hflags[2]);
    return s->fail(NS_ENOTADMISSIBLE, buf);
  }
  if (!(flags & NS_NO_PROJECT)) {
    ns::launch_slip(s->dim, s->N, s->nslip, s->slip_idx, s->slip_n, s->S[tgt],
                    s->stream);
    e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return s->hipfail(e, "slip projection");
  }
  s->cur = tgt;
  s->has_state = true;
  return NS_OK;
}

int ns_get_state(ns_solver *s, double *U, int flags) {
  if (!s || !U) return NS_EINVAL;
  if (!s->has_state) return s->fail(NS_ESTATE, "no state set");
  hipError_t e = hipSuccess;
  if (flags & NS_ON_DEVICE) {
    ns::launch_nodes_to_cm(s->nc, s->S[s->cur], s->N, 0, s->N, U, s->N, s->stream);
    e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  } else {
    e = download_nodes(s->S[s->cur], s->N, s->nc, 0, s->N, U, s->N, s->stream);
  }
  if (e != hipSuccess) return s->hipfail(e, "state download");
  return NS_OK;
}

int ns_compute_dt(ns_solver *s, double *dt) {
  if (!s || !dt) return NS_EINVAL;
  if (!s->has_state) return s->fail(NS_ESTATE, "no state set");
  // prim + graph viscosity + reduction, without the rest of the stage
  const int o1 = others(s->cur, 0);
  ns::launch_clear_flags(s->flags, s->stream);
  if (s->mixed)
    ns::launch_dt_only(s->dim, s->gas, s->devgraph32(), s->args32(s->cur, o1, 0.0, 1.0, 0),
                       s->prm.cfl, s->stream, &Profiler::before, &Profiler::after,
                       &s->prof);
  else
    ns::launch_dt_only(s->dim, s->gas, s->devgraph(), s->args(s->cur, o1, 0.0, 1.0, 0),
                       s->prm.cfl, s->stream, &Profiler::before, &Profiler::after,
                       &s->prof);
  int rc = read_flags(s);
  if (rc != NS_OK) return rc;
  *dt = *s->htau;
  return NS_OK;
}

int ns_step(ns_solver *s, double dt) {
  if (!s) return NS_EINVAL;
  if (!(dt > 0.0) || !std::isfinite(dt)) return s->fail(NS_EINVAL, "dt must be positive");
  return ssprk3(s, dt, false, nullptr);
}

int ns_step_cfl(ns_solver *s, double *dt) {
  if (!s) return NS_EINVAL;
  return ssprk3(s, 0.0, true, dt);
}

int ns_step_adaptive(ns_solver *s, double c_start, double *dt, double *c_used) {
  if (!s) return NS_EINVAL;
  if (!(c_start > 0.0 && c_start <= 64.0))
    return s->fail(NS_EINVAL, "c_start must be in (0, 64]");
  if (!s->has_state) return s->fail(NS_ESTATE, "no state set");
  double c = c_start;
  for (int k = 0; k < 24; ++k, c *= 0.5) {
    s->adaptive = true;
    s->cfl_now = c;
    ns::launch_clear_flags(s->flags, s->stream);
    const int o1 = ssprk3_enqueue(s, 0.0, true);
    s->adaptive = false;
    const int rc = read_flags(s);
    if (rc != NS_OK) return rc;
    if (s->hflags[1] || s->hflags[3]) continue;  // restart with c / 2
    s->cur = o1;
    if (dt) *dt = *s->htau;
    if (c_used) *c_used = c;
    return NS_OK;
  }
  return s->fail(NS_EBOUNDS, "no CFL number c_start / 2^k, k < 24, kept the states admissible");
}

namespace {
// Multigrid levels (NS_PC_GMG): level 0 is the solver's mesh; a direction is
// coarsened while it has at least 4 cells (8 nodes if periodic), to
// ceil(cells/2) cells; stop at about 512 nodes or when nothing coarsens.
// The level structure is built (and its buffers allocated) once; the element
// tables, which depend on the viscous data, on every call.
int mg_build(ns_solver *s, const ns_viscous *v) {
  const int dim = s->dim;
  std::vector<ns::ParGrid> grids{par_grid(s)};
  std::vector<std::array<double, 3>> hs{{s->mg.h[0], s->mg.h[1], s->mg.h[2]}};
  while (grids.size() < 16 && grids.back().N > 512) {
    ns::ParGrid g = grids.back();
    std::array<double, 3> h = hs.back();
    bool any = false;
    for (int d = 0; d < dim; ++d) {
      const int64_t n = g.n[d], cells = g.per[d] ? n : n - 1;
      if (g.per[d] ? n < 8 : cells < 4) continue;
      const int64_t cc = (cells + 1) / 2;
      h[d] *= (double)cells / (double)cc;
      g.n[d] = g.per[d] ? cc : cc + 1;
      any = true;
    }
    if (!any) break;
    g.N = g.n[0] * g.n[1] * g.n[2];
    grids.push_back(g);
    hs.push_back(h);
  }
  const int nlev = (int)grids.size();
  hipError_t e = hipSuccess;
  if (s->mgl.empty()) {
    s->mgl.resize(nlev);
    for (int l = 0; l < nlev && e == hipSuccess; ++l) {
      ns::MGLevel &L = s->mgl[l];
      L.G = grids[l];
      const int64_t N = L.G.N, dN = (int64_t)dim * N;
      const int64_t nb = (N + ns::kParBlock - 1) / ns::kParBlock;
      float *tab = nullptr;
      ns::Q1Tables t;
      ns::build_q1_tables(dim, hs[l].data(), 1.0, 0.0, 1.0, &t);
      if (e == hipSuccess) e = s->alloc(&tab, t.packed().size());
      L.tab = tab;
      if (e == hipSuccess) e = s->alloc(&L.rm, N);
      for (float **pv : {&L.diag, &L.x, &L.y, &L.b, &L.d})
        if (e == hipSuccess) e = s->alloc(pv, dN);
      if (e == hipSuccess) e = s->alloc(&L.lmax, 1);
      if (e == hipSuccess) e = s->alloc(&L.gpart, nb);
    }
    if (e == hipSuccess) e = s->alloc(&s->mg_z, (size_t)dim * s->N);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      s->mgl.clear();
      return s->fail(NS_ENOMEM, "multigrid levels");
    }
  }
  e = hipStreamSynchronize(s->stream);
  for (int l = 0; l < (int)s->mgl.size() && e == hipSuccess; ++l) {
    ns::Q1Tables t;
    ns::build_q1_tables(dim, hs[l].data(), v->mu, v->lambda, v->kappa / v->cv, &t);
    const std::vector<double> td = t.packed();
    const std::vector<float> tf(td.begin(), td.end());
    e = hipMemcpy(const_cast<float *>(s->mgl[l].tab), tf.data(), tf.size() * sizeof(float),
                  hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return s->hipfail(e, "multigrid tables");
  return NS_OK;
}
}  // namespace

int ns_set_viscous(ns_solver *s, const ns_viscous *v) {
  if (!s || !v) return NS_EINVAL;
  const double vals[] = {v->mu, v->lambda, v->kappa, v->cv, v->cg_rtol};
  for (double x : vals)
    if (!std::isfinite(x)) return s->fail(NS_EINVAL, "viscous data must be finite");
  if (!(v->mu >= 0.0) || !(v->lambda >= 0.0) || !(v->kappa >= 0.0) || !(v->cv > 0.0) ||
      !(v->cg_rtol > 0.0 && v->cg_rtol < 1.0) || v->cg_maxit < 1 ||
      (v->fct != NS_FCT_AUTO && v->fct != NS_FCT_ALWAYS) ||
      (v->precond != NS_PC_JACOBI && v->precond != NS_PC_GMG))
    return s->fail(NS_EINVAL, "viscous data out of range (need mu, lambda, kappa >= 0, "
                              "cv > 0, 0 < cg_rtol < 1, cg_maxit >= 1, fct 0 or 1, "
                              "precond 0 or 1)");
  ns::Q1Tables t;
  ns::build_q1_tables(s->dim, s->mg.h, v->mu, v->lambda, v->kappa / v->cv, &t);
  const std::vector<double> tab = t.packed();
  hipError_t e = hipSuccess;
  if (!s->ptab) {
    const int64_t N = s->N, dN = (int64_t)s->dim * N;
    const int64_t nblocks = (N + ns::kParBlock - 1) / ns::kParBlock;
    ns::ParBufs &B = s->pb;
    double **dvecs[] = {&B.Vn, &B.x, &B.r, &B.p, &B.q, &B.b, &B.diag};
    double **nvecs[] = {&B.rm, &B.en, &B.K, &B.eH, &B.eL, &B.w, &B.Rp, &B.Rm};
    for (double **d : dvecs)
      if (e == hipSuccess) e = s->alloc(d, dN);
    for (double **d : nvecs)
      if (e == hipSuccess) e = s->alloc(d, N);
    if (e == hipSuccess) e = s->alloc(&B.cellK, (int64_t)(1 << s->dim) * N);
    if (e == hipSuccess) e = s->alloc(&B.partial, 3 * nblocks);
    if (e == hipSuccess) e = s->alloc(&B.cg, 1);
    if (e == hipSuccess) e = s->alloc(&B.scal, 4);
    if (e == hipSuccess) e = s->alloc(&s->ptab, tab.size());
    if (e == hipSuccess) e = s->alloc(&s->backup, (size_t)s->nc * N);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return s->fail(NS_ENOMEM, std::string("parabolic buffers: ") + hipGetErrorString(e));
    }
    B.tab = s->ptab;
    B.mi = s->mi;
    B.fixed = s->wall;
    B.flags = s->flags;
  }
  e = hipStreamSynchronize(s->stream);
  if (e == hipSuccess)
    e = hipMemcpy(s->ptab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) return s->hipfail(e, "element table upload");
  if (v->precond == NS_PC_GMG) {
    const int rc = mg_build(s, v);
    if (rc != NS_OK) return rc;
  }
  s->vprm = *v;
  s->viscous = true;
  return NS_OK;
}

int ns_step_parabolic(ns_solver *s, double dt) {
  if (!s) return NS_EINVAL;
  if (!(dt > 0.0) || !std::isfinite(dt)) return s->fail(NS_EINVAL, "dt must be positive");
  if (!s->has_state) return s->fail(NS_ESTATE, "no state set");
  if (!s->viscous) return s->fail(NS_ESTATE, "ns_set_viscous has not been called");
  if (s->nnr > 0)
    return s->fail(NS_ESTATE, "non-reflecting boundaries are for the Euler step only");
  const int o = others(s->cur, 0);
  const int rc = par_step(s, dt, s->cur, o);
  if (rc == NS_OK) s->cur = o;
  return rc;
}

int ns_step_strang(ns_solver *s, double tau) {
  if (!s) return NS_EINVAL;
  if (!(tau > 0.0) || !std::isfinite(tau)) return s->fail(NS_EINVAL, "tau must be positive");
  if (s->nnr > 0)
    return s->fail(NS_ESTATE, "non-reflecting boundaries are for the Euler step only");
  return strang(s, tau, false, nullptr);
}

int ns_step_strang_cfl(ns_solver *s, double *tau) {
  if (!s) return NS_EINVAL;
  if (s->nnr > 0)
    return s->fail(NS_ESTATE, "non-reflecting boundaries are for the Euler step only");
  return strang(s, 0.0, true, tau);
}

int ns_set_boundary(ns_solver *s, const ns_boundary *b) {
  if (!s || !b) return NS_EINVAL;
  if (s->pack) return s->fail(NS_EINVAL, "boundary kinds are set per solver, not per pack");
  const int dim = s->dim, nc = s->nc;
  const ns::MeshGraph &m = s->mg;
  if (b->method != NS_NR_CHARACTERISTIC && b->method != NS_NR_GODUNOV)
    return s->fail(NS_EINVAL, "unknown non-reflecting method");
  bool any_nr = false;
  for (int f = 0; f < 2 * dim; ++f) {
    if (b->kind[f] != NS_BC_SLIP && b->kind[f] != NS_BC_NONREFLECTING)
      return s->fail(NS_EINVAL, "unknown boundary kind");
    if (b->kind[f] != NS_BC_NONREFLECTING || m.periodic[f / 2]) continue;
    any_nr = true;
    // admissible far-field state with (gamma-1)/2 v_n^D <= a^D on this face
    const double *u = b->state[f];
    double m2 = 0.0;
    bool fin = std::isfinite(u[0]) && std::isfinite(u[dim + 1]);
    for (int k = 0; k < dim; ++k) { fin = fin && std::isfinite(u[1 + k]); m2 += u[1 + k] * u[1 + k]; }
    const double p = s->gas.gm1 * (u[dim + 1] - 0.5 * m2 / u[0]);
    if (!fin || !(u[0] > 0.0) || !(p > 0.0))
      return s->fail(NS_EINVAL, "far-field state of a non-reflecting face not admissible");
    const double vn = (f % 2 ? 1.0 : -1.0) * u[1 + f / 2] / u[0];
    if (0.5 * s->gas.gm1 * vn > std::sqrt(s->gas.gamma * p / u[0]))
      return s->fail(NS_EINVAL, "far-field state violates (gamma-1)/2 v_n <= a on its face");
  }
  (void)any_nr;
  // node sets and normals (eq. def_ns_nio) from the faces' integrals of phi_i
  const int64_t N = s->N;
  std::vector<int32_t> sidx, nidx;
  std::vector<double> sn, nn, nud;
  for (int64_t i = 0; i < N; ++i) {
    int64_t a[3];
    m.coords(i, a);
    double ns_[3] = {0, 0, 0}, nr_[3] = {0, 0, 0};
    int first_nr = -1;
    bool on_s = false, on_nr = false;
    for (int f = 0; f < 2 * dim; ++f) {
      const int d = f / 2;
      if (m.periodic[d] || a[d] != (f % 2 ? m.n[d] - 1 : 0)) continue;
      double w = 1.0;  // int over face f of phi_i
      for (int e = 0; e < dim; ++e)
        if (e != d) w *= m.ml(e, a[e]);
      const double sg = f % 2 ? 1.0 : -1.0;
      if (b->kind[f] == NS_BC_NONREFLECTING) {
        nr_[d] += sg * w;
        on_nr = true;
        if (first_nr < 0) first_nr = f;
      } else {
        ns_[d] += sg * w;
        on_s = true;
      }
    }
    auto unit = [dim](double *v) {
      double l = 0.0;
      for (int k = 0; k < dim; ++k) l += v[k] * v[k];
      l = std::sqrt(l);
      for (int k = 0; k < dim; ++k) v[k] /= l;
      return l > 0.0;
    };
    if (on_s && unit(ns_)) {
      sidx.push_back((int32_t)i);
      for (int k = 0; k < dim; ++k) sn.push_back(ns_[k]);
    }
    if (on_nr && unit(nr_)) {
      nidx.push_back((int32_t)i);
      for (int k = 0; k < dim; ++k) nn.push_back(nr_[k]);
      for (int c = 0; c < nc; ++c) nud.push_back(b->state[first_nr][c]);
    }
  }
  // structure of arrays on the device
  const int nsl = (int)sidx.size(), nnr = (int)nidx.size();
  std::vector<double> snT((size_t)dim * nsl), nnT((size_t)dim * nnr), udT((size_t)nc * nnr);
  for (int t = 0; t < nsl; ++t)
    for (int k = 0; k < dim; ++k) snT[(size_t)k * nsl + t] = sn[(size_t)t * dim + k];
  for (int t = 0; t < nnr; ++t) {
    for (int k = 0; k < dim; ++k) nnT[(size_t)k * nnr + t] = nn[(size_t)t * dim + k];
    for (int c = 0; c < nc; ++c) udT[(size_t)c * nnr + t] = nud[(size_t)t * nc + c];
  }
  // a captured step holds the old lists: drop it
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return s->hipfail(e, "stream synchronize");
  for (hipGraphExec_t &gx : s->step_graph) {
    if (gx) (void)hipGraphExecDestroy(gx);
    gx = nullptr;
  }
  s->free_one(s->slip_idx, s->nslip);
  s->free_one(s->slip_n, (size_t)dim * s->nslip);
  s->free_one(s->nr_idx, s->nnr);
  s->free_one(s->nr_n, (size_t)dim * s->nnr);
  s->free_one(s->nr_ud, (size_t)nc * s->nnr);
  s->nslip = 0;
  s->nnr = 0;
  if ((e = s->alloc(&s->slip_idx, nsl)) != hipSuccess ||
      (e = s->alloc(&s->slip_n, (size_t)dim * nsl)) != hipSuccess ||
      (e = s->alloc(&s->nr_idx, nnr)) != hipSuccess ||
      (e = s->alloc(&s->nr_n, (size_t)dim * nnr)) != hipSuccess ||
      (e = s->alloc(&s->nr_ud, (size_t)nc * nnr)) != hipSuccess) {
    (void)hipGetLastError();
    return s->fail(NS_ENOMEM, "boundary lists");
  }
  struct { void *dst; const void *src; size_t n; } ups[] = {
      {s->slip_idx, sidx.data(), sidx.size() * sizeof(int32_t)},
      {s->slip_n, snT.data(), snT.size() * sizeof(double)},
      {s->nr_idx, nidx.data(), nidx.size() * sizeof(int32_t)},
      {s->nr_n, nnT.data(), nnT.size() * sizeof(double)},
      {s->nr_ud, udT.data(), udT.size() * sizeof(double)}};
  for (auto &u : ups) {
    if (u.n == 0) continue;
    e = hipMemcpyAsync(u.dst, u.src, u.n, hipMemcpyHostToDevice, s->stream);
    if (e != hipSuccess) return s->hipfail(e, "boundary upload");
  }
  e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return s->hipfail(e, "boundary upload");
  s->nslip = nsl;
  s->nnr = nnr;
  s->nr_method = b->method;
  return NS_OK;
}

int ns_parabolic_info(ns_solver *s, ns_par_info *out) {
  if (!s || !out) return NS_EINVAL;
  *out = s->pinfo;
  return NS_OK;
}

namespace {
// The graph of one CFL step from the current buffer (see ns_solver), or null
// if it cannot be captured (or the profiler, which records events around
// every launch, is on).  A replay launches the same kernels with the same
// arguments in the same order as ssprk3_enqueue + launch_add_scalar.
hipGraphExec_t step_graph(ns_solver *s) {
  if (s->graphs_off || s->prof.on) return nullptr;
  hipGraphExec_t &ex = s->step_graph[s->cur];
  if (ex) return ex;
  hipError_t e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    s->graphs_off = true;
    return nullptr;
  }
  const int last = s->last_out;
  (void)ssprk3_enqueue(s, 0.0, true);
  ns::launch_add_scalar(s->tacc, s->tau, s->stream, s->nmem);
  s->last_out = last;
  hipGraph_t gr = nullptr;
  e = hipStreamEndCapture(s->stream, &gr);
  if (e == hipSuccess) e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
  if (gr) (void)hipGraphDestroy(gr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    ex = nullptr;
    s->graphs_off = true;
  }
  return ex;
}
}  // namespace

extern "C++" {
namespace {
// An event for the end of an asynchronous call (from the pool, or new).
int take_event(ns_solver *s, hipEvent_t *ev) {
  *ev = nullptr;
  if (!s->ev_pool.empty()) {
    *ev = s->ev_pool.back();
    s->ev_pool.pop_back();
    return NS_OK;
  }
  hipError_t e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
  if (e != hipSuccess) return s->hipfail(e, "event create");
  return NS_OK;
}

// A new asynchronous run: the sticky status and the time start at 0.
void open_async(ns_solver *s) {
  if (s->async_open) return;
  ns::launch_clear_flags(s->flags, s->stream, s->nmem);
  ns::launch_persist_reset(s->pdone, s->pcnt, s->pticket, s->pstop, s->nmem, true, s->stream);
  ns::launch_set_scalar(s->tacc, 0.0, s->stream, s->nmem);
  if (s->give_up) __atomic_store_n(s->give_up, 0, __ATOMIC_SEQ_CST);
  s->async_open = true;
}

// After a run's status readback (hpstop): did a persistent launch of the run
// give up?  Then its steps stopped part-way: the state is undefined until a
// new one is set, and the give-up word is cleared for the next run.
bool persistent_gave_up(ns_solver *s) {
  if (s->hpstop[2] == 0) return false;
  s->err = s->hpstop[2] & 4 ? "persistent steps gave up: give-up word set"
                            : "persistent steps gave up: wait limit reached";
  s->has_state = false;
  std::fill(s->mset.begin(), s->mset.end(), 0);
  if (s->give_up) __atomic_store_n(s->give_up, 0, __ATOMIC_SEQ_CST);
  return true;
}

// Records the end of an asynchronous call (ev) after its launches.
int close_call(ns_solver *s, hipEvent_t ev, hipError_t e, const char *what) {
  if (e == hipSuccess) e = hipEventRecord(ev, s->stream);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) {
    s->ev_pool.push_back(ev);
    return s->hipfail(e, what);
  }
  s->inflight.push_back(ev);
  return NS_OK;
}

template <typename LT>
ns::PersistArgsT<LT> persist_args(const ns_solver *s, const ns::StageArgsT<LT> &a,
                                  int nsteps, double wait_s, int items_step,
                                  const ns::PersistPlan &plan) {
  ns::PersistArgsT<LT> P{};
  P.A = a;
  for (int b = 0; b < 3; ++b) P.S[b] = s->S[b];
  P.cur = s->cur;
  P.nsteps = nsteps;
  P.cfl = s->prm.cfl;
  P.tacc = s->tacc;
  P.mblk = s->pmblk;
  P.rblk = s->prblk;
  P.sblk = s->psblk;
  P.mslip = s->pmslip;
  P.slip_idx = s->slip_idx;
  P.slip_n = s->slip_n;
  P.nslip = s->nslip;
  P.pcnt = s->pcnt;
  P.done = s->pdone;
  P.ticket = s->pticket;
  P.stop = s->pstop;
  P.give_up = give_up_device(s->give_up);
  P.items_step = (uint32_t)items_step;
  P.items = (uint32_t)((int64_t)nsteps * items_step);
  int dev = s->device, khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) {
    (void)hipGetLastError();
    khz = 100000;  // the 100 MHz constant clock of the CDNA parts
  }
  P.wait_ticks = (uint64_t)std::min(wait_s * 1e3 * khz, 1.8e19);
  P.plan = plan;
  return P;
}
}  // namespace
}  // extern "C++"

int ns_step_cfl_async(ns_solver *s, int nsteps) {
  if (!s || nsteps < 0) return NS_EINVAL;
  if (!s->has_state) return s->fail(NS_ESTATE, "no state set");
  hipEvent_t ev = nullptr;
  int rc = take_event(s, &ev);
  if (rc != NS_OK) return rc;
  open_async(s);
  hipError_t e = hipSuccess;
  for (int k = 0; k < nsteps && e == hipSuccess; ++k) {
    const hipGraphExec_t g = step_graph(s);
    const int o1 = others(s->cur, 0);
    if (g) {
      e = hipGraphLaunch(g, s->stream);
      if (e != hipSuccess) break;
    } else {
      (void)ssprk3_enqueue(s, 0.0, true);
      ns::launch_add_scalar(s->tacc, s->tau, s->stream, s->nmem);
    }
    s->last_out = o1;
    s->cur = o1;
  }
  return close_call(s, ev, e, "asynchronous step launch");
}

int ns_step_cfl_persistent(ns_solver *s, int nsteps, double wait_s) {
  if (!s || nsteps < 0 || !(wait_s > 0.0) || !std::isfinite(wait_s)) return NS_EINVAL;
  if (!s->has_state) return s->fail(NS_ESTATE, "no state set");
  if (s->prm.indicator != NS_IND_ENTROPY || s->prm.limiter != NS_LIM_CONVEX ||
      s->prm.passes != 2)
    return s->fail(NS_EINVAL, "persistent steps need the entropy indicator and convex "
                              "limiting with two passes");
  if (s->nnr > 0)
    return s->fail(NS_EINVAL, "persistent steps do not treat non-reflecting boundaries");
  if (s->fp32_eval)
    return s->fail(NS_EINVAL, "persistent steps run FP64 or FP32-storage arithmetic only");
  if (!s->give_up && !(s->give_up = take_give_up_word()))
    return s->fail(NS_ENOMEM, "no give-up word left (pinned host memory)");
  if (s->pgrid <= 0) {
    s->pgrid = ns::persist_grid(s->dim, s->gas.seven != 0, s->mixed);
    if (s->pgrid <= 0) return s->fail(NS_EHIP, "occupancy query of the persistent kernel");
  }
  ns::PersistPlan plan;
  ns::persist_plan(s->dim, s->rows_tot, s->roots_tot, s->slips_tot, s->nmem, &plan);
  const int64_t items_step = plan.off[plan.nph];
  if ((int64_t)nsteps * items_step > (int64_t)INT32_MAX)
    return s->fail(NS_EINVAL, "too many steps for one persistent launch");
  hipEvent_t ev = nullptr;
  int rc = take_event(s, &ev);
  if (rc != NS_OK) return rc;
  open_async(s);
  if (nsteps > 0) {
    const int64_t items = (int64_t)nsteps * items_step;
    // twice the widest phase: the next phase's items are taken while one
    // ends, without many more workgroups waiting
    const int grid =
        (int)std::min<int64_t>(std::min<int64_t>(s->pgrid, items), 2 * s->rows_tot + 8);
    ns::launch_persist_reset(s->pdone, s->pcnt, s->pticket, s->pstop, s->nmem, false,
                             s->stream);
    if (s->mixed)
      ns::launch_persistent(s->dim, s->gas, s->devgraph32(),
                            persist_args(s, s->args32(s->cur, s->cur, 0.0, 1.0, 0), nsteps,
                                         wait_s, (int)items_step, plan),
                            grid, s->stream);
    else
      ns::launch_persistent(s->dim, s->gas, s->devgraph(),
                            persist_args(s, s->args(s->cur, s->cur, 0.0, 1.0, 0), nsteps,
                                         wait_s, (int)items_step, plan),
                            grid, s->stream);
    for (int k = 0; k < nsteps; ++k) s->cur = others(s->cur, 0);
    s->last_out = s->cur;
  }
  return close_call(s, ev, hipSuccess, "persistent step launch");
}

int ns_cancel(ns_solver *s) {
  if (!s) return NS_EINVAL;
  if (s->give_up) __atomic_store_n(s->give_up, 1, __ATOMIC_SEQ_CST);
  return NS_OK;
}

int ns_inflight(ns_solver *s, int *calls) {
  if (!s || !calls) return NS_EINVAL;
  while (!s->inflight.empty()) {
    const hipError_t e = hipEventQuery(s->inflight.front());
    if (e == hipErrorNotReady) break;
    if (e != hipSuccess) return s->hipfail(e, "event query");
    s->ev_pool.push_back(s->inflight.front());
    s->inflight.pop_front();
  }
  *calls = (int)s->inflight.size();
  return NS_OK;
}

int ns_query(ns_solver *s, int *done) {
  if (!s || !done) return NS_EINVAL;
  int n = 0;
  const int rc = ns_inflight(s, &n);
  *done = n == 0;
  return rc;
}

struct ns_pack {
  ns_solver *s = nullptr;
};

int ns_pack_footprint(const ns_graph *const *graphs, int count, const ns_params *p,
                      int64_t *bytes) {
  if (!graphs || count < 1 || !p || !bytes) return NS_EINVAL;
  std::vector<const ns::MeshGraph *> m;
  for (int r = 0; r < count; ++r) {
    if (!graphs[r] || graphs[r]->mg.dim != graphs[0]->mg.dim) return NS_EINVAL;
    m.push_back(&graphs[r]->mg);
  }
  *bytes = footprint(packed(m.data(), count), p);
  return NS_OK;
}

int ns_pack_create(const ns_graph *const *graphs, int count, const ns_params *p,
                   void *hip_stream, ns_pack **out) {
  if (!graphs || count < 1 || !p || !out) {
    g_create_error = "null argument or empty pack";
    return NS_EINVAL;
  }
  std::vector<const ns::MeshGraph *> m;
  for (int r = 0; r < count; ++r) {
    if (!graphs[r] || graphs[r]->mg.dim != graphs[0]->mg.dim) {
      g_create_error = "pack members must be graphs of one dimension";
      return NS_EINVAL;
    }
    m.push_back(&graphs[r]->mg);
  }
  ns_pack *k = new (std::nothrow) ns_pack;
  if (!k) { g_create_error = "host allocation"; return NS_ENOMEM; }
  const int rc = create_impl(packed(m.data(), count), p, hip_stream, &k->s);
  if (rc != NS_OK) {
    delete k;
    return rc;
  }
  *out = k;
  return NS_OK;
}

void ns_pack_destroy(ns_pack *k) {
  if (!k) return;
  ns_solver_destroy(k->s);
  delete k;
}

int ns_pack_set_state(ns_pack *k, int r, const double *U) {
  if (!k || !U) return NS_EINVAL;
  ns_solver *s = k->s;
  if (r < 0 || r >= s->nmem) return s->fail(NS_EINVAL, "no such pack member");
  const int64_t Nr = s->mgs[r].N, b0 = s->mbase[r], nc = s->nc, dim = s->dim;
  for (int64_t i = 0; i < Nr; ++i) {
    const double rho = U[i], E = U[(dim + 1) * Nr + i];
    double m2 = 0.0;
    bool fin = std::isfinite(rho) && std::isfinite(E);
    for (int d = 0; d < dim; ++d) {
      const double mk = U[(1 + d) * Nr + i];
      fin = fin && std::isfinite(mk);
      m2 += mk * mk;
    }
    if (!fin || !(rho > 0.0) || !(E - 0.5 * m2 / rho > 0.0)) {
      char buf[128];
      snprintf(buf, sizeof buf, "state of pack member %d not admissible at node %lld", r,
               (long long)i);
      return s->fail(NS_ENOTADMISSIBLE, buf);
    }
  }
  hipError_t e = upload_nodes(s->S[s->cur], s->N, (int)nc, b0, Nr, U, Nr, s->stream);
  if (e != hipSuccess) return s->hipfail(e, "state upload");
  const int64_t t0 = s->mslip[r], t1 = s->mslip[r + 1];
  ns::launch_slip(s->dim, s->N, (int)(t1 - t0), s->slip_idx + t0, s->slip_n + t0,
                  s->S[s->cur], s->stream, s->nslip);
  e = hipStreamSynchronize(s->stream);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return s->hipfail(e, "state upload");
  s->mset[r] = 1;
  s->has_state = std::all_of(s->mset.begin(), s->mset.end(), [](char c) { return c != 0; });
  return NS_OK;
}

int ns_pack_get_state(ns_pack *k, int r, double *U) {
  if (!k || !U) return NS_EINVAL;
  ns_solver *s = k->s;
  if (r < 0 || r >= s->nmem) return s->fail(NS_EINVAL, "no such pack member");
  if (!s->mset[r]) return s->fail(NS_ESTATE, "no state set");
  const int64_t Nr = s->mgs[r].N;
  hipError_t e = download_nodes(s->S[s->cur], s->N, s->nc, s->mbase[r], Nr, U, Nr, s->stream);
  if (e != hipSuccess) return s->hipfail(e, "state download");
  return NS_OK;
}

int ns_pack_step_cfl_async(ns_pack *k, int nsteps) {
  if (!k) return NS_EINVAL;
  return ns_step_cfl_async(k->s, nsteps);
}

int ns_pack_inflight(ns_pack *k, int *calls) {
  if (!k) return NS_EINVAL;
  return ns_inflight(k->s, calls);
}

int ns_pack_finish(ns_pack *k, int *status, double *t) {
  if (!k || !status || !t) return NS_EINVAL;
  ns_solver *s = k->s;
  if (!s->async_open) return s->fail(NS_ESTATE, "no asynchronous steps enqueued");
  s->async_open = false;
  const int nm = s->nmem;
  std::vector<int> fl(4 * (size_t)nm);
  std::vector<double> ta(nm);
  hipError_t e = hipMemcpyAsync(fl.data(), s->flags, fl.size() * sizeof(int),
                                hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ta.data(), s->tacc, nm * sizeof(double), hipMemcpyDeviceToHost,
                       s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->hpstop, s->pstop, 4 * sizeof(int), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return s->hipfail(e, "asynchronous step status");
  const bool gave_up = persistent_gave_up(s);
  for (int r = 0; r < nm; ++r) {
    status[r] = gave_up                                           ? NS_EABORT
                : fl[4 * r]                                       ? NS_ECFL
                : fl[4 * r + 1] || (s->fp32_eval && fl[4 * r + 3]) ? NS_EBOUNDS
                                                                  : NS_OK;
    t[r] = ta[r];
  }
  return NS_OK;
}

int ns_pack_step_cfl_persistent(ns_pack *k, int nsteps, double wait_s) {
  if (!k) return NS_EINVAL;
  return ns_step_cfl_persistent(k->s, nsteps, wait_s);
}

int ns_pack_cancel(ns_pack *k) {
  if (!k) return NS_EINVAL;
  return ns_cancel(k->s);
}

const char *ns_pack_error(const ns_pack *k) {
  if (!k) return ns_create_error();
  return k->s->err.c_str();
}

int ns_async_finish(ns_solver *s, double *t) {
  if (!s) return NS_EINVAL;
  if (!s->async_open) return s->fail(NS_ESTATE, "no asynchronous steps enqueued");
  s->async_open = false;
  hipError_t e = hipMemcpyAsync(s->hflags, s->flags, 4 * sizeof(int), hipMemcpyDeviceToHost,
                                s->stream);
  double tt = 0.0;
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->htau, s->tacc, sizeof(double), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(s->hpstop, s->pstop, 4 * sizeof(int), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return s->hipfail(e, "asynchronous step status");
  tt = *s->htau;
  if (t) *t = tt;
  if (persistent_gave_up(s)) return NS_EABORT;
  if (s->hflags[0]) return s->fail(NS_ECFL, "a step exceeded the stage CFL limit");
  if (s->hflags[1] || (s->fp32_eval && s->hflags[3]))
    return s->fail(NS_EBOUNDS, "a stage produced an inadmissible state");
  return NS_OK;
}

int ns_fe_stage(ns_solver *s, double dt) {
  if (!s) return NS_EINVAL;
  if (!s->has_state) return s->fail(NS_ESTATE, "no state set");
  if (!(dt > 0.0) || !std::isfinite(dt)) return s->fail(NS_EINVAL, "dt must be positive");
  const int o1 = others(s->cur, 0);
  ns::launch_clear_flags(s->flags, s->stream);
  ns::launch_set_scalar(s->tau, dt, s->stream);
  run_stage(s, s->cur, o1, 0.0, 1.0, 1, false);
  s->last_out = o1;
  int rc = read_flags(s);
  if (rc != NS_OK) return rc;
  if (s->hflags[0]) return s->fail(NS_ECFL, "dt exceeds the stage CFL limit");
  if (s->hflags[1]) return s->fail(NS_EBOUNDS, "the stage produced an inadmissible state");
  return NS_OK;
}

int ns_get_debug(ns_solver *s, int what, double *out) {
  if (!s || !out) return NS_EINVAL;
  const int64_t N = s->N, W = s->W, nc = s->nc, Np = s->Np;
  const double *src = nullptr;
  const float *srcf = nullptr;  // FP32 storage in the mixed-precision mode
  int64_t count = 0;
  bool edge = false, node = false;  // node: a node vector (node_layout.hpp)
  int K = (int)nc, Kout = (int)nc;   // its components, the first Kout exported
  switch (what) {
    case NS_DBG_STAGE_OUT: src = s->S[s->last_out]; count = nc * N; node = true; break;
    case NS_DBG_D: src = s->d; srcf = s->df; count = W * Np; edge = true; break;
    case NS_DBG_ALPHA: src = s->alpha; srcf = s->alphaf; count = N; break;
    case NS_DBG_UL: src = s->UL; count = nc * N; node = true; break;
    case NS_DBG_FH:
      src = s->FH; srcf = s->FHf; count = (nc + (s->dim == 3)) * N; node = true;
      K = (int)nc + (s->dim == 3); break;
    case NS_DBG_BOUNDS: src = s->bnds; count = 3 * N; node = true; K = Kout = 3; break;
    case NS_DBG_LT1: src = s->lt1; srcf = s->lt1f; count = W * Np; edge = true; break;
    case NS_DBG_LT2: src = s->lt2; srcf = s->lt2f; count = W * Np; edge = true; break;
    case NS_DBG_U1: src = s->U1; count = nc * N; node = true; break;
    case NS_DBG_ROOTS: {
      uint32_t c[2];
      hipError_t e = hipMemcpyAsync(c, s->qcnt, sizeof(c), hipMemcpyDeviceToHost, s->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
      if (e != hipSuccess) return s->hipfail(e, "debug download");
      out[0] = c[0];
      out[1] = c[1];
      return NS_OK;
    }
    default: return s->fail(NS_EINVAL, "unknown debug array");
  }
  const bool f32 = s->mixed && srcf != nullptr;
  const bool raw = edge || node || f32;  // downloaded to tmp, then rearranged
  std::vector<double> tmp(raw ? count : 0);
  std::vector<float> tmpf(f32 ? count : 0);
  hipError_t e = f32 ? hipMemcpyAsync(tmpf.data(), srcf, count * sizeof(float),
                                      hipMemcpyDeviceToHost, s->stream)
                     : hipMemcpyAsync(raw ? tmp.data() : out, src, count * sizeof(double),
                                      hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return s->hipfail(e, "debug download");
  if (f32)
    for (int64_t t = 0; t < count; ++t) tmp[t] = tmpf[t];
  if (edge) {
    for (int k = 0; k < W; ++k)
      for (int64_t i = 0; i < N; ++i)
        out[k * N + i] = tmp[((i >> 6) * W + k) * 64 + (i & 63)];
  } else if (node) {
    for (int c = 0; c < Kout; ++c)  // out holds Kout*N values
      for (int64_t i = 0; i < N; ++i) out[c * N + i] = tmp[ns::node_at(K, c, i, N)];
  } else if (raw) {
    std::copy(tmp.begin(), tmp.end(), out);
  }
  return NS_OK;
}

extern "C++" {
namespace {
// Fills *out from the current state and the last stage's limiter arrays;
// part holds 7 * kStatsParts + 7 doubles of device scratch (the last 7 the
// result).  Synchronises the solver's stream.
int stats_into(ns_solver *s, double *part, ns_stats_t *out) {
  const int lim = s->prm.limiter == NS_LIM_CONVEX && s->stage_ran;
  const int mode = lim ? (s->prm.passes == 2 ? 2 : 1) : 0;
  double *res = part + 7 * ns::kStatsParts;
  const double *U = s->S[s->cur];
  if (s->mixed)
    ns::launch_stats(s->dim, s->devgraph32(), U, s->lt1f, s->lt2f, mode, part, res, s->stream);
  else
    ns::launch_stats(s->dim, s->devgraph(), U, s->lt1, s->lt2, mode, part, res, s->stream);
  double h[7];
  uint32_t c[2] = {0, 0};
  hipError_t e = hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c, s->qcnt, sizeof(c), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return s->hipfail(e, "statistics");
  *out = ns_stats_t{};
  out->min_rho = h[0];
  out->argmin_rho = (int64_t)h[1];
  out->min_eps = h[2];
  out->argmin_eps = (int64_t)h[3];
  out->edges = (int64_t)h[4];
  out->limited1 = mode >= 1 ? (int64_t)h[5] : -1;
  out->limited2 = mode == 2 ? (int64_t)h[6] : -1;
  out->roots1 = lim ? (int64_t)c[0] : -1;
  out->roots2 = mode == 2 ? (int64_t)c[1] : -1;
  out->cg_it_v = s->pinfo.it_v;
  out->cg_it_e = s->pinfo.it_e;
  out->cg_it_l = s->pinfo.it_l;
  out->fct = s->pinfo.fct;
  out->min_eH = s->pinfo.min_eH;
  out->fp64_redo = s->fp64_redo;
  return NS_OK;
}
}  // namespace
}  // extern "C++"

int ns_stats(ns_solver *s, ns_stats_t *out) {
  if (!s || !out) return NS_EINVAL;
  if (!s->has_state) return s->fail(NS_ESTATE, "no state set");
  double *part = nullptr;
  hipError_t e = hipMallocAsync((void **)&part, (7 * ns::kStatsParts + 7) * sizeof(double),
                                s->stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return s->fail(NS_ENOMEM, "statistics scratch does not fit");
  }
  const int rc = stats_into(s, part, out);
  (void)hipFreeAsync(part, s->stream);
  return rc;
}

// ---- statistics without allocation ------------------------------------
// The partial results of ns_stats_noalloc live in this fixed array, one copy
// in each device's memory for as long as the process runs.  In host code its
// name only stands in for the device array: the device address is looked up
// once per device with hipGetSymbolAddress and kept in g_scratch.
static __device__ __align__(256) double scratch[7 * ns::kStatsParts + 7];

extern "C++" {
namespace {
std::mutex g_scratch_mu;
std::vector<double *> g_scratch;  // index: device; null until looked up

// Device address of `scratch` on device dev, which must be current.
hipError_t scratch_address(int dev, double **p) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch.size() <= dev) g_scratch.resize(dev + 1, nullptr);
  if (!g_scratch[dev]) {
    void *q = nullptr;
    const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = static_cast<double *>(q);
  }
  *p = g_scratch[dev];
  return hipSuccess;
}
}  // namespace
}  // extern "C++"

int ns_stats_noalloc(ns_solver *s, ns_stats_t *out) {
  if (!s || !out) return NS_EINVAL;
  if (!s->has_state) return s->fail(NS_ESTATE, "no state set");
  // the statistics kernels stride over the rows with at most kStatsParts
  // workgroups, so the partial results of any mesh fit in `scratch`
  static_assert(sizeof(scratch) == (7 * ns::kStatsParts + 7) * sizeof(double),
                "statistics scratch size");
  const int prev = ns::current_device();
  if (prev != s->device) ns::use_device(s->device);
  double *part = nullptr;
  int rc = NS_OK;
  const hipError_t e = scratch_address(s->device, &part);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    rc = s->fail(NS_EHIP, std::string("statistics scratch lookup: ") + hipGetErrorString(e));
  } else {
    rc = stats_into(s, part, out);
  }
  if (prev != s->device) ns::use_device(prev);
  return rc;
}

int ns_sync(ns_solver *s) {
  if (!s) return NS_EINVAL;
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return s->hipfail(e, "stream synchronize");
  return NS_OK;
}

void *ns_stream(ns_solver *s) { return s ? (void *)s->stream : nullptr; }

int ns_profile_enable(ns_solver *s, int on) {
  if (!s) return NS_EINVAL;
  s->prof.reset();
  s->prof.on = on != 0;
  return NS_OK;
}

int ns_profile_count(ns_solver *s) {
  if (!s) return 0;
  return (int)s->prof.names.size();
}

int ns_profile_get(ns_solver *s, int k, const char **name, int64_t *launches,
                   double *total_ms) {
  if (!s) return NS_EINVAL;
  s->prof.flush();
  if (k < 0 || k >= (int)s->prof.names.size()) return NS_EINVAL;
  if (name) *name = s->prof.names[k].c_str();
  if (launches) *launches = s->prof.launches[k];
  if (total_ms) *total_ms = s->prof.total_ms[k];
  return NS_OK;
}

int ns_copy_bench(ns_solver *s, int64_t bytes, int reps, int word,
                  double *avg_ms) {
  if (!s || !avg_ms || bytes < 16 || reps < 1 || (word != 8 && word != 16))
    return NS_EINVAL;
  const char *label = word == 8 ? "copy8" : "copy";
  const int64_t n16 = bytes / 16;
  void *a = nullptr, *b = nullptr;
  hipError_t e = hipMalloc(&a, n16 * 16);
  if (e == hipSuccess) e = hipMalloc(&b, n16 * 16);
  if (e != hipSuccess) {
    if (a) (void)hipFree(a);
    (void)hipGetLastError();
    return s->fail(NS_ENOMEM, "copy buffers do not fit");
  }
  hipEvent_t t0, t1;
  (void)hipEventCreate(&t0);
  (void)hipEventCreate(&t1);
  e = hipMemsetAsync(a, 0, n16 * 16, s->stream);
  ns::launch_copy(a, b, n16, word, s->stream);  // warm-up
  (void)hipEventRecord(t0, s->stream);
  for (int r = 0; r < reps; ++r) {
    Profiler::before(&s->prof, label);
    ns::launch_copy(r % 2 ? b : a, r % 2 ? a : b, n16, word, s->stream);
    Profiler::after(&s->prof);
  }
  (void)hipEventRecord(t1, s->stream);
  if (e == hipSuccess) e = hipEventSynchronize(t1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  (void)hipFree(a);
  (void)hipFree(b);
  if (e != hipSuccess) return s->hipfail(e, "copy benchmark");
  *avg_ms = ms / reps;
  return NS_OK;
}

int64_t ns_device_bytes(const ns_solver *s) { return s ? s->bytes : 0; }

const char *ns_last_error(const ns_solver *s) {
  return s ? s->err.c_str() : "null solver";
}

}  // extern "C"
