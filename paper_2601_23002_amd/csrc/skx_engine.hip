// Serving engine of libskx: continuous batching of independent density
// optimisations on one device.
//
// Requests are queued on submit (inputs copied). Every engine step admits
// queued requests in arrival order while a slot is free and their device
// footprint fits the HBM budget, then advances every resident solve by a
// fixed number of fused step sequences: one launch per kernel over all
// resident solves of one precision, exactly the schedule of skx_run_batch.
// A solve's arithmetic does not depend on which other solves share its
// launches, so an engine result equals the result of solving alone.
// Mixed-precision requests run their FP32 phase in the FP32 group and move
// to the FP64 group for the refinement; finished solves leave at once and
// their slots are refilled on the next step.
#include "skx_host.hpp"
#include "skx_device.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <string>
#include <vector>

using namespace skx;
using namespace skx::host;

namespace {

// step sequences per engine step: a solve that finishes (or leaves its FP32
// phase) mid-chunk idles until the chunk ends, and queued requests wait for
// it too (measured on MI355X, serving at 200 requests/s: 53.0-53.3 served
// per second with 4, 53.6 with 3, 54.2-54.6 with 2, 54.7 with 1)
constexpr int ENGINE_CHUNK = 2;

struct Queued {
  uint64_t ticket;
  skx_request req;                       // pointers re-aimed at the vectors below
  std::vector<double> pos, zval, rc;
  std::vector<int> species;
  size_t bytes;
};

struct Resident {
  uint64_t ticket;
  skx_ctx *ctx = nullptr;
  int mode;                              // SKX_FP64 / SKX_FP32 / SKX_MIXED
  int prec;                              // instance now running: 0 FP64, 1 FP32
  skx_opt_params opt;
  double t_arrival, t_admit;
  OptState o32{};                        // FP32 phase of a mixed solve
  bool had_fp32 = false;
  size_t bytes;
};

struct Finished {
  skx_result res;
  double *rho_dev = nullptr;             // engine-owned until polled
};

struct Group {
  std::vector<Resident *> members;
  bool dirty = true;
  SolveDev *ddev = nullptr;
  int *dfirst = nullptr;
  int *dphase = nullptr;
  int cap = 0;
  BatchLaunch bl{};
  // one engine step of this group (normalisation, the step sequences, the
  // phase gather) captured for the current membership
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void drop_graph() {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  }
};

}  // namespace

struct skx_engine {
  int device = 0;
  hipStream_t stream = nullptr;          // set-up, results, the FP64 group
  hipStream_t stream32 = nullptr;        // the FP32 group, overlapping the FP64 group's steps
  size_t budget = 0, used = 0;
  size_t held = 0;                       // finished densities waiting to be polled
  int max_slots = 0;
  uint64_t next_ticket = 1;
  std::deque<Queued> queue;
  std::vector<Resident *> resident;
  Group group[2];                        // by precision: 0 FP64, 1 FP32
  std::deque<Finished> done;
  // contexts of finished solves kept for reuse by a request of the same grid
  // (their device arenas stay allocated: no allocation or free, and so no
  // device-wide synchronisation, per request)
  // (bytes: the footprint of the context's arenas as allocated, i.e. for
  // the largest history length it has held)
  struct Pooled { skx_ctx *ctx; int n1, n2, n3, mode, m; size_t bytes; };
  std::vector<Pooled> pool;
  size_t pooled = 0;                     // bytes held by pooled contexts
  std::chrono::steady_clock::time_point t0;
  std::string err;
  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

hipStream_t group_stream(skx_engine *e, const Group &g) {
  return &g == &e->group[1] ? e->stream32 : e->stream;
}

int eng_fail(skx_engine *e, int code, const std::string &m) {
  e->err = m;
  return code;
}

bool valid_size(int n) {
  if (n < 8 || n > 512 || (n & 1)) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

size_t footprint(const skx_request &r) {
  const int m = std::min(std::max(r.opt.lbfgs_m, 1), MMAX);
  const long long M = (long long)r.n1 * r.n2 * r.n3;
  size_t b = 8 * (size_t)M;                          // finished density
  if (r.fn.precision != SKX_FP32)
    b += instance_bytes(r.n1, r.n2, r.n3, 0, m, r.fn.precision != SKX_MIXED);
  if (r.fn.precision != SKX_FP64) b += instance_bytes(r.n1, r.n2, r.n3, 1, m, true);
  const int n = std::max(r.n1, std::max(r.n2, r.n3));
  b += 16 * (size_t)(3 * (n / 2) * (n / 2) + 1);     // kernel tables
  return b;
}

int upload_state(skx_engine *e, Instance &I, const skx_opt_params &p, double gtol) {
  OptState st;
  init_state(st, p, gtol, 0, I.prec);
  hipError_t he = hipMemcpyAsync(I.st, &st, sizeof(OptState), hipMemcpyHostToDevice, e->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(e->stream);
  if (he != hipSuccess) return eng_fail(e, SKX_E_DEVICE, std::string("state upload: ") + hipGetErrorString(he));
  return SKX_OK;
}

double phase_gtol(const Resident &r) {
  if (r.mode == SKX_MIXED && r.prec == 1) {
    const double sw = r.opt.fp32_switch_gtol > 0 ? r.opt.fp32_switch_gtol : 1e-5;
    return std::max(sw, r.opt.gtol);
  }
  return r.opt.gtol;
}

// Set up one queued request as a resident solve (context, tables, V_loc,
// uniform start) on the engine stream.
int admit(skx_engine *e, Queued &q, int pooled_idx, Resident *&out) {
  const skx_request &r = q.req;
  skx_ctx *c = nullptr;
  int rc = SKX_OK;
  size_t bytes = q.bytes;
  if (pooled_idx >= 0) {
    // a reused context keeps its arenas, which may be larger than this
    // request needs (a longer history): charge what is allocated
    c = e->pool[pooled_idx].ctx;
    bytes = std::max(bytes, e->pool[pooled_idx].bytes + 8 * (size_t)r.n1 * r.n2 * r.n3);
    e->pooled -= e->pool[pooled_idx].bytes;
    e->pool.erase(e->pool.begin() + pooled_idx);
  } else {
    rc = skx_create(&c, e->device, (void *)e->stream);
    if (rc) return eng_fail(e, rc, "context creation failed");
  }
  auto bad = [&](int code) {
    std::string m = "request " + std::to_string(q.ticket) + ": " + c->err;
    skx_destroy(c);
    return eng_fail(e, code, m);
  };
  rc = skx_set_cell(c, r.lattice, r.n1, r.n2, r.n3);
  if (!rc) rc = skx_set_ions(c, r.nions, r.pos, r.species, r.nspecies, r.zval, r.rc);
  if (!rc) rc = skx_set_functional(c, &r.fn);
  if (rc) return bad(rc);
  const int mode = c->fn.precision;
  const int m = std::min(std::max(r.opt.lbfgs_m, 1), MMAX);
  if (mode != SKX_FP32 && (rc = prepare(c, 0, m))) return bad(rc);
  if (mode != SKX_FP64 && (rc = prepare(c, 1, m))) return bad(rc);
  Resident *s = new Resident();
  s->ticket = q.ticket;
  s->ctx = c;
  s->mode = mode;
  s->prec = mode == SKX_FP64 ? 0 : 1;
  s->opt = r.opt;
  s->t_arrival = r.t_arrival;
  s->t_admit = e->now();
  s->bytes = bytes;
  Instance &I = c->inst[s->prec];
  hipError_t he = start_uniform(c, I, e->stream);
  if (he != hipSuccess) { delete s; return bad(SKX_E_DEVICE); }
  rc = upload_state(e, I, s->opt, phase_gtol(*s));
  if (rc) { skx_destroy(c); delete s; return rc; }
  out = s;
  return SKX_OK;
}

hipError_t group_step(skx_engine *e, Group &g) {
  hipStream_t s = group_stream(e, g);
  hipError_t he = launch_normalize(g.bl, s);
  for (int k = 0; k < ENGINE_CHUNK && he == hipSuccess; ++k) he = step_sequence(g.bl, s);
  if (he == hipSuccess) he = gather_phases(g.ddev, (int)g.members.size(), g.dphase, s);
  return he;
}

// Capture group_step into a graph (left without one if capture is refused).
void capture_group(skx_engine *e, Group &g) {
  if (!graphs_enabled() || g.members.empty()) return;
  hipStream_t s = group_stream(e, g);
  if (hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  const hipError_t ec = group_step(e, g);
  hipError_t ee = hipStreamEndCapture(s, &g.graph);
  if (ec == hipSuccess && ee == hipSuccess) ee = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
  if (ec != hipSuccess || ee != hipSuccess) {
    g.drop_graph();
    (void)hipGetLastError();
  }
}

int rebuild(skx_engine *e, Group &g, int prec) {
  const int n = (int)g.members.size();
  g.dirty = false;
  g.drop_graph();
  if (n == 0) return SKX_OK;
  // set-up work of newly admitted or promoted members is on e->stream
  (void)hipStreamSynchronize(e->stream);
  (void)hipStreamSynchronize(group_stream(e, g));
  if (n > g.cap) {
    if (g.ddev) hipFree(g.ddev);
    if (g.dfirst) hipFree(g.dfirst);
    if (g.dphase) hipFree(g.dphase);
    g.ddev = nullptr; g.dfirst = nullptr; g.dphase = nullptr; g.cap = 0;
    const int cap = std::max(n, 2 * g.cap + 8);
    hipError_t he = hipMalloc((void **)&g.ddev, sizeof(SolveDev) * batch_desc_count(cap));
    if (he == hipSuccess) he = hipMalloc((void **)&g.dfirst, sizeof(int) * batch_first_count(cap));
    if (he == hipSuccess) he = hipMalloc((void **)&g.dphase, sizeof(int) * cap);
    if (he != hipSuccess) return eng_fail(e, SKX_E_NOMEM, "batch descriptor allocation");
    g.cap = cap;
  }
  std::vector<SolveDev> hs;
  hs.reserve(n);
  for (Resident *r : g.members) hs.push_back(r->ctx->inst[prec].h);
  int rc = build_batch(g.members[0]->ctx, hs, prec, g.ddev, g.dfirst, g.bl, e->stream);
  if (rc) return eng_fail(e, rc, g.members[0]->ctx->err);
  // build_batch reads hs from pageable memory: finish before hs goes away
  // (and before the group's own stream uses the descriptors)
  (void)hipStreamSynchronize(e->stream);
  capture_group(e, g);
  return SKX_OK;
}

void finish(skx_engine *e, Resident *r, const OptState &o) {
  Finished f{};
  f.res.ticket = r->ticket;
  skx_ctx *c = r->ctx;
  Instance &I = c->inst[r->prec];
  energy_from(o.e_acc, c->e_ii, &f.res.r.e);
  f.res.r.gnorm = o.rnorm;
  f.res.r.resets = o.resets;
  if (r->had_fp32) {
    f.res.r.fp32_iters = r->o32.iters;
    f.res.r.fp32_evals = r->o32.evals;
    f.res.r.iters = r->o32.iters + o.iters;
    f.res.r.evals = r->o32.evals + o.evals;
  } else {
    f.res.r.iters = o.iters;
    f.res.r.evals = o.evals;
    if (r->prec == 1) { f.res.r.fp32_iters = o.iters; f.res.r.fp32_evals = o.evals; }
  }
  if (o.phase == PH_FAILED && o.status < 0) f.res.r.status = o.status;
  else f.res.r.status = (o.phase == PH_DONE && o.status == 0) ? SKX_OK : SKX_NOT_CONVERGED;
  f.res.npoints = I.h.M;
  f.res.t_admit = r->t_admit;
  if (hipMallocAsync((void **)&f.rho_dev, sizeof(double) * I.h.M, e->stream) == hipSuccess) {
    square_out(I, o.par, f.rho_dev, e->stream);
    e->held += sizeof(double) * (size_t)I.h.M;
  } else {
    f.rho_dev = nullptr;
  }
  (void)hipStreamSynchronize(e->stream);
  f.res.t_done = e->now();
  // the resident's bytes include its finished density, now counted in held
  const size_t arena = r->bytes - std::min(r->bytes, sizeof(double) * (size_t)I.h.M);
  if ((int)e->pool.size() < e->max_slots) {
    // the history length the arenas were allocated for
    int m = 1;
    for (const Instance &J : c->inst)
      if (J.mem) m = std::max(m, J.m_alloc);
    e->pool.push_back({c, c->n1, c->n2, c->n3, r->mode, m, r->bytes});
    e->pooled += arena;
    e->pool.back().bytes = arena;
  } else {
    skx_destroy(c);
  }
  e->used -= std::min(e->used, r->bytes);
  e->done.push_back(f);
  delete r;
}

}  // namespace

extern "C" {

int skx_engine_create(skx_engine **out, int device, size_t hbm_budget_bytes, int max_slots) {
  if (!out) return SKX_E_INVALID;
  *out = nullptr;
  if (max_slots < 1 || hbm_budget_bytes == 0) return SKX_E_INVALID;
  if (hipSetDevice(device) != hipSuccess) return SKX_E_DEVICE;
  skx_engine *e = new skx_engine();
  e->device = device;
  e->budget = hbm_budget_bytes;
  e->max_slots = max_slots;
  if (hipStreamCreateWithFlags(&e->stream, hipStreamNonBlocking) != hipSuccess) {
    delete e;
    return SKX_E_DEVICE;
  }
  if (hipStreamCreateWithFlags(&e->stream32, hipStreamNonBlocking) != hipSuccess) {
    (void)hipStreamDestroy(e->stream);
    delete e;
    return SKX_E_DEVICE;
  }
  e->t0 = std::chrono::steady_clock::now();
  *out = e;
  return SKX_OK;
}

double skx_engine_clock(const skx_engine *e) { return e ? e->now() : 0.0; }

const char *skx_engine_last_error(const skx_engine *e) { return e ? e->err.c_str() : "null engine"; }

int skx_engine_submit(skx_engine *e, const skx_request *req, uint64_t *ticket) {
  if (!e || !req || !ticket) return SKX_E_INVALID;
  const skx_request &r = *req;
  if (!valid_size(r.n1) || !valid_size(r.n2) || !valid_size(r.n3))
    return eng_fail(e, SKX_E_INVALID, "grid sizes must be even and 5-smooth in 8..512");
  if (r.nions < 1 || r.nspecies < 1 || !r.pos || !r.species || !r.zval || !r.rc)
    return eng_fail(e, SKX_E_INVALID, "ions, species, zval and rc are required");
  if (r.opt.lbfgs_m < 1 || r.opt.lbfgs_m > MMAX || !(r.opt.gtol > 0) || r.opt.max_iter < 1)
    return eng_fail(e, SKX_E_INVALID, "bad optimiser parameters");
  if (r.fn.precision < SKX_FP64 || r.fn.precision > SKX_MIXED)
    return eng_fail(e, SKX_E_INVALID, "bad precision mode");
  Queued q;
  q.ticket = e->next_ticket++;
  q.req = r;
  q.pos.assign(r.pos, r.pos + 3 * (size_t)r.nions);
  q.species.assign(r.species, r.species + r.nions);
  q.zval.assign(r.zval, r.zval + r.nspecies);
  q.rc.assign(r.rc, r.rc + r.nspecies);
  q.bytes = footprint(r);
  if (q.bytes > e->budget) return eng_fail(e, SKX_E_INVALID, "request exceeds the HBM budget");
  e->queue.push_back(std::move(q));
  Queued &b = e->queue.back();
  b.req.pos = b.pos.data();
  b.req.species = b.species.data();
  b.req.zval = b.zval.data();
  b.req.rc = b.rc.data();
  *ticket = b.ticket;
  return SKX_OK;
}

int skx_engine_step(skx_engine *e) {
  if (!e) return SKX_E_INVALID;
  (void)hipSetDevice(e->device);
  // admission in arrival order; a pooled context of the same grid, mode
  // and history length is reused, others are freed when the budget needs
  // their memory
  while (!e->queue.empty() && (int)e->resident.size() < e->max_slots) {
    const Queued &qf = e->queue.front();
    const int m = std::min(std::max(qf.req.opt.lbfgs_m, 1), MMAX);
    int mi = -1;
    for (size_t i = 0; i < e->pool.size() && mi < 0; ++i) {
      const skx_engine::Pooled &p = e->pool[i];
      if (p.n1 == qf.req.n1 && p.n2 == qf.req.n2 && p.n3 == qf.req.n3 &&
          p.mode == qf.req.fn.precision && p.m >= m)
        mi = (int)i;
    }
    // a reused context brings its arenas (counted in pooled) and needs only
    // the result density beyond them
    const size_t reuse = mi >= 0 ? e->pool[mi].bytes : 0;
    const size_t need = std::max(qf.bytes, reuse + 8 * (size_t)qf.req.n1 * qf.req.n2 * qf.req.n3);
    while (e->used + e->held + e->pooled - reuse + need > e->budget) {
      int victim = -1;
      for (size_t i = 0; i < e->pool.size() && victim < 0; ++i)
        if ((int)i != mi) victim = (int)i;
      if (victim < 0) break;
      skx_destroy(e->pool[victim].ctx);
      e->pooled -= e->pool[victim].bytes;
      e->pool.erase(e->pool.begin() + victim);
      if (mi > victim) --mi;
    }
    if (e->used + e->held + e->pooled - reuse + need > e->budget) break;
    Queued q = std::move(e->queue.front());
    e->queue.pop_front();
    q.req.pos = q.pos.data();
    q.req.species = q.species.data();
    q.req.zval = q.zval.data();
    q.req.rc = q.rc.data();
    Resident *r = nullptr;
    int rc = admit(e, q, mi, r);
    if (rc) {
      // the request fails alone: report it as a finished result
      Finished f{};
      f.res.ticket = q.ticket;
      f.res.r.status = rc;
      f.res.t_admit = f.res.t_done = e->now();
      e->done.push_back(f);
      continue;
    }
    e->used += r->bytes;
    e->resident.push_back(r);
    e->group[r->prec].members.push_back(r);
    e->group[r->prec].dirty = true;
  }
  // one fused chunk of step sequences per precision group
  for (int p = 0; p < 2; ++p) {
    Group &g = e->group[p];
    if (g.dirty) {
      int rc = rebuild(e, g, p);
      if (rc) return rc;
    }
    if (g.members.empty()) continue;
    // replay the captured step while the membership and the graph switch
    // hold; launch eagerly otherwise
    if (g.exec && !graphs_enabled()) g.drop_graph();
    hipError_t he = g.exec ? hipGraphLaunch(g.exec, group_stream(e, g)) : group_step(e, g);
    if (he != hipSuccess) return eng_fail(e, SKX_E_DEVICE, std::string("step kernels: ") + hipGetErrorString(he));
  }
  // collect phases, retire or promote finished solves
  for (int p = 0; p < 2; ++p) {
    Group &g = e->group[p];
    const int n = (int)g.members.size();
    if (n == 0) continue;
    std::vector<int> ph(n);
    hipStream_t gs = group_stream(e, g);
    hipError_t he = hipMemcpyAsync(ph.data(), g.dphase, sizeof(int) * n, hipMemcpyDeviceToHost, gs);
    if (he == hipSuccess) he = hipStreamSynchronize(gs);
    if (he != hipSuccess) return eng_fail(e, SKX_E_DEVICE, std::string("step execution: ") + hipGetErrorString(he));
    std::vector<Resident *> keep;
    for (int i = 0; i < n; ++i) {
      Resident *r = g.members[i];
      if (ph[i] != PH_DONE && ph[i] != PH_FAILED) { keep.push_back(r); continue; }
      g.dirty = true;
      OptState o;
      Instance &I = r->ctx->inst[r->prec];
      (void)hipMemcpyAsync(&o, I.st, sizeof(OptState), hipMemcpyDeviceToHost, e->stream);
      (void)hipStreamSynchronize(e->stream);
      const bool promote = r->mode == SKX_MIXED && r->prec == 1 &&
                           !(o.phase == PH_FAILED && o.status < 0);
      if (promote) {
        r->o32 = o;
        r->had_fp32 = true;
        Instance &I64 = r->ctx->inst[0];
        promote_phi(I, o.par, I64, e->stream);
        r->prec = 0;
        if (upload_state(e, I64, r->opt, r->opt.gtol)) {
          e->resident.erase(std::find(e->resident.begin(), e->resident.end(), r));
          finish(e, r, o);
          continue;
        }
        e->group[0].members.push_back(r);
        e->group[0].dirty = true;
        continue;
      }
      e->resident.erase(std::find(e->resident.begin(), e->resident.end(), r));
      finish(e, r, o);
    }
    g.members.swap(keep);
  }
  return (int)e->resident.size();
}

int skx_engine_poll(skx_engine *e, skx_result *out, double **rho_host, int max, int *n_out) {
  if (!e || !n_out || (max > 0 && !out)) return SKX_E_INVALID;
  (void)hipSetDevice(e->device);
  int k = 0;
  while (k < max && !e->done.empty()) {
    Finished f = e->done.front();
    e->done.pop_front();
    out[k] = f.res;
    if (f.rho_dev) {
      if (rho_host && rho_host[k])
        hipMemcpy(rho_host[k], f.rho_dev, sizeof(double) * f.res.npoints, hipMemcpyDeviceToHost);
      (void)hipFreeAsync(f.rho_dev, e->stream);
      e->held -= std::min(e->held, sizeof(double) * (size_t)f.res.npoints);
    }
    ++k;
  }
  *n_out = k;
  return SKX_OK;
}

int skx_engine_cancel(skx_engine *e, uint64_t ticket) {
  if (!e) return SKX_E_INVALID;
  (void)hipSetDevice(e->device);
  Finished f{};
  f.res.ticket = ticket;
  f.res.r.status = SKX_CANCELLED;
  for (auto it = e->queue.begin(); it != e->queue.end(); ++it) {
    if (it->ticket != ticket) continue;
    f.res.t_admit = f.res.t_done = e->now();
    e->queue.erase(it);
    e->done.push_back(f);
    return SKX_OK;
  }
  for (auto it = e->resident.begin(); it != e->resident.end(); ++it) {
    Resident *r = *it;
    if (r->ticket != ticket) continue;
    // the steps end with both streams synchronised; set-up work of the
    // request may still be queued on the engine stream
    (void)hipStreamSynchronize(e->stream);
    (void)hipStreamSynchronize(e->stream32);
    for (Group &g : e->group) {
      auto m = std::find(g.members.begin(), g.members.end(), r);
      if (m != g.members.end()) {
        g.members.erase(m);
        g.dirty = true;
      }
    }
    e->resident.erase(it);
    f.res.t_admit = r->t_admit;
    f.res.t_done = e->now();
    skx_destroy(r->ctx);
    e->used -= std::min(e->used, r->bytes);
    delete r;
    e->done.push_back(f);
    return SKX_OK;
  }
  return eng_fail(e, SKX_E_INVALID, "no queued or resident request has this ticket");
}

int skx_engine_pending(const skx_engine *e) {
  if (!e) return 0;
  return (int)(e->queue.size() + e->resident.size() + e->done.size());
}

void skx_engine_destroy(skx_engine *e) {
  if (!e) return;
  (void)hipSetDevice(e->device);
  (void)hipStreamSynchronize(e->stream32);
  (void)hipStreamSynchronize(e->stream);
  for (Resident *r : e->resident) {
    skx_destroy(r->ctx);
    delete r;
  }
  for (Finished &f : e->done)
    if (f.rho_dev) hipFreeAsync(f.rho_dev, e->stream);
  for (skx_engine::Pooled &p : e->pool) skx_destroy(p.ctx);
  e->pool.clear();
  (void)hipStreamSynchronize(e->stream);
  for (Group &g : e->group) {
    g.drop_graph();
    if (g.ddev) hipFree(g.ddev);
    if (g.dfirst) hipFree(g.dfirst);
    if (g.dphase) hipFree(g.dphase);
  }
  hipStreamDestroy(e->stream32);
  (void)hipStreamDestroy(e->stream);
  delete e;
}

}  // extern "C"
