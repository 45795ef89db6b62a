// Serving: continuous batching of independent time-stepping requests.
#include "host_internal.h"

using namespace lemh;

// ============================================================== serving ====
// Continuous batching of independent time-stepping requests.  Each request
// is planned on admission (partition, decay-bound buffers, Krylov
// calibration) with all of its device memory taken from one pool of the
// configured size; every tick advances every active request by one step,
// with the blocks of all LEM requests in shared Krylov launches (one per
// launch shape).  Each block's arithmetic depends only on its own request,
// so results do not depend on what else is in the batch.
namespace {

struct ServerReq {
  uint64_t id = 0;
  int state = LEM_REQ_QUEUED;
  lem_operator op{};
  std::vector<double> nu_field;
  double dt = 0;
  int n_steps = 0, done = 0;
  std::vector<double> x0, result;
  lem_plan_s* plan = nullptr;
  double* buf[2] = {nullptr, nullptr};
  int method = LEM_METHOD_KRYLOV, core = 0, halo = 0;
  int64_t bytes = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  lem_status error = LEM_OK;
  int slot = -1;  // index of this request's status word while active
  int64_t N() const { return op.ndim == 1 ? (int64_t)op.n : (int64_t)op.n * op.n; }
};

}  // namespace

struct lem_server_s {
  lem_server_options opt{};
  hipStream_t st = nullptr;
  bool own_stream = false;
  // Requests served by the whole-grid global method are chains of small
  // dependent launches; independent requests run on side streams (default
  // priority) so that their chains overlap.
  static constexpr int kSide = 4;
  hipStream_t side[kSide] = {};
  hipEvent_t ev_fork = nullptr, ev_join[kSide] = {};
  char* pool = nullptr;
  lem::Arena* arena = nullptr;
  std::deque<uint64_t> queue;
  std::map<uint64_t, ServerReq> reqs;
  std::vector<uint64_t> active;
  uint64_t next = 1;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  lem::KBlock* d_table = nullptr;
  lem::KBlock* h_table = nullptr;
  double* d_diag = nullptr;
  lem::KronBlock* d_ktable = nullptr;  // Kronecker-factored blocks of every step of a tick
  lem::KronBlock* h_ktable = nullptr;
  size_t kcap = 0;
  // one status word per active request (slot), so that a failure latched by
  // one request's kernels is attributed to that request alone
  int* d_rstatus = nullptr;
  std::vector<int> h_rstatus, free_slots;
  size_t cap = 0;
  int64_t ticks = 0;
  double dof_steps = 0;
  int n_done = 0, n_failed = 0;
  int status_seen = 0;

  double now_ms() const {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  ~lem_server_s() {
    if (!opt.dry_run) hipStreamSynchronize(st);
    for (auto& kv : reqs) delete kv.second.plan;  // arena ranges die with the pool
    if (!opt.dry_run) {
      hipFree(pool);
      hipFree(d_table);
      hipFree(d_diag);
      hipFree(d_rstatus);
      hipFree(d_ktable);
      hipHostFree(h_table);
      hipHostFree(h_ktable);
      for (int k = 0; k < kSide; ++k) {
        if (side[k]) hipStreamDestroy(side[k]);
        if (ev_join[k]) hipEventDestroy(ev_join[k]);
      }
      if (ev_fork) hipEventDestroy(ev_fork);
      if (own_stream) hipStreamDestroy(st);
    }
    delete arena;
  }
};

namespace {

lem_status server_grow(lem_server_s* s, size_t blocks) {
  if (blocks <= s->cap) return LEM_OK;
  size_t cap = std::max<size_t>(blocks, 2 * s->cap);
  LEM_HIP(hipStreamSynchronize(s->st));
  hipFree(s->d_table);
  hipFree(s->d_diag);
  hipHostFree(s->h_table);
  s->d_table = nullptr; s->d_diag = nullptr; s->h_table = nullptr;
  LEM_HIP(hipMalloc(&s->d_table, cap * sizeof(lem::KBlock)));
  LEM_HIP(hipMalloc(&s->d_diag, cap * sizeof(double)));
  LEM_HIP(hipHostMalloc(&s->h_table, cap * sizeof(lem::KBlock), hipHostMallocDefault));
  s->cap = cap;
  return LEM_OK;
}

lem_status server_grow_k(lem_server_s* s, size_t blocks) {
  if (blocks <= s->kcap) return LEM_OK;
  size_t cap = std::max<size_t>(blocks, 2 * s->kcap);
  LEM_HIP(hipStreamSynchronize(s->st));
  hipFree(s->d_ktable);
  hipHostFree(s->h_ktable);
  s->d_ktable = nullptr; s->h_ktable = nullptr;
  LEM_HIP(hipMalloc(&s->d_ktable, cap * sizeof(lem::KronBlock)));
  LEM_HIP(hipHostMalloc(&s->h_ktable, cap * sizeof(lem::KronBlock), hipHostMallocDefault));
  s->kcap = cap;
  return LEM_OK;
}

// Partition choice for one request: core side c in {16, 32, 64} (dividing n)
// with the fewest local points per core point, under the box limits of the
// Krylov kernel; the global method when no core qualifies or the overhead is
// above opt.max_overhead.
void choose_partition(const lem_server_s* s, ServerReq& r, const Op& op) {
  const double G = growth_factor(op);
  bool clamped = false;
  Box b0{0, 0, 16, op.ndim == 2 ? 16 : 1, 0};
  const int h = halo_from_bound(op, b0, s->opt.halo_tol, s->opt.halo_min, s->opt.halo_max, G,
                                &clamped);
  r.method = LEM_METHOD_GLOBAL;
  r.core = 0;
  r.halo = 0;
  if (clamped) return;
  if (op.ndim == 2 && !op.variable) {
    // constant coefficients: Kronecker-factored local exponentials; per core
    // point a box costs 2 L (L + c) / c flops and (L / c)^2 gathered values
    double best = INFINITY;
    for (int c : {16, 32, 64}) {
      const int L = c + 2 * h;
      if (op.n % c || L >= op.n || L > lem::kron_max_side()) continue;
      const double cost = (double)L * (L + c) / c + 8.0 * ((double)L / c) * ((double)L / c);
      if (cost < best) { best = cost; r.core = c; }
    }
    if (r.core) {
      r.method = LEM_METHOD_KRONECKER;
      r.halo = h;
      return;
    }
  }
  double best = INFINITY;
  for (int c : {16, 32, 64}) {
    if (op.n % c || c + 2 * h >= op.n) continue;
    const int L = c + 2 * h;
    const int64_t nloc = op.ndim == 2 ? (int64_t)L * L : L;
    if (nloc > lem::krylov_big_max_n()) continue;
    const double ov = op.ndim == 2 ? (double)L * L / ((double)c * c) : (double)L / c;
    if (ov < best) { best = ov; r.core = c; }
  }
  if (r.core && best <= s->opt.max_overhead) {
    r.method = LEM_METHOD_KRYLOV;
    r.halo = h;
  } else {
    r.core = 0;
  }
}

void server_release(lem_server_s* s, ServerReq& r);

// Admission of the queue head; LEM_ERR_BUDGET leaves it queued.
lem_status server_admit(lem_server_s* s, ServerReq& r) {
  Op op;
  LEM_TRY(build_op(&r.op, r.dt, &op));
  choose_partition(s, r, op);
  lem_options o;
  lem_options_default(&o);
  o.method = r.method;
  o.n_states = 1;
  o.core = r.core;
  o.halo = r.halo;
  o.krylov_tol = s->opt.krylov_tol;
  o.krylov_m_max = s->opt.krylov_m_max;
  o.max_substeps = s->opt.max_substeps;
  o.dry_run = s->opt.dry_run;
  // a global step is a long chain of small launches: replay it from a graph
  o.use_graph = r.method == LEM_METHOD_GLOBAL ? 1 : 0;
  // the 1D exponentials of a Kronecker-factored request by GEMMs only (no
  // latency-bound pivoting chain in the admission path)
  o.expm = LEM_EXPM_TAYLOR;
  const size_t before = s->arena->in_use();
  lem_plan_t p = nullptr;
  LEM_TRY(create_plan(&r.op, r.dt, &o, s->st, s->arena, &p));
  const int64_t N = r.N();
  for (int q = 0; q < 2; ++q) {
    r.buf[q] = (double*)s->arena->alloc(N * sizeof(double));
    if (!r.buf[q]) {
      s->arena->release(r.buf[0]);
      r.buf[0] = r.buf[1] = nullptr;
      delete p;
      return fail(LEM_ERR_BUDGET, "memory budget exhausted");
    }
  }
  if (!s->opt.dry_run) {
    hipError_t e = hipMemcpyAsync(r.buf[0], r.x0.data(), N * sizeof(double),
                                  hipMemcpyHostToDevice, s->st);
    if (e != hipSuccess) {
      s->arena->release(r.buf[0]);
      s->arena->release(r.buf[1]);
      r.buf[0] = r.buf[1] = nullptr;
      delete p;
      return fail(LEM_ERR_HIP, "state upload failed");
    }
  }
  r.plan = p;
  r.bytes = (int64_t)(s->arena->in_use() - before);
  r.state = LEM_REQ_ACTIVE;
  r.t_admit = s->now_ms();
  if (!s->opt.dry_run) {
    // the request's kernels latch into its own slot (the global method's
    // graph, captured at its first step, takes this pointer)
    r.slot = s->free_slots.back();
    s->free_slots.pop_back();
    p->d_status = s->d_rstatus + r.slot;
    p->gw.status = p->d_status;
    if (hipMemsetAsync(p->d_status, 0, sizeof(int), s->st) != hipSuccess) {
      server_release(s, r);
      return fail(LEM_ERR_HIP, "status reset failed");
    }
  }
  return LEM_OK;
}

void server_release(lem_server_s* s, ServerReq& r) {
  if (r.slot >= 0) s->free_slots.push_back(r.slot);
  r.slot = -1;
  delete r.plan;  // returns its ranges to the arena
  r.plan = nullptr;
  s->arena->release(r.buf[0]);
  s->arena->release(r.buf[1]);
  r.buf[0] = r.buf[1] = nullptr;
}

}  // namespace

extern "C" {

void lem_server_options_default(lem_server_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->hbm_budget = (size_t)8 << 30;
  o->max_active = 256;
  o->halo_tol = 1e-8;
  o->halo_min = 4;
  o->halo_max = 56;
  o->max_overhead = 4.0;
  o->krylov_tol = 1e-12;
  o->krylov_m_max = 30;
  o->max_substeps = 64;
  o->dry_run = 0;
  o->steps_per_tick = 1;
}

lem_status lem_server_create(const lem_server_options* opt, void* stream, lem_server_t* out) {
  if (!opt || !out) return fail(LEM_ERR_INVALID, "NULL argument");
  *out = nullptr;
  if (opt->hbm_budget < 4096 || opt->max_active < 1 || !(opt->halo_tol > 0) ||
      opt->halo_min < 0 || opt->halo_max < opt->halo_min || !(opt->max_overhead >= 1) ||
      !(opt->krylov_tol > 0) || opt->krylov_m_max < 2 ||
      opt->krylov_m_max > lem::krylov_big_max_m() ||
      opt->max_substeps < 1 || opt->steps_per_tick < 1)
    return fail(LEM_ERR_INVALID, "invalid server options");
  auto s = new lem_server_s();
  s->opt = *opt;
  s->st = (hipStream_t)stream;
  if (!opt->dry_run && s->st == nullptr) {
    // a stream of its own (default priority) so that steps can be replayed
    // from captured graphs, which the legacy null stream does not allow
    if (hipStreamCreateWithFlags(&s->st, hipStreamNonBlocking) != hipSuccess) {
      delete s;
      return fail(LEM_ERR_HIP, "could not create the serving stream");
    }
    s->own_stream = true;
  }
  if (opt->dry_run) {
    s->arena = new lem::Arena((char*)(uintptr_t)4096, opt->hbm_budget);
  } else {
    if (hipMalloc(&s->pool, opt->hbm_budget) != hipSuccess) {
      hipGetLastError();
      delete s;
      return fail(LEM_ERR_NOMEM, "could not reserve the serving pool");
    }
    s->arena = new lem::Arena(s->pool, opt->hbm_budget);
    bool ok = hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming) == hipSuccess;
    for (int k = 0; ok && k < lem_server_s::kSide; ++k)
      ok = hipStreamCreateWithFlags(&s->side[k], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&s->ev_join[k], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      delete s;
      return fail(LEM_ERR_HIP, "could not create the serving side streams");
    }
    if (hipMalloc(&s->d_rstatus, sizeof(int) * opt->max_active) != hipSuccess ||
        hipMemsetAsync(s->d_rstatus, 0, sizeof(int) * opt->max_active, s->st) != hipSuccess ||
        server_grow(s, 4096) != LEM_OK) {
      delete s;
      return fail(LEM_ERR_NOMEM, "could not allocate serving tables");
    }
    s->h_rstatus.assign(opt->max_active, 0);
    for (int k = opt->max_active - 1; k >= 0; --k) s->free_slots.push_back(k);
  }
  *out = s;
  return LEM_OK;
}

lem_status lem_server_submit(lem_server_t s, const lem_operator* op, double dt, int32_t n_steps,
                             const double* x0_host, uint64_t* id) {
  if (!s || !op || !x0_host || !id) return fail(LEM_ERR_INVALID, "NULL argument");
  if (n_steps < 1) return fail(LEM_ERR_INVALID, "n_steps must be >= 1");
  if (op->forcing) return fail(LEM_ERR_UNSUPPORTED, "served requests take no forcing");
  if (op->vel_faces) return fail(LEM_ERR_UNSUPPORTED, "served requests take no face velocities");
  Op chk;
  LEM_TRY(build_op(op, dt, &chk));
  ServerReq r;
  r.id = s->next++;
  r.op = *op;
  r.dt = dt;
  r.n_steps = n_steps;
  const int64_t N = r.N();
  if ((size_t)(2 * N * sizeof(double)) > s->opt.hbm_budget)
    return fail(LEM_ERR_BUDGET, "request state alone exceeds the memory budget");
  if (op->nu_field) {
    r.nu_field.assign(op->nu_field, op->nu_field + N);
    r.op.nu_field = r.nu_field.data();
  }
  r.x0.assign(x0_host, x0_host + N);
  r.t_submit = s->now_ms();
  *id = r.id;
  auto it = s->reqs.emplace(r.id, std::move(r)).first;
  if (!it->second.nu_field.empty()) it->second.op.nu_field = it->second.nu_field.data();
  s->queue.push_back(*id);
  return LEM_OK;
}

lem_status lem_server_tick(lem_server_t s, int32_t* n_active, int32_t* n_queued) {
  if (!s) return fail(LEM_ERR_INVALID, "server is NULL");
  // 1. admission, first come first served
  while (!s->queue.empty() && (int)s->active.size() < s->opt.max_active) {
    ServerReq& r = s->reqs[s->queue.front()];
    lem_status st = server_admit(s, r);
    if (st == LEM_ERR_BUDGET) {
      if (s->active.empty()) {  // cannot fit even alone: fail it
        r.state = LEM_REQ_FAILED;
        r.error = st;
        s->n_failed++;
        s->queue.pop_front();
        continue;
      }
      break;
    }
    s->queue.pop_front();
    if (st != LEM_OK) {
      r.state = LEM_REQ_FAILED;
      r.error = st;
      s->n_failed++;
      continue;
    }
    s->active.push_back(r.id);
  }
  // 2. steps_per_tick steps of every active request (at most the steps it
  // has left).  Whole-grid global requests run their steps on side streams;
  // the blocks of all LEM requests go into one shared launch per shape and
  // step, the tables of every step uploaded at once.
  std::vector<int> take(s->active.size(), 0);
  for (size_t a = 0; a < s->active.size(); ++a) {
    const ServerReq& r = s->reqs[s->active[a]];
    take[a] = std::min(s->opt.steps_per_tick, r.n_steps - r.done);
  }
  if (!s->opt.dry_run && !s->active.empty()) {
    int kmax = 0;
    size_t need = 0;
    for (size_t a = 0; a < s->active.size(); ++a) {
      kmax = std::max(kmax, take[a]);
      need += (size_t)take[a] * s->reqs[s->active[a]].plan->kb_host.size();
    }
    LEM_TRY(server_grow(s, std::max<size_t>(need, 1)));
    int n_side = 0;
    LEM_HIP(hipEventRecord(s->ev_fork, s->st));  // states uploaded at admission
    for (size_t a = 0; a < s->active.size(); ++a) {
      ServerReq& r = s->reqs[s->active[a]];
      if (!r.plan->kb_host.empty() || r.method == LEM_METHOD_KRONECKER) continue;
      // whole-grid Krylov launches of its own
      hipStream_t ss = s->side[n_side % lem_server_s::kSide];
      if (n_side < lem_server_s::kSide) LEM_HIP(hipStreamWaitEvent(ss, s->ev_fork, 0));
      ++n_side;
      for (int k = 0; k < take[a]; ++k)
        LEM_TRY(run_step(r.plan, r.buf[(r.done + k) & 1], r.buf[(r.done + k + 1) & 1], ss));
    }
    struct Launch { LaunchKey key; size_t lds, off; int count; };
    std::vector<Launch> launches;
    size_t off = 0;
    int diag = 0;
    for (int k = 0; k < kmax; ++k) {
      std::map<LaunchKey, std::vector<lem::KBlock>> groups;
      std::map<LaunchKey, size_t> lds;
      for (size_t a = 0; a < s->active.size(); ++a) {
        ServerReq& r = s->reqs[s->active[a]];
        if (take[a] <= k || r.plan->kb_host.empty()) continue;
        const lem_plan_s* p = r.plan;
        for (const auto& bk : p->buckets)
          for (int i = bk.first; i < bk.first + bk.count; ++i) {
            lem::KBlock kb = p->kb_host[i];
            kb.xin = r.buf[(r.done + k) & 1];
            kb.xout = r.buf[(r.done + k + 1) & 1];
            kb.coef = p->d_coef;
            kb.vwork = p->d_vwork + kb.v_off;
            kb.status = s->d_rstatus + r.slot;
            kb.diag = diag++;
            const LaunchKey key{bk.variant, bk.nt, bk.pmax, bk.vlds};
            groups[key].push_back(kb);
            lds[key] = std::max(lds[key], bk.lds);
          }
      }
      for (auto& g : groups) {
        // costliest blocks first (as in a plan's own launches)
        std::stable_sort(g.second.begin(), g.second.end(),
                         [](const lem::KBlock& x, const lem::KBlock& y) {
                           return block_cost(x.ndim, x.Lx * x.Ly + x.aug, x.m, x.nsub) >
                                  block_cost(y.ndim, y.Lx * y.Ly + y.aug, y.m, y.nsub);
                         });
        std::memcpy(s->h_table + off, g.second.data(), g.second.size() * sizeof(lem::KBlock));
        launches.push_back({g.first, lds[g.first], off, (int)g.second.size()});
        off += g.second.size();
      }
    }
    if (off) LEM_HIP(hipMemcpyAsync(s->d_table, s->h_table, off * sizeof(lem::KBlock),
                                    hipMemcpyHostToDevice, s->st));
    // Kronecker-factored requests: every block of every such request in one
    // launch per step (blocks carry their request's pointers)
    size_t kneed = 0;
    for (size_t a = 0; a < s->active.size(); ++a) {
      const ServerReq& r = s->reqs[s->active[a]];
      if (r.method == LEM_METHOD_KRONECKER) kneed += (size_t)take[a] * r.plan->boxes.size();
    }
    std::vector<std::pair<size_t, int>> klaunch;  // (offset, count) per step
    std::vector<int> kmaxL, kmaxC;
    if (kneed) {
      LEM_TRY(server_grow_k(s, kneed));
      size_t koff = 0;
      for (int k = 0; k < kmax; ++k) {
        const size_t k0 = koff;
        int maxL = 0, maxC = 0;
        for (size_t a = 0; a < s->active.size(); ++a) {
          ServerReq& r = s->reqs[s->active[a]];
          if (take[a] <= k || r.method != LEM_METHOD_KRONECKER) continue;
          const lem_plan_s* p = r.plan;
          const int c = p->boxes[0].cx, L = p->kron_L;
          maxL = std::max(maxL, L);
          maxC = std::max(maxC, c);
          for (const Box& b : p->boxes) {
            lem::KronBlock kb{};
            kb.ox = b.ox; kb.oy = b.oy; kb.c = c; kb.h = b.h; kb.L = L; kb.n = p->op.n; kb.ns = 1;
            kb.x_in = r.buf[(r.done + k) & 1];
            kb.x_out = r.buf[(r.done + k + 1) & 1];
            kb.ex = p->d_ex;
            kb.ey = p->d_ex + (size_t)c * L;
            kb.status = s->d_rstatus + r.slot;
            s->h_ktable[koff++] = kb;
          }
        }
        klaunch.push_back({k0, (int)(koff - k0)});
        kmaxL.push_back(maxL);
        kmaxC.push_back(maxC);
      }
      LEM_HIP(hipMemcpyAsync(s->d_ktable, s->h_ktable, koff * sizeof(lem::KronBlock),
                             hipMemcpyHostToDevice, s->st));
    }
    for (size_t k = 0; k < klaunch.size(); ++k) {
      if (!klaunch[k].second) continue;
      hipError_t e = lem::launch_kron(s->d_ktable + klaunch[k].first, klaunch[k].second, 1,
                                      kmaxL[k], kmaxC[k], nullptr, nullptr, s->d_rstatus, s->st);
      if (e != hipSuccess)
        return fail(LEM_ERR_HIP, std::string("serving launch: ") + hipGetErrorString(e));
    }
    // launches of step k + 1 follow those of step k on the serving stream
    for (const Launch& L : launches) {
      // every block carries its request's status word (the launch's own is unused)
      hipError_t e = launch_bucket(L.key.variant, s->d_table + L.off, L.count, 1, L.key.nt,
                                   L.key.pmax, L.key.vlds, L.lds, nullptr, nullptr, nullptr,
                                   nullptr, s->d_diag, s->d_rstatus, nullptr, 0, s->st);
      if (e != hipSuccess)
        return fail(LEM_ERR_HIP, std::string("serving launch: ") + hipGetErrorString(e));
    }
    // the retiring copies below (on the serving stream) follow the side streams
    for (int k = 0; k < std::min(n_side, lem_server_s::kSide); ++k) {
      LEM_HIP(hipEventRecord(s->ev_join[k], s->side[k]));
      LEM_HIP(hipStreamWaitEvent(s->st, s->ev_join[k], 0));
    }
  }
  // 3. advance counters, retire finished and failed requests
  std::vector<uint64_t> finished, still;
  for (size_t a = 0; a < s->active.size(); ++a) {
    ServerReq& r = s->reqs[s->active[a]];
    r.done += take[a];
    s->dof_steps += (double)r.N() * take[a];
    if (r.done == r.n_steps) finished.push_back(s->active[a]);
    else still.push_back(s->active[a]);
  }
  for (uint64_t id : finished) {
    ServerReq& r = s->reqs[id];
    r.result.resize(r.N());
    if (s->opt.dry_run) {
      r.result = r.x0;
    } else {
      LEM_HIP(hipMemcpyAsync(r.result.data(), r.buf[r.n_steps & 1], r.N() * sizeof(double),
                             hipMemcpyDeviceToHost, s->st));
    }
  }
  if (!s->opt.dry_run) {
    LEM_HIP(hipStreamSynchronize(s->st));
    LEM_HIP(hipMemcpy(s->h_rstatus.data(), s->d_rstatus, s->h_rstatus.size() * sizeof(int),
                      hipMemcpyDeviceToHost));
  }
  const double t = s->now_ms();
  // a request whose kernels latched a failure leaves the batch now
  auto failed_now = [&](ServerReq& r) {
    if (r.slot < 0) return false;
    const int bits = s->h_rstatus[r.slot];
    if (!bits) return false;
    s->status_seen |= bits;
    server_release(s, r);
    r.state = LEM_REQ_FAILED;
    r.error = (lem_status)device_status_of(bits);
    r.t_done = t;
    s->n_failed++;
    return true;
  };
  for (uint64_t id : finished) {
    ServerReq& r = s->reqs[id];
    if (failed_now(r)) continue;
    server_release(s, r);
    r.state = LEM_REQ_DONE;
    r.t_done = t;
    s->n_done++;
  }
  std::vector<uint64_t> kept;
  for (uint64_t id : still)
    if (!failed_now(s->reqs[id])) kept.push_back(id);
  s->active.swap(kept);
  s->ticks++;
  if (n_active) *n_active = (int32_t)s->active.size();
  if (n_queued) *n_queued = (int32_t)s->queue.size();
  return LEM_OK;
}

lem_status lem_server_poll(lem_server_t s, uint64_t id, int32_t* state) {
  if (!s || !state) return fail(LEM_ERR_INVALID, "NULL argument");
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return fail(LEM_ERR_NOT_FOUND, "unknown request id");
  *state = it->second.state;
  return LEM_OK;
}

lem_status lem_server_request_info(lem_server_t s, uint64_t id, lem_request_info* info) {
  if (!s || !info) return fail(LEM_ERR_INVALID, "NULL argument");
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return fail(LEM_ERR_NOT_FOUND, "unknown request id");
  const ServerReq& r = it->second;
  std::memset(info, 0, sizeof(*info));
  info->state = r.state;
  info->method = r.method;
  info->core = r.core;
  info->halo = r.halo;
  info->n_steps = r.n_steps;
  info->steps_done = r.done;
  info->bytes = r.bytes;
  info->t_submit_ms = r.t_submit;
  info->t_admit_ms = r.t_admit;
  info->t_done_ms = r.t_done;
  info->error = r.error;
  if (r.plan) {
    lem_plan_info pi;
    fill_info(r.plan, &pi);
    info->n_blocks = pi.n_blocks;
    info->m_max = pi.m_max;
    info->substeps_max = pi.substeps_max;
  }
  return LEM_OK;
}

lem_status lem_server_fetch(lem_server_t s, uint64_t id, double* x_host) {
  if (!s || !x_host) return fail(LEM_ERR_INVALID, "NULL argument");
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return fail(LEM_ERR_NOT_FOUND, "unknown request id");
  ServerReq& r = it->second;
  if (r.state == LEM_REQ_FAILED) {
    const lem_status e = r.error;
    s->reqs.erase(it);
    return fail(e, "request failed");
  }
  if (r.state != LEM_REQ_DONE) return fail(LEM_ERR_INVALID, "request is not finished");
  std::memcpy(x_host, r.result.data(), r.result.size() * sizeof(double));
  s->reqs.erase(it);
  return LEM_OK;
}

lem_status lem_server_query(lem_server_t s, lem_server_info* info) {
  if (!s || !info) return fail(LEM_ERR_INVALID, "NULL argument");
  std::memset(info, 0, sizeof(*info));
  info->n_queued = (int32_t)s->queue.size();
  info->n_active = (int32_t)s->active.size();
  info->n_done = s->n_done;
  info->n_failed = s->n_failed;
  info->ticks = s->ticks;
  info->bytes_in_use = (int64_t)s->arena->in_use();
  info->bytes_budget = (int64_t)s->opt.hbm_budget;
  info->dof_steps = s->dof_steps;
  info->device_status = device_status_of(s->status_seen);
  return LEM_OK;
}

lem_status lem_server_destroy(lem_server_t s) {
  delete s;
  return LEM_OK;
}

}  // extern "C"

