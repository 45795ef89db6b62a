// Plan life cycle: the global method, one step of any method (optionally
// replayed from a HIP graph), option checks, plan creation with the Krylov
// partition autotuner, and the plan calls of the C ABI.
#include "host_internal.h"

namespace lemh {

void dfree(lem_plan_s* p, void* ptr) {
  if (!ptr) return;
  auto it = std::find(p->allocs.begin(), p->allocs.end(), ptr);
  if (it != p->allocs.end()) p->allocs.erase(it);
  if (p->arena) p->arena->release(ptr);
  else hipFree(ptr);
}

lem_status upload(void* dst, const void* src, size_t bytes, hipStream_t st) {
  LEM_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
  return LEM_OK;
}

// --------------------------------------------------------------- global ----
lem_status alloc_global(lem_plan_s* p, int m, int ns, int nsub, lem::GlobalWork* w,
                        bool forced) {
  const Op& op = p->op;
  w->N = op.N();
  w->force = forced ? p->d_force : nullptr;
  w->gscale = op.dt / nsub;
  w->xa = w->ya = nullptr;
  w->ns = ns; w->n = op.n; w->ndim = op.ndim; w->m = m; w->nsub = nsub;
  const double sc = 1.0 / nsub;
  for (int q = 0; q < 5; ++q) w->w[q] = op.w[q] * sc;
  w->chx = op.chx * sc; w->chy = op.chy * sc; w->sub_scale = sc;
  w->mux = op.variable ? p->d_coef : nullptr;
  w->muy = op.variable ? p->d_coef + op.N() : nullptr;
  w->ax = op.varvel ? p->d_coef + 2 * op.N() : nullptr;
  w->ay = op.varvel ? p->d_coef + 3 * op.N() : nullptr;
  w->tol = p->opt.krylov_tol;
  w->status = p->d_status;
  const int64_t tot = (w->N + (forced ? 1 : 0)) * ns;  // plus the augmented coordinate
  const int G = lem::global_grid(tot, ns);
  const int K = lem::kMaxKrylov + 1;
  if (forced) {
    LEM_TRY(dalloc(p, &w->xa, (size_t)tot, &p->bytes_work));
    LEM_TRY(dalloc(p, &w->ya, (size_t)tot, &p->bytes_work));
  }
  LEM_TRY(dalloc(p, &w->V, (size_t)(m + 1) * tot, &p->bytes_work));
  LEM_TRY(dalloc(p, &w->W, (size_t)tot, &p->bytes_work));
  LEM_TRY(dalloc(p, &w->Wt, (size_t)tot, &p->bytes_work));
  LEM_TRY(dalloc(p, &w->part, lem::global_part_doubles(G, ns), &p->bytes_work));
  LEM_TRY(dalloc(p, &w->h1, (size_t)K * ns, &p->bytes_work));
  LEM_TRY(dalloc(p, &w->h2, (size_t)K * ns, &p->bytes_work));
  LEM_TRY(dalloc(p, &w->hn, (size_t)K * ns, &p->bytes_work));
  LEM_TRY(dalloc(p, &w->H, (size_t)ns * (m + 1) * m, &p->bytes_work));
  LEM_TRY(dalloc(p, &w->f, (size_t)ns * m, &p->bytes_work));
  LEM_TRY(dalloc(p, &w->beta, (size_t)ns, &p->bytes_work));
  LEM_TRY(dalloc(p, &w->inv, (size_t)ns, &p->bytes_work));
  LEM_TRY(dalloc(p, &w->est, (size_t)ns, &p->bytes_work));
  LEM_TRY(dalloc(p, &w->estsum, (size_t)ns, &p->bytes_work));
  LEM_HIP(hipMemsetAsync(w->estsum, 0, (size_t)ns * 8, p->stream));
  return LEM_OK;
}

void free_global(lem_plan_s* p, lem::GlobalWork* w) {
  for (void* q : {(void*)w->V, (void*)w->W, (void*)w->Wt, (void*)w->part, (void*)w->h1,
                  (void*)w->h2, (void*)w->hn, (void*)w->H, (void*)w->f, (void*)w->beta,
                  (void*)w->inv, (void*)w->est, (void*)w->estsum, (void*)w->xa, (void*)w->ya})
    if (q) dfree(p, q);
}

lem_status plan_global(lem_plan_s* p, hipStream_t st) {
  const Op& op = p->op;
  const lem_options& o = p->opt;
  if (256 % p->ns != 0)
    return fail(LEM_ERR_UNSUPPORTED, "the global method needs n_states dividing 256");
  if (op.variable) LEM_TRY(upload_coef(p, st));
  const int mcal = std::min(std::max(o.krylov_m_max, 4), lem::kMaxKrylov);
  std::vector<int> jl;
  for (int j = 2; j <= mcal; ++j) jl.push_back(j);
  int nsc = 1;
  while ((1 << nsc) <= o.max_substeps && nsc < 12) ++nsc;
  lem::GlobalWork cw{};
  const int64_t before = p->bytes_work;
  LEM_TRY(alloc_global(p, mcal, 1, 1, &cw));
  double *d_probe, *d_calib, *d_est;
  int *d_mcal, *d_jl;
  int64_t* d_coff;
  const int64_t cstride = 2 + (int64_t)(mcal + 1) * mcal;
  LEM_TRY(dalloc(p, &d_probe, (size_t)op.N()));
  LEM_TRY(dalloc(p, &d_calib, (size_t)cstride));
  LEM_TRY(dalloc(p, &d_est, (size_t)nsc * jl.size()));
  LEM_TRY(dalloc(p, &d_mcal, 1));
  LEM_TRY(dalloc(p, &d_jl, jl.size()));
  LEM_TRY(dalloc(p, &d_coff, 1));
  int64_t zero = 0;
  LEM_TRY(upload(d_mcal, &mcal, sizeof(int), st));
  LEM_TRY(upload(d_jl, jl.data(), jl.size() * sizeof(int), st));
  LEM_TRY(upload(d_coff, &zero, sizeof(int64_t), st));
  LEM_HIP(lem::launch_probe_fill(d_probe, op.N(), 777u, st));
  LEM_HIP(lem::global_arnoldi(cw, d_probe, d_calib, st));
  LEM_HIP(lem::launch_krylov_estimates(d_calib, d_mcal, d_coff, d_jl, (int)jl.size(), nsc, d_est,
                                       1, mcal, st));
  std::vector<double> est((size_t)nsc * jl.size());
  LEM_HIP(hipMemcpyAsync(est.data(), d_est, est.size() * 8, hipMemcpyDeviceToHost, st));
  LEM_HIP(hipStreamSynchronize(st));
  int mm = 0, ss = 0;
  const bool ok =
      choose_m(est.data(), jl, nsc, o.krylov_tol, o.krylov_m, mcal, op.ndim, 0, &mm, &ss);
  free_global(p, &cw);
  for (void* q : {(void*)d_probe, (void*)d_calib, (void*)d_est, (void*)d_mcal, (void*)d_jl,
                  (void*)d_coff})
    dfree(p, q);
  p->bytes_work = before;
  if (!ok)
    return fail(LEM_ERR_NOT_CONVERGED, "no global Krylov dimension/sub-step pair meets krylov_tol");
  p->m.assign(1, mm);
  p->nsub.assign(1, ss);
  LEM_TRY(alloc_global(p, mm, p->ns, ss, &p->gw, p->forced));
  return LEM_OK;
}

// ----------------------------------------------------------------- step ----
lem_status run_one(lem_plan_s* p, const double* src, double* dst, hipStream_t st) {
  if (p->method == LEM_METHOD_ROSENBROCK) return ere_run_one(p, src, dst, st);
  switch (p->global_box ? LEM_METHOD_KRYLOV : p->method) {
    case LEM_METHOD_KRYLOV:
      return launch_buckets(p, p->d_kb, p->buckets, p->ns, src, dst, p->d_vwork, p->d_diag,
                            nullptr, 0, st);
    case LEM_METHOD_DENSE: {
      const int64_t es = (int64_t)p->rows_p * p->cols_p;
      if (p->d_xp)
        LEM_HIP(lem::dense_split_pieces(src, p->N * p->ns, p->opt.precision == LEM_BF16X3 ? 3 : 2,
                                        p->d_xp, st));
      LEM_HIP(lem::dense_apply(p->opt.precision, p->tile, p->d_db, dense_operand(p), es, p->d_core,
                               src, dst, p->op.n, p->op.ndim, p->ns, p->rows, p->rows_p, p->cols,
                               p->cols_p, (int)p->boxes.size(), p->d_bias, p->d_status, st,
                               p->d_xp, p->N));
      return LEM_OK;
    }
    case LEM_METHOD_KRONECKER:
      LEM_HIP(lem::launch_kron(p->d_kron, (int)p->boxes.size(), p->ns, p->kron_L,
                               p->boxes[0].cx, src, dst, p->d_status, st));
      return LEM_OK;
    default:
      LEM_HIP(lem::global_step(p->gw, src, dst, st));
      return LEM_OK;
  }
}

// A 1D dense plan with one stored block on cores tiling the grid, small
// enough for two states per workgroup in LDS, steps in one launch per call.
bool resident_fits(const lem_plan_s* p) {
  if (p->method != LEM_METHOD_DENSE || p->op.ndim != 1 || p->opt.precision != LEM_FP64 ||
      p->U != 1 || !p->d_core || p->boxes.empty())
    return false;
  const int rows = p->rows, h = p->boxes[0].h;
  for (size_t i = 0; i < p->boxes.size(); ++i) {
    const Box& b = p->boxes[i];
    if (b.cx != rows || b.h != h || b.ox != (int)i * rows) return false;
  }
  if (p->cols != rows + 2 * h || 2 * h + rows > p->op.n) return false;
  return lem::dense_resident_members(p->op.n, p->ns, rows, p->cols, (int)p->boxes.size()) > 0;
}

lem_status run_step(lem_plan_s* p, const double* src, double* dst, hipStream_t st) {
  if (!p->opt.use_graph || st == nullptr) return run_one(p, src, dst, st);
  auto key = std::make_pair((const void*)src, (void*)dst);
  auto it = p->graphs.find(key);
  if (it == p->graphs.end()) {
    hipGraph_t g;
    hipGraphExec_t ex;
    LEM_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    lem_status s = run_one(p, src, dst, st);
    hipError_t e = hipStreamEndCapture(st, &g);
    if (s != LEM_OK) return s;
    if (e != hipSuccess) return fail(LEM_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      hipGraphDestroy(g);
      return fail(LEM_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    it = p->graphs.emplace(key, std::make_pair(g, ex)).first;
  }
  LEM_HIP(hipGraphLaunch(it->second.second, st));
  return LEM_OK;
}

lem_status check_options(const lem_options* o) {
  if (!o) return fail(LEM_ERR_INVALID, "options are NULL");
  if (o->method < 0 || o->method > 4 || o->method == LEM_METHOD_ROSENBROCK)
    return fail(LEM_ERR_INVALID, "unknown method");
  if (o->precision < 0 || o->precision > 3) return fail(LEM_ERR_INVALID, "unknown precision");
  if (o->precision != LEM_FP64 && o->method != LEM_METHOD_DENSE)
    return fail(LEM_ERR_UNSUPPORTED, "reduced precision applies to the dense method only");
  if (o->n_states < 1) return fail(LEM_ERR_INVALID, "n_states must be >= 1");
  if (o->core < 0 || o->halo < 0) return fail(LEM_ERR_INVALID, "core and halo must be >= 0");
  if (o->halo == 0 && (o->halo_min < 0 || o->halo_max < o->halo_min || !(o->halo_tol > 0)))
    return fail(LEM_ERR_INVALID, "decay-bound halo needs 0 <= halo_min <= halo_max, halo_tol > 0");
  const int mlim = o->method == LEM_METHOD_GLOBAL ? lem::kMaxKrylov : lem::krylov_big_max_m();
  if (o->krylov_m < 0 || o->krylov_m > mlim || o->krylov_m_max < 2 || o->krylov_m_max > mlim)
    return fail(LEM_ERR_INVALID, "Krylov dimension must be in [2, " + std::to_string(mlim) + "]");
  if (o->max_substeps < 1) return fail(LEM_ERR_INVALID, "max_substeps must be >= 1");
  if (!(o->krylov_tol > 0)) return fail(LEM_ERR_INVALID, "krylov_tol must be > 0");
  if (o->expm != LEM_EXPM_PADE && o->expm != LEM_EXPM_TAYLOR)
    return fail(LEM_ERR_INVALID, "unknown local exponential algorithm");
  if (o->columns && (o->method != LEM_METHOD_KRYLOV || o->core <= 0))
    return fail(LEM_ERR_UNSUPPORTED, "column-wise cores need the Krylov method and a core width");
  if (o->tile < -1 || o->tile >= lem::kApplyConfigs)
    return fail(LEM_ERR_INVALID, "tile must be -1 or a shape id in [0, 7]");
  if (o->core_max != 0 && o->core_max != 16 && o->core_max != 32 && o->core_max != 64)
    return fail(LEM_ERR_INVALID, "core_max must be 0, 16, 32 or 64");
  return LEM_OK;
}

void fill_info(const lem_plan_s* p, lem_plan_info* in) {
  std::memset(in, 0, sizeof(*in));
  in->n_blocks = (int)p->boxes.size();
  in->n_unique = p->U;
  in->halo_min = INT32_MAX;
  in->halo_max = 0;
  in->n_loc_max = 0;
  for (const auto& b : p->boxes) {
    const int64_t nl = (int64_t)box_lx(b, p->op.n) * box_ly(b, p->op.n, p->op.ndim);
    in->n_loc_total += nl;
    in->n_loc_max = std::max<int>(in->n_loc_max, (int)nl);
    in->halo_min = std::min(in->halo_min, b.h);
    in->halo_max = std::max(in->halo_max, b.h);
  }
  if (p->boxes.empty()) in->halo_min = 0;
  in->halo_clamped = p->n_clamped;
  in->m_min = p->m.empty() ? 0 : *std::min_element(p->m.begin(), p->m.end());
  in->m_max = p->m.empty() ? 0 : *std::max_element(p->m.begin(), p->m.end());
  in->substeps_max = p->nsub.empty() ? 0 : *std::max_element(p->nsub.begin(), p->nsub.end());
  in->squarings = p->squarings;
  in->bytes_blocks = p->bytes_blocks;
  in->bytes_work = p->bytes_work;
  in->plan_ms = p->plan_ms;
  in->tile_config = p->tile;
  in->resident_steps = p->resident ? 1 : 0;
  for (const auto& bk : p->buckets)
    for (int i = bk.first; i < bk.first + bk.count && i < (int)p->kb_host.size(); ++i) {
      const lem::KBlock& k = p->kb_host[i];
      const double bytes = (double)p->ns * (k.Lx * k.Ly + k.aug) * 8.0 *
                           ((double)k.m * (k.m + 1) + 3.0 * k.m) * k.nsub;
      in->krylov_bytes_step += bytes;
      if (!bk.vlds) in->krylov_bytes_streamed += bytes;
    }
}

bool overlap(const void* a, const void* b, size_t bytes) {
  const char* x = (const char*)a;
  const char* y = (const char*)b;
  return x < y + bytes && y < x + bytes;
}

// lem_status of latched device status bits (non-finite values first).
int device_status_of(int bits) {
  return (bits & lem::kStatusNonFinite)     ? LEM_ERR_NONFINITE
         : (bits & lem::kStatusNotConverged) ? LEM_ERR_NOT_CONVERGED
                                             : LEM_OK;
}

lem_status create_plan_one(const lem_operator* op, double dt, const lem_options* opt,
                           void* stream, lem::Arena* arena, lem_plan_t* out);

// Time of one step of a Krylov plan on a probe state (ms, median of three
// after one warm-up step); buffers from hipMalloc.
lem_status time_krylov_step(lem_plan_s* p, double* ms) {
  const int64_t tot = p->N * p->ns;
  double *a = nullptr, *b = nullptr;
  hipStream_t st = p->stream;
  LEM_TRY(dalloc(p, &a, (size_t)tot));
  LEM_TRY(dalloc(p, &b, (size_t)tot));
  LEM_HIP(lem::launch_probe_fill(a, tot, 4242u, st));
  hipEvent_t e[4];
  for (auto& ev : e) LEM_HIP(hipEventCreate(&ev));
  lem_status s = run_one(p, a, b, st);
  for (int r = 0; r < 3 && s == LEM_OK; ++r) {
    if (hipEventRecord(e[r], st) != hipSuccess) s = fail(LEM_ERR_HIP, "event record failed");
    if (s == LEM_OK) s = run_one(p, a, b, st);
  }
  if (s == LEM_OK && hipEventRecord(e[3], st) != hipSuccess) s = fail(LEM_ERR_HIP, "event record failed");
  if (s == LEM_OK && hipEventSynchronize(e[3]) != hipSuccess) s = fail(LEM_ERR_HIP, "event sync failed");
  float t[3] = {0, 0, 0};
  for (int r = 0; r < 3 && s == LEM_OK; ++r) hipEventElapsedTime(&t[r], e[r], e[r + 1]);
  std::sort(t, t + 3);
  *ms = t[1];
  for (auto& ev : e) hipEventDestroy(ev);
  dfree(p, a);
  dfree(p, b);
  // the timing steps latched into the plan's status word and estimates: start clean
  if (s == LEM_OK) s = hipMemsetAsync(p->d_status, 0, sizeof(int), st) == hipSuccess
                           ? LEM_OK : fail(LEM_ERR_HIP, "status reset failed");
  if (s == LEM_OK && p->d_diag)
    s = hipMemsetAsync(p->d_diag, 0, p->boxes.size() * p->ns * sizeof(double), st) == hipSuccess
            ? LEM_OK : fail(LEM_ERR_HIP, "estimate reset failed");
  return s;
}

// Uneven Krylov partitions with autotune: the partitions whose largest core is
// 32 and 64 points, each with Krylov dimensions capped at 30 and at the
// caller's cap, are planned and timed on a probe state; the fastest is kept.
// (Boxes of 64^2 cores cut the buffer overhead, but each is one workgroup with
// a long Arnoldi chain; dimensions above 30 save sub-steps but run on the
// large-box kernel: whether either pays depends on the operator, the grid and
// the CUs.)
lem_status create_plan(const lem_operator* op, double dt, const lem_options* opt, void* stream,
                       lem::Arena* arena, lem_plan_t* out) {
  if (!opt || !out || opt->method != LEM_METHOD_KRYLOV || opt->core != 0 || !opt->autotune ||
      opt->dry_run || arena || opt->core_max == 16)
    return create_plan_one(op, dt, opt, stream, arena, out);
  const auto t0 = std::chrono::steady_clock::now();
  lem_plan_t best = nullptr;
  double best_ms = INFINITY;
  // candidates: largest core 32 or 64, Krylov dimensions capped at 30 (the
  // LDS / streamed kernel) or at the caller's cap (the large-box kernel for
  // dimensions above 30)
  std::vector<std::pair<int, int>> cands;
  for (int cm : {32, 64}) {
    if (opt->core_max && cm > opt->core_max) continue;
    cands.push_back({cm, std::min(opt->krylov_m_max, lem::krylov_lds_max_m())});
    if (opt->krylov_m_max > lem::krylov_lds_max_m()) cands.push_back({cm, opt->krylov_m_max});
  }
  for (const auto& cand : cands) {
    lem_options o = *opt;
    o.core_max = cand.first;
    o.krylov_m_max = cand.second;
    lem_plan_t p = nullptr;
    lem_status s = create_plan_one(op, dt, &o, stream, arena, &p);
    if (s == LEM_ERR_UNSUPPORTED) continue;  // boxes past the kernels' limits
    if (s != LEM_OK) {
      delete best;
      return s;
    }
    double ms = INFINITY;
    s = time_krylov_step(p, &ms);
    if (s != LEM_OK) {
      delete p;
      delete best;
      return s;
    }
    if (ms < best_ms) {
      delete best;
      best = p;
      best_ms = ms;
    } else {
      delete p;
    }
  }
  if (!best) return create_plan_one(op, dt, opt, stream, arena, out);
  best->opt.core_max = opt->core_max;
  best->opt.krylov_m_max = opt->krylov_m_max;
  best->plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = best;
  return LEM_OK;
}

lem_status create_plan_one(const lem_operator* op, double dt, const lem_options* opt,
                           void* stream, lem::Arena* arena, lem_plan_t* out) {
  if (!out) return fail(LEM_ERR_INVALID, "out is NULL");
  *out = nullptr;
  LEM_TRY(check_options(opt));
  const auto t0 = std::chrono::steady_clock::now();
  auto p = new lem_plan_s();
  auto guard = [&](lem_status s) { if (s != LEM_OK) delete p; return s; };
  p->arena = arena;
  p->opt = *opt;
  p->method = opt->method;
  p->ns = opt->n_states;
  p->dry = opt->dry_run != 0;
  p->stream = (hipStream_t)stream;
  lem_status s = build_op(op, dt, &p->op);
  if (s != LEM_OK) return guard(s);
  if (p->method == LEM_METHOD_DENSE && p->op.variable &&
      (op->forcing != nullptr || opt->precision >= LEM_BF16X2 || opt->core <= 0))
    return guard(fail(LEM_ERR_UNSUPPORTED, "variable-coefficient stored blocks take a uniform core, "
                                           "FP64 or FP32 and no forcing"));
  p->N = p->op.N();
  p->forced = op->forcing != nullptr;
  if (p->forced) {
    for (int64_t e = 0; e < p->N * p->ns; ++e)
      if (!std::isfinite(op->forcing[e])) return guard(fail(LEM_ERR_INVALID, "forcing must be finite"));
  }
  if (p->method == LEM_METHOD_GLOBAL && p->N + (p->forced ? 1 : 0) <= 4096 &&
      p->opt.krylov_m_max <= lem::krylov_lds_max_m()) {
    // the whole grid fits one box: the global method is the Krylov step on
    // a single box that keeps the periodic coupling (D = 1)
    p->global_box = true;
    p->boxes.push_back({0, 0, p->op.n, p->op.ndim == 2 ? p->op.n : 1, 0});
  }
  if (p->method == LEM_METHOD_KRONECKER && (p->op.ndim != 2 || p->op.variable || p->forced))
    return guard(fail(LEM_ERR_UNSUPPORTED, "the Kronecker-factored method takes a 2D constant-"
                                           "coefficient operator and no forcing"));
  if (p->method == LEM_METHOD_KRYLOV || p->method == LEM_METHOD_DENSE ||
      p->method == LEM_METHOD_KRONECKER) {
    if (p->opt.core == 0 && p->method == LEM_METHOD_KRYLOV && p->op.ndim == 1)
      p->opt.core = std::min(64, p->op.n);
    if (p->opt.core == p->op.n)
      return guard(fail(LEM_ERR_INVALID, "a single core covering the grid is the global method"));
    s = make_partition(p);
    if (s != LEM_OK) return guard(s);
  }
  if (p->method == LEM_METHOD_KRONECKER &&
      (2 * p->boxes[0].h + p->boxes[0].cx > lem::kron_max_side() ||
       p->boxes[0].cx > lem::kron_max_core()))
    return guard(fail(LEM_ERR_UNSUPPORTED, "Kronecker-factored boxes are at most " +
                                               std::to_string(lem::kron_max_side()) +
                                               " points per side, cores at most " +
                                               std::to_string(lem::kron_max_core())));
  if (p->method == LEM_METHOD_KRYLOV && p->opt.columns) {
    // column-wise boxes stay on the kernels of boxes up to 4096 points: a
    // column partition on the large-box kernel's 12-points-per-lane shape
    // with an ensemble ended its process (cause not yet established)
    for (const Box& b : p->boxes)
      if ((int64_t)box_lx(b, p->op.n) * box_ly(b, p->op.n, p->op.ndim) + (p->forced ? 1 : 0) > 4096)
        return guard(fail(LEM_ERR_UNSUPPORTED, "column-wise Krylov boxes are limited to 4096 points"));
  }
  if (p->method == LEM_METHOD_KRYLOV) {
    // the Krylov kernels hold a basis row of at most 9216 points (the box
    // plus the augmented coordinate of a forced step)
    for (const Box& b : p->boxes)
      if ((int64_t)box_lx(b, p->op.n) * box_ly(b, p->op.n, p->op.ndim) + (p->forced ? 1 : 0) >
          lem::krylov_big_max_n())
        return guard(fail(LEM_ERR_UNSUPPORTED, "local box larger than 9216 points (9215 when forced)"));
  }
  if (!p->dry) {
    hipStream_t st = p->stream;
    s = dalloc(p, &p->d_status, 1);
    if (s != LEM_OK) return guard(s);
    if (hipMemsetAsync(p->d_status, 0, sizeof(int), st) != hipSuccess)
      return guard(fail(LEM_ERR_HIP, "hipMemsetAsync failed"));
    if (!arena) {  // serving plans step between the server's own buffers
      s = dalloc(p, &p->d_tmp, (size_t)p->N * p->ns, &p->bytes_work);
      if (s != LEM_OK) return guard(s);
    }
    if (p->forced) {
      s = dalloc(p, &p->d_force, (size_t)p->N * p->ns, &p->bytes_work);
      if (s == LEM_OK) s = upload(p->d_force, op->forcing, (size_t)p->N * p->ns * 8, st);
      if (s != LEM_OK) return guard(s);
    }
    if (p->method == LEM_METHOD_KRYLOV || p->global_box) s = plan_krylov(p, st);
    else if (p->method == LEM_METHOD_DENSE) s = plan_dense(p, st, op->forcing);
    else if (p->method == LEM_METHOD_KRONECKER) s = plan_kron(p, st);
    else s = plan_global(p, st);
    if (s != LEM_OK) return guard(s);
    if (p->method == LEM_METHOD_DENSE) {
      s = choose_tile(p, st);
      if (s != LEM_OK) return guard(s);
      p->resident = resident_fits(p);
    }
    if (hipStreamSynchronize(st) != hipSuccess)
      return guard(fail(LEM_ERR_HIP, "plan synchronization failed"));
  } else if (p->method == LEM_METHOD_KRYLOV) {
    p->m.assign(p->boxes.size(), opt->krylov_m);
    p->nsub.assign(p->boxes.size(), 1);
  }
  p->plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = p;
  return LEM_OK;
}


}  // namespace lemh

using namespace lemh;

namespace lem {

lem_status set_error(lem_status s, const char* msg) { return fail(s, msg); }

lem_status global_expmv_in(const lem_operator* op, double t, const double* x, double* y,
                           int32_t n_states, double tol, int32_t m_max, void* stream,
                           Arena* arena) {
  if (!op || !x || !y) return fail(LEM_ERR_INVALID, "NULL argument");
  lem_options o;
  lem_options_default(&o);
  o.method = LEM_METHOD_GLOBAL;
  o.n_states = n_states;
  o.krylov_tol = tol;
  o.krylov_m_max = m_max;
  lem_plan_t p = nullptr;
  LEM_TRY(create_plan(op, t, &o, stream, arena, &p));
  const size_t bytes = (size_t)p->N * p->ns * sizeof(double);
  if (overlap(x, y, bytes)) {
    delete p;
    return fail(LEM_ERR_INVALID, "x and y overlap");
  }
  hipStream_t st = (hipStream_t)stream;
  p->stream = st;
  lem_status s = run_one(p, x, y, st);
  if (s == LEM_OK && hipStreamSynchronize(st) != hipSuccess)
    s = fail(LEM_ERR_HIP, "synchronization failed");
  int bits = 0;
  if (s == LEM_OK && hipMemcpy(&bits, p->d_status, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
    s = fail(LEM_ERR_HIP, "status copy failed");
  delete p;  // returns its memory (to the arena when one is given)
  if (s == LEM_OK && bits)
    s = fail((lem_status)device_status_of(bits), device_status_of(bits) == LEM_ERR_NONFINITE
                                                     ? "non-finite values in the global Krylov action"
                                                     : "global Krylov estimate above tolerance");
  return s;
}

size_t global_expmv_bound(const lem_operator* op, int32_t n_states, int32_t m_max) {
  const int64_t N = op->ndim == 1 ? (int64_t)op->n : (int64_t)op->n * op->n;
  const bool forced = op->forcing != nullptr;
  const bool variable = op->nu_field != nullptr || op->vel_faces != nullptr;
  const int64_t ns = std::max(n_states, 1);
  const int64_t mc = std::min(std::max(m_max, 4), kMaxKrylov);
  const int64_t K = kMaxKrylov + 1;
  const int64_t Na = N + (forced ? 1 : 0), tot = Na * ns;
  // persistent: status word, face coefficients, forcing
  const int64_t keep = 1 + (variable ? 4 * N : 0) + (forced ? N * ns : 0);
  // calibration (one state, dimension mc) and the step (n_states, dimension
  // <= mc) are never allocated at once
  const int64_t calib = (mc + 3) * Na + (int64_t)global_part_doubles(global_grid(N, 1), 1) +
                        3 * K + 2 * (mc + 1) * mc + 8 * mc + N + 16;
  const int64_t step = (mc + 3) * tot + (int64_t)global_part_doubles(global_grid(tot, ns), (int)ns) +
                       3 * K * ns + ns * (mc + 1) * mc + ns * mc + 4 * ns + (forced ? 2 * tot : 0);
  return (size_t)(keep + std::max(calib, step)) * sizeof(double) + 64 * 256;
}

}  // namespace lem

// ================================================================ C ABI ====
extern "C" {

void lem_options_default(lem_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->method = LEM_METHOD_KRYLOV;
  o->precision = LEM_FP64;
  o->n_states = 1;
  o->core = 0;
  o->halo = 0;
  o->halo_min = 4;
  o->halo_max = 64;
  o->halo_tol = 1e-8;
  o->krylov_m = 0;
  o->krylov_m_max = 30;
  o->max_substeps = 64;
  o->krylov_tol = 1e-13;
  o->use_graph = 0;
  o->autotune = 0;
  o->dry_run = 0;
  o->core_max = 0;
  o->tile = -1;
}

lem_status lem_plan(const lem_operator* op, double dt, const lem_options* opt, void* stream,
                    lem_plan_t* out) {
  return create_plan(op, dt, opt, stream, nullptr, out);
}

lem_status lem_step(lem_plan_t p, const double* x_in, double* x_out, int32_t n_steps,
                    void* stream) {
  if (!p) return fail(LEM_ERR_INVALID, "plan is NULL");
  if (p->dry) return fail(LEM_ERR_INVALID, "a dry-run plan cannot step");
  if (!p->d_tmp) return fail(LEM_ERR_INVALID, "a serving plan is stepped by its server");
  if (!x_in || !x_out) return fail(LEM_ERR_INVALID, "state pointers must not be NULL");
  if (n_steps < 1) return fail(LEM_ERR_INVALID, "n_steps must be >= 1");
  const size_t bytes = (size_t)p->N * p->ns * sizeof(double);
  if (overlap(x_in, x_out, bytes)) return fail(LEM_ERR_INVALID, "x_in and x_out overlap");
  hipStream_t st = (hipStream_t)stream;
  p->stream = st;
  if (p->resident) {
    LEM_HIP(lem::dense_resident_steps(p->d_core, p->d_bias, x_in, x_out, p->d_status, p->op.n,
                                      p->ns, p->rows, p->cols, (int)p->boxes.size(),
                                      p->boxes[0].h, n_steps, st));
    return LEM_OK;
  }
  // last step writes x_out; earlier steps alternate x_out / tmp backwards
  const double* src = x_in;
  for (int k = 0; k < n_steps; ++k) {
    double* dst = ((n_steps - 1 - k) % 2 == 0) ? x_out : p->d_tmp;
    LEM_TRY(run_step(p, src, dst, st));
    src = dst;
  }
  return LEM_OK;
}

lem_status lem_global_expmv(const lem_operator* op, double t, const double* x, double* y,
                            int32_t n_states, double tol, int32_t m_max, void* stream) {
  return lem::global_expmv_in(op, t, x, y, n_states, tol, m_max, stream, nullptr);
}

lem_status lem_plan_query(lem_plan_t p, lem_plan_info* info) {
  if (!p || !info) return fail(LEM_ERR_INVALID, "NULL argument");
  fill_info(p, info);
  if (p->dry) return LEM_OK;
  LEM_HIP(hipStreamSynchronize(p->stream));
  int st = 0;
  LEM_HIP(hipMemcpy(&st, p->d_status, sizeof(int), hipMemcpyDeviceToHost));
  info->device_status = device_status_of(st);
  if (p->ere_small && p->ere_count > 0) {  // doublings taken at the last refresh
    std::vector<int> sq(p->boxes.size() * p->ns);
    LEM_HIP(hipMemcpy(sq.data(), p->d_ere_s, sq.size() * sizeof(int), hipMemcpyDeviceToHost));
    for (int v : sq) info->squarings = std::max(info->squarings, v);
  }
  double mx = 0.0;
  if ((p->method == LEM_METHOD_KRYLOV || p->global_box) && p->d_diag) {
    std::vector<double> d(p->boxes.size() * p->ns);
    LEM_HIP(hipMemcpy(d.data(), p->d_diag, d.size() * 8, hipMemcpyDeviceToHost));
    for (double v : d) mx = std::max(mx, v);
  } else if (p->method == LEM_METHOD_GLOBAL && p->gw.estsum) {
    std::vector<double> d(p->ns);
    LEM_HIP(hipMemcpy(d.data(), p->gw.estsum, d.size() * 8, hipMemcpyDeviceToHost));
    for (double v : d) mx = std::max(mx, v);
  }
  info->max_estimate = mx;
  return LEM_OK;
}

lem_status lem_plan_copy_maps(lem_plan_t p, int32_t* boxes, int32_t* gather, int32_t* scatter) {
  if (!p) return fail(LEM_ERR_INVALID, "plan is NULL");
  const int n = p->op.n;
  const int ndim = p->op.ndim;
  int64_t gi = 0, si = 0;
  for (size_t k = 0; k < p->boxes.size(); ++k) {
    const Box& b = p->boxes[k];
    if (boxes) {
      boxes[5 * k + 0] = b.ox; boxes[5 * k + 1] = b.oy; boxes[5 * k + 2] = b.cx;
      boxes[5 * k + 3] = ndim == 2 ? b.cy : 1; boxes[5 * k + 4] = b.h;
    }
    const int hx = box_hx(b, n), hy = box_hy(b, n, ndim);
    const int Lx = box_lx(b, n), Ly = box_ly(b, n, ndim);
    if (gather)
      for (int ly = 0; ly < Ly; ++ly)
        for (int lx = 0; lx < Lx; ++lx) {
          const int gx = ((b.ox - hx + lx) % n + n) % n;
          const int gy = ndim == 2 ? ((b.oy - hy + ly) % n + n) % n : 0;
          gather[gi++] = gy * n + gx;
        }
    if (scatter) {
      const int cy = ndim == 2 ? b.cy : 1;
      for (int ry = 0; ry < cy; ++ry)
        for (int rx = 0; rx < b.cx; ++rx) scatter[si++] = (b.oy + ry) * n + b.ox + rx;
    }
  }
  return LEM_OK;
}

lem_status lem_plan_copy_krylov(lem_plan_t p, int32_t* m, int32_t* substeps) {
  if (!p) return fail(LEM_ERR_INVALID, "plan is NULL");
  if (p->method == LEM_METHOD_DENSE) return fail(LEM_ERR_INVALID, "dense plan has no Krylov data");
  for (size_t i = 0; i < p->m.size(); ++i) {
    if (m) m[i] = p->m[i];
    if (substeps) substeps[i] = p->nsub[i];
  }
  return LEM_OK;
}

lem_status lem_plan_copy_block(lem_plan_t p, int32_t unique, double* out, int32_t* rows,
                               int32_t* cols) {
  if (!p) return fail(LEM_ERR_INVALID, "plan is NULL");
  if (p->method != LEM_METHOD_DENSE || p->dry)
    return fail(LEM_ERR_INVALID, "only a dense plan stores local exponentials");
  if (unique < 0 || unique >= p->U) return fail(LEM_ERR_INVALID, "block index out of range");
  if (rows) *rows = p->rows;
  if (cols) *cols = p->cols;
  if (out) {
    LEM_HIP(hipStreamSynchronize(p->stream));
    LEM_HIP(hipMemcpy(out, p->d_core + (size_t)unique * p->rows * p->cols,
                      (size_t)p->rows * p->cols * 8, hipMemcpyDeviceToHost));
  }
  return LEM_OK;
}

lem_status lem_plan_destroy(lem_plan_t p) {
  if (!p) return LEM_OK;
  if (!p->dry) hipStreamSynchronize(p->stream);
  delete p;
  return LEM_OK;
}


}  // extern "C"
