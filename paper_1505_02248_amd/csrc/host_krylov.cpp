// Planning and launching of the Krylov local actions (section 4.3): the
// partition into cores and buffers, per-block Krylov dimensions calibrated on
// a probe, launch buckets by kernel shape.
#include "host_internal.h"

namespace lemh {

// ------------------------------------------------------------- partition --
lem_status make_partition(lem_plan_s* p) {
  const Op& op = p->op;
  const lem_options& o = p->opt;
  const int n = op.n;
  const double G = growth_factor(op);
  auto pick_halo = [&](Box b) -> int {
    if (o.halo > 0) return o.halo;
    bool cl = false;
    const int h = halo_from_bound(op, b, o.halo_tol, o.halo_min, o.halo_max, G, &cl);
    if (cl) p->n_clamped++;
    return h;
  };
  if (o.core > 0) {
    const int c = o.core;
    if (n % c) return fail(LEM_ERR_INVALID, "core side must divide n");
    const int nb = n / c;
    if (o.columns) {  // cores of c x n: whole columns, buffers across columns only
      for (int bx = 0; bx < nb; ++bx) p->boxes.push_back({bx * c, 0, c, n, 0});
    } else if (op.ndim == 1) {
      for (int bx = 0; bx < nb; ++bx) p->boxes.push_back({bx * c, 0, c, 1, 0});
    } else {
      for (int by = 0; by < nb; ++by)
        for (int bx = 0; bx < nb; ++bx) p->boxes.push_back({bx * c, by * c, c, c, 0});
    }
    // a uniform partition of a constant operator has one halo for all blocks
    if (!op.variable) {
      const int h = pick_halo(p->boxes[0]);
      if (o.halo <= 0 && p->n_clamped) p->n_clamped = (int)p->boxes.size();
      for (auto& b : p->boxes) b.h = h;
    } else {
      for (auto& b : p->boxes) b.h = pick_halo(b);
    }
  } else {
    if (op.ndim != 2 || p->method != LEM_METHOD_KRYLOV)
      return fail(LEM_ERR_UNSUPPORTED, "uneven cores need the 2D Krylov method");
    if (n % 64) return fail(LEM_ERR_INVALID, "uneven cores need n divisible by 64");
    // Per 64x64 tile choose the core side c in {16, 32, 64} with the least
    // modelled cost: local points per core point, weighted up when the Krylov
    // basis must stream through device memory instead of staying in LDS.
    const int cands[3] = {16, 32, 64};
    const int cmax = o.core_max > 0 ? o.core_max : 64;
    const int mguess = std::max(8, std::min(o.krylov_m_max, 30));
    for (int ty = 0; ty < n / 64; ++ty)
      for (int tx = 0; tx < n / 64; ++tx) {
        double best = INFINITY;
        std::vector<Box> bestb;
        int best_cl = 0;
        for (int c : cands) {
          if (c > cmax) continue;
          std::vector<Box> bs;
          int cl_before = p->n_clamped;
          for (int by = 0; by < 64 / c; ++by)
            for (int bx = 0; bx < 64 / c; ++bx) {
              Box b{tx * 64 + bx * c, ty * 64 + by * c, c, c, 0};
              b.h = pick_halo(b);
              bs.push_back(b);
            }
          const int cl = p->n_clamped - cl_before;
          p->n_clamped = cl_before;
          double cost = 0;
          for (auto& b : bs) {
            const int L = c + 2 * b.h;
            cost += block_cost(2, L * L + (p->forced ? 1 : 0), std::min(mguess, 16), 1);
          }
          if (cost < best) { best = cost; bestb = bs; best_cl = cl; }
        }
        p->n_clamped += best_cl;
        p->boxes.insert(p->boxes.end(), bestb.begin(), bestb.end());
      }
  }
  for (auto& b : p->boxes) {
    const int Lx = box_lx(b, n);
    const int Ly = box_ly(b, n, op.ndim);
    if ((b.cx < n && Lx >= n) || (op.ndim == 2 && b.cy < n && Ly >= n))
      return fail(LEM_ERR_INVALID, "box (core + 2*halo) reaches itself through the periodic wrap;"
                                   " use a larger grid, a smaller halo or the global method");
  }
  return LEM_OK;
}

// --------------------------------------------------------------- Krylov ----
// Face coefficient arrays of a variable operator: mux, muy, then (face
// velocities) ax, ay, N doubles each.
lem_status upload_coef(lem_plan_s* p, hipStream_t st) {
  const Op& op = p->op;
  const size_t N = (size_t)op.N();
  LEM_TRY(dalloc(p, &p->d_coef, (op.varvel ? 4 : 2) * N, &p->bytes_work));
  LEM_TRY(upload(p->d_coef, op.mux.data(), N * 8, st));
  LEM_TRY(upload(p->d_coef + N, op.muy.data(), N * 8, st));
  if (op.varvel) {
    LEM_TRY(upload(p->d_coef + 2 * N, op.ax.data(), N * 8, st));
    LEM_TRY(upload(p->d_coef + 3 * N, op.ay.data(), N * 8, st));
  }
  return LEM_OK;
}

lem::KBlock make_kblock(const lem_plan_s* p, const Box& b, int m, int nsub, int ns, int diag,
                        bool forced = false) {
  lem::KBlock k{};
  k.aug = forced ? 1 : 0;
  k.gscale = p->op.dt / nsub;
  k.force = forced ? p->d_force : nullptr;
  const double sc = 1.0 / nsub;
  const Op& op = p->op;
  k.w0 = op.w[0] * sc; k.wW = op.w[1] * sc; k.wE = op.w[2] * sc; k.wS = op.w[3] * sc;
  k.wN = op.w[4] * sc;
  k.chx = op.chx * sc; k.chy = op.chy * sc; k.sub_scale = sc;
  k.tol = p->opt.krylov_tol;
  k.x_off = 0;
  k.mu_off = op.variable ? 0 : -1;
  k.varvel = op.varvel ? 1 : 0;
  k.v_off = 0;
  k.n = op.n; k.ndim = op.ndim;
  k.ox = b.ox; k.oy = b.oy; k.cx = b.cx; k.cy = b.cy;
  k.h = box_hx(b, op.n); k.hy = box_hy(b, op.n, op.ndim);
  k.Lx = box_lx(b, op.n); k.Ly = box_ly(b, op.n, op.ndim);
  k.m = m; k.nsub = nsub; k.ns = ns; k.diag = diag;
  k.periodic = (b.cx == op.n ? 1 : 0) | (op.ndim == 2 && b.cy == op.n ? 2 : 0);
  return k;
}


// nloc counts the basis row (box points plus the augmented coordinate of a
// forced step, aug = 1).
LaunchKey launch_key(int ndim, int nloc, int m, size_t* lds, int aug) {
  int nt, pm;
  lem::krylov_lds_config(ndim, nloc, &nt, &pm);
  if (nt == 0 || m > lem::krylov_lds_max_m()) {
    lem::krylov_big_config(nloc, &nt, &pm);
    if (nt == 0 || m > lem::krylov_big_max_m()) return {-1, 0, 0, false};
    *lds = lem::krylov_big_lds_bytes(nt, pm, m);
    return {aug ? 4 : 3, nt, pm, false};
  }
  const size_t with_v = lem::krylov_lds_bytes(nt, m, nloc, true, aug);
  const int variant = aug ? 2 : 1;  // 2: kernels with the augmented coordinate
  if (pm <= 8 && nt <= 256 && with_v <= 160 * 1024) {  // wide shapes stream the basis
    *lds = with_v;
    return {variant, nt, pm, true};
  }
  *lds = lem::krylov_lds_bytes(nt, m, nloc, false, aug);
  return {variant, nt, pm, false};
}

// Relative cost of one block step with Krylov dimension m and nsub sub-steps:
// basis work grows like m (orthogonalization) per point and iteration, and a
// streamed basis costs about four times an LDS-resident one.
double block_cost(int ndim, int nloc, int m, int nsub) {
  size_t lds;
  const LaunchKey k = launch_key(ndim, nloc, m, &lds);
  if (k.variant < 0) return INFINITY;
  // the large-box kernel reads each direction twice more per column
  const double f = k.vlds ? 1.0 : (k.variant >= 3 ? 4.5 : 4.0);
  return f * nsub * (double)nloc * (m * (m + 3.0) + 40.0);
}

// Groups blocks by launch shape; assigns global-basis offsets. Reorders kb.
lem_status bucketize(std::vector<lem::KBlock>& kb, std::vector<lem_plan_s::Bucket>& buckets,
                     int ns, int64_t* vwork_doubles) {
  std::map<LaunchKey, std::vector<int>> groups;
  std::vector<size_t> need(kb.size());
  for (size_t i = 0; i < kb.size(); ++i) {
    const int nloc = kb[i].Lx * kb[i].Ly + kb[i].aug;  // basis row (plus augmented coordinate)
    const LaunchKey key = launch_key(kb[i].ndim, nloc, kb[i].m, &need[i], kb[i].aug);
    if (key.variant < 0)
      return fail(LEM_ERR_UNSUPPORTED, "local box larger than 9216 points (9215 when forced)");
    const size_t stage = key.variant >= 3 ? 0
                         : lem::krylov_stage_bytes(key.nt, key.vlds, kb[i].mu_off >= 0,
                                                   kb[i].varvel != 0, kb[i].ndim, kb[i].Lx,
                                                   kb[i].Ly);
    kb[i].stage = (stage > 0 && need[i] + stage <= 160 * 1024) ? 1 : 0;
    if (kb[i].stage) need[i] += stage;
    groups[key].push_back((int)i);
  }
  std::vector<lem::KBlock> out;
  buckets.clear();
  int64_t voff = 0;
  // costliest blocks first within a launch: workgroups are dispatched in
  // order, so the cheap ones fill the last round instead of the long ones
  // starting late (every block writes only its own core rows and slots)
  for (auto& g : groups) {
    std::vector<double> c(kb.size(), 0.0);
    for (int i : g.second)
      c[i] = block_cost(kb[i].ndim, kb[i].Lx * kb[i].Ly + kb[i].aug, kb[i].m, kb[i].nsub);
    std::stable_sort(g.second.begin(), g.second.end(), [&](int x, int y) { return c[x] > c[y]; });
  }
  for (auto& g : groups) {
    lem_plan_s::Bucket bk{g.first.variant, g.first.nt, g.first.pmax, g.first.vlds, 0,
                          (int)out.size(), (int)g.second.size()};
    for (int i : g.second) {
      lem::KBlock k = kb[i];
      bk.lds = std::max(bk.lds, need[i]);
      bk.cost += (double)ns * block_cost(k.ndim, k.Lx * k.Ly + k.aug, k.m, k.nsub);
      if (!g.first.vlds) {
        k.v_off = voff;
        voff += (int64_t)(k.m + 1 + k.aug) * (k.Lx * k.Ly + k.aug) * ns;
        if (g.first.variant >= 3) voff += lem::krylov_big_pad(g.first.nt, g.first.pmax);
      }
      out.push_back(k);
    }
    buckets.push_back(bk);
  }
  kb.swap(out);
  *vwork_doubles = voff;
  return LEM_OK;
}

// Large-box blocks with variable coefficients read their stencil weights from
// a table computed once (shared by the members) instead of the coefficient
// arrays: one slice of 5 * NT * P doubles per such block, pointers set here
// (before the table upload), values by fill_weights (after it).
lem_status attach_weights(lem_plan_s* p, std::vector<lem::KBlock>& kb,
                          const std::vector<lem_plan_s::Bucket>& bks, double** d_w) {
  *d_w = nullptr;
  int64_t nw = 0;
  for (const auto& bk : bks)
    if (bk.variant >= 3)
      for (int i = bk.first; i < bk.first + bk.count; ++i)
        if (kb[i].mu_off >= 0) nw += 5 * (int64_t)bk.nt * bk.pmax;
  if (nw == 0) return LEM_OK;
  LEM_TRY(dalloc(p, d_w, (size_t)nw, &p->bytes_work));
  int64_t off = 0;
  for (const auto& bk : bks)
    if (bk.variant >= 3)
      for (int i = bk.first; i < bk.first + bk.count; ++i)
        if (kb[i].mu_off >= 0) {
          kb[i].wts = *d_w + off;
          off += 5 * (int64_t)bk.nt * bk.pmax;
        }
  return LEM_OK;
}

lem_status fill_weights(const lem_plan_s* p, const lem::KBlock* d_kb,
                        const std::vector<lem_plan_s::Bucket>& bks, hipStream_t st) {
  for (const auto& bk : bks)
    if (bk.variant >= 3)
      LEM_HIP(lem::launch_krylov_weights(d_kb + bk.first, bk.count, bk.nt, bk.pmax, p->d_coef,
                                         st));
  return LEM_OK;
}

// One Krylov launch of a bucket's blocks with the kernel its variant names.
hipError_t launch_bucket(int variant, const lem::KBlock* blocks, int count, int ns, int nt,
                         int pmax, bool vlds, size_t lds, const double* src, double* dst,
                         const double* coef, double* vwork, double* diag, int* status,
                         double* calib, int mode, hipStream_t s) {
  if (variant >= 3)
    return lem::launch_krylov_big(blocks, count, ns, nt, pmax, lds, src, dst, coef, vwork, diag,
                                  status, calib, mode, variant == 4, s);
  return lem::launch_krylov_lds(blocks, count, ns, nt, pmax, vlds, lds, src, dst, coef, vwork,
                                diag, status, calib, mode, variant == 2, s);
}

lem_status launch_buckets(const lem_plan_s* p, const lem::KBlock* d_kb,
                          const std::vector<lem_plan_s::Bucket>& bks, int ns, const double* src,
                          double* dst, double* vwork, double* diag, double* calib, int mode,
                          hipStream_t st) {
  auto launch = [&](const lem_plan_s::Bucket& b, hipStream_t s) -> lem_status {
    hipError_t e = launch_bucket(b.variant, d_kb + b.first, b.count, ns, b.nt, b.pmax, b.vlds,
                                 b.lds, src, dst, p->d_coef, vwork, diag, p->d_status, calib,
                                 mode, s);
    if (e != hipSuccess)
      return fail(LEM_ERR_HIP, std::string("Krylov launch: ") + hipGetErrorString(e));
    return LEM_OK;
  };
  // calibration launches, single buckets and plans without side streams run
  // in order on the caller's stream
  if (mode != 0 || bks.size() < 2 || p->side.empty() || st == nullptr) {
    for (const auto& b : bks) LEM_TRY(launch(b, st));
    return LEM_OK;
  }
  // blocks write disjoint core rows, estimate slots and basis slices, so the
  // buckets are independent: fork, launch, join
  size_t big = 0;
  for (size_t i = 1; i < bks.size(); ++i)
    if (bks[i].cost > bks[big].cost) big = i;
  LEM_HIP(hipEventRecord(p->ev_fork, st));
  LEM_TRY(launch(bks[big], st));
  size_t k = 0;
  for (size_t i = 0; i < bks.size(); ++i) {
    if (i == big) continue;
    hipStream_t s = p->side[k % p->side.size()];
    if (k < p->side.size()) LEM_HIP(hipStreamWaitEvent(s, p->ev_fork, 0));
    LEM_TRY(launch(bks[i], s));
    ++k;
  }
  for (size_t j = 0; j < std::min(k, p->side.size()); ++j) {
    LEM_HIP(hipEventRecord(p->ev_join[j], p->side[j]));
    LEM_HIP(hipStreamWaitEvent(st, p->ev_join[j], 0));
  }
  return LEM_OK;
}

// Choose (m, nsub) from calibration estimates est[sub][j] of one block: the
// cheapest pair (block_cost) whose estimate meets half the tolerance.
bool choose_m(const double* est, const std::vector<int>& jl, int nsc, double tol, int mfix,
              int mcal, int ndim, int nloc, int* m, int* nsub) {
  double best = INFINITY;
  for (int e = 0; e < nsc; ++e)
    for (size_t q = 0; q < jl.size(); ++q) {
      const int j = jl[q];
      if (mfix > 0 && j != mfix) continue;
      if (!(est[e * jl.size() + q] <= 0.5 * tol)) continue;
      const int mm = (mfix > 0) ? j : std::min(j + 2, mcal);
      const double cost = nloc > 0 ? block_cost(ndim, nloc, mm, 1 << e)
                                   : (double)(1 << e) * (mm + 8);
      if (cost < best) { best = cost; *m = mm; *nsub = 1 << e; }
    }
  return best < INFINITY;
}

lem_status plan_krylov(lem_plan_s* p, hipStream_t st) {
  const Op& op = p->op;
  const lem_options& o = p->opt;
  const int nb = (int)p->boxes.size();
  // coefficient arrays
  if (op.variable) LEM_TRY(upload_coef(p, st));
  // Calibration representatives.  Krylov convergence is governed by the
  // box shape and the norm of dt*A_M: blocks with the same box and a row-sum
  // norm within the same 15% bucket share one calibration, taken on the
  // member with the largest norm (the runtime estimate still checks every
  // block every step).  Identical boxes of a constant operator share one.
  std::vector<int> rep(nb, -1);
  std::vector<int> reps;
  {
    std::map<std::tuple<int, int, int, int>, int> seen;
    std::vector<double> rho(nb, 0.0);
    for (int i = 0; i < nb; ++i) {
      const Box& b = p->boxes[i];
      int bucket = 0;
      if (op.variable) {
        rho[i] = block_rho(op, b);
        bucket = (int)std::floor(std::log(std::max(rho[i], 1e-300)) / std::log(1.15));
      }
      auto key = std::make_tuple(b.cx, b.cy, b.h, bucket);
      auto it = seen.find(key);
      if (it != seen.end()) {
        rep[i] = it->second;
        if (rho[i] > rho[reps[it->second]]) reps[it->second] = i;
        continue;
      }
      seen[key] = (int)reps.size();
      rep[i] = (int)reps.size();
      reps.push_back(i);
    }
  }
  const int mcal = std::min(std::max(o.krylov_m_max, 4), lem::kMaxKrylov);
  std::vector<int> jl;
  for (int j = 2; j <= mcal; ++j) jl.push_back(j);
  int nsc = 1;
  while ((1 << nsc) <= o.max_substeps && nsc < 12) ++nsc;
  // calibration blocks (ns = 1, unscaled weights, m = mcal)
  std::vector<lem::KBlock> cb;
  for (size_t r = 0; r < reps.size(); ++r)
    cb.push_back(make_kblock(p, p->boxes[reps[r]], mcal, 1, 1, (int)r));
  std::vector<lem_plan_s::Bucket> cbk;
  int64_t cv = 0;
  LEM_TRY(bucketize(cb, cbk, 1, &cv));
  double* d_cw = nullptr;
  LEM_TRY(attach_weights(p, cb, cbk, &d_cw));
  lem::KBlock* d_cb;
  double *d_probe, *d_cv, *d_calib, *d_cdiag, *d_est;
  int *d_mcal, *d_jl;
  int64_t* d_coff;
  const int64_t cstride = 2 + (int64_t)(mcal + 1) * mcal;
  const int nr = (int)cb.size();
  LEM_TRY(dalloc(p, &d_cb, cb.size()));
  LEM_TRY(dalloc(p, &d_probe, (size_t)op.N()));
  LEM_TRY(dalloc(p, &d_cv, (size_t)std::max<int64_t>(cv, 1)));
  LEM_TRY(dalloc(p, &d_calib, (size_t)nr * cstride));
  LEM_TRY(dalloc(p, &d_cdiag, (size_t)nr));
  LEM_TRY(dalloc(p, &d_est, (size_t)nr * nsc * jl.size()));
  LEM_TRY(dalloc(p, &d_mcal, (size_t)nr));
  LEM_TRY(dalloc(p, &d_jl, jl.size()));
  LEM_TRY(dalloc(p, &d_coff, (size_t)nr));
  std::vector<int> mc(nr, mcal);
  std::vector<int64_t> coff(nr);
  for (int k = 0; k < nr; ++k) coff[k] = (int64_t)k * cstride;
  LEM_TRY(upload(d_cb, cb.data(), cb.size() * sizeof(lem::KBlock), st));
  LEM_TRY(fill_weights(p, d_cb, cbk, st));
  LEM_TRY(upload(d_mcal, mc.data(), nr * sizeof(int), st));
  LEM_TRY(upload(d_jl, jl.data(), jl.size() * sizeof(int), st));
  LEM_TRY(upload(d_coff, coff.data(), nr * sizeof(int64_t), st));
  LEM_HIP(lem::launch_probe_fill(d_probe, op.N(), 12345u, st));
  LEM_TRY(launch_buckets(p, d_cb, cbk, 1, d_probe, nullptr, d_cv, d_cdiag, d_calib, 1, st));
  LEM_HIP(lem::launch_krylov_estimates(d_calib, d_mcal, d_coff, d_jl, (int)jl.size(), nsc,
                                       d_est, nr, mcal, st));
  std::vector<double> est((size_t)nr * nsc * jl.size());
  LEM_HIP(hipMemcpyAsync(est.data(), d_est, est.size() * 8, hipMemcpyDeviceToHost, st));
  LEM_HIP(hipStreamSynchronize(st));
  // per representative choice (calibration row r = representative r)
  std::vector<int> rm(nr), rs(nr);
  for (int r = 0; r < nr; ++r) {
    int mm = 0, ss = 0;
    const Box& rb = p->boxes[reps[r]];
    const int rnloc = box_lx(rb, op.n) * box_ly(rb, op.n, op.ndim) + (p->forced ? 1 : 0);
    if (!choose_m(&est[(size_t)r * nsc * jl.size()], jl, nsc, o.krylov_tol, o.krylov_m, mcal,
                  op.ndim, rnloc, &mm, &ss))
      return fail(LEM_ERR_NOT_CONVERGED,
                  "no Krylov dimension <= " + std::to_string(mcal) + " with <= " +
                      std::to_string(o.max_substeps) + " sub-steps meets krylov_tol");
    rm[r] = mm;
    rs[r] = ss;
  }
  for (void* q : {(void*)d_cb, (void*)d_probe, (void*)d_cv, (void*)d_calib, (void*)d_cdiag,
                  (void*)d_est, (void*)d_mcal, (void*)d_jl, (void*)d_coff})
    dfree(p, q);
  if (d_cw) dfree(p, d_cw);
  // step blocks
  p->m.resize(nb);
  p->nsub.resize(nb);
  std::vector<lem::KBlock> kb;
  for (int i = 0; i < nb; ++i) {
    p->m[i] = rm[rep[i]];
    p->nsub[i] = rs[rep[i]];
    kb.push_back(make_kblock(p, p->boxes[i], p->m[i], p->nsub[i], p->ns, i, p->forced));
  }
  int64_t vw = 0;
  LEM_TRY(bucketize(kb, p->buckets, p->ns, &vw));
  if (p->buckets.size() > 1 && !p->arena) {  // serving plans launch through the server
    const size_t ns_side = std::min<size_t>(p->buckets.size() - 1, 3);
    LEM_HIP(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
    for (size_t i = 0; i < ns_side; ++i) {
      hipStream_t s;
      hipEvent_t e;
      LEM_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      p->side.push_back(s);
      LEM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      p->ev_join.push_back(e);
    }
  }
  LEM_TRY(attach_weights(p, kb, p->buckets, &p->d_wts));
  p->kb_host = kb;
  LEM_TRY(dalloc(p, &p->d_kb, kb.size(), &p->bytes_work));
  LEM_TRY(upload(p->d_kb, kb.data(), kb.size() * sizeof(lem::KBlock), st));
  LEM_TRY(fill_weights(p, p->d_kb, p->buckets, st));
  LEM_TRY(dalloc(p, &p->d_vwork, (size_t)std::max<int64_t>(vw, 1), &p->bytes_work));
  LEM_TRY(dalloc(p, &p->d_diag, (size_t)nb * p->ns, &p->bytes_work));
  LEM_HIP(hipMemsetAsync(p->d_diag, 0, (size_t)nb * p->ns * 8, st));
  return LEM_OK;
}


}  // namespace lemh
