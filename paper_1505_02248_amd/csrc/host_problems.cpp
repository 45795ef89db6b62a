// Problem-specific planners: exponential Rosenbrock-Euler LEM for viscous
// Burgers (section 4.2) and the complex Schroedinger operator (section 4.1).
#include "host_internal.h"

namespace lemh {

// ----------------------------------------------------- exponential Rosenbrock
// phi_1(dt J_M) of every (block, member) at the state x (Jacobian refresh).
lem_status ere_refresh(lem_plan_s* p, const double* x, hipStream_t st) {
  const int nb = (int)p->boxes.size(), U = nb * p->ns, n2 = 2 * p->ere_nl;
  if (p->ere_small) {
    LEM_HIP(lem::ere_phi1(x, p->d_ere_boxes, nb, p->ns, p->ere_nl, p->ere_rows, p->op.n, p->op.dt,
                          p->ere_dx, p->ere_nu, p->d_ere_R, p->d_phi, p->d_ere_s, p->d_status,
                          st));
    return LEM_OK;
  }
  LEM_HIP(lem::ere_assemble(x, p->d_ere_boxes, nb, p->ns, p->ere_nl, p->op.n, p->op.dt,
                            p->ere_dx, p->ere_nu, p->d_ere_A, st));
  int sq = 0;
  LEM_TRY(dense_expm(p, p->d_ere_A, p->d_ere_R, n2, U, st, &sq, &p->ere_work, p->d_ere_s));
  p->squarings = std::max(p->squarings, sq);
  LEM_HIP(lem::ere_extract(p->d_ere_R, p->d_ere_boxes, nb, p->ns, p->ere_nl, p->ere_rows,
                           p->d_phi, st));
  return LEM_OK;
}

lem_status ere_run_one(lem_plan_s* p, const double* src, double* dst, hipStream_t st) {
  if (p->ere_count % p->ere_refresh == 0) LEM_TRY(ere_refresh(p, src, st));
  LEM_HIP(lem::ere_step(src, p->d_f, p->d_phi, p->d_ere_boxes, (int)p->boxes.size(), p->ns,
                        p->ere_nl, p->ere_rows, p->op.n, p->op.dt, p->ere_dx, p->ere_nu, dst, st));
  p->ere_count++;
  return LEM_OK;
}


}  // namespace lemh

using namespace lemh;

extern "C" {

lem_status lem_ere_plan(const lem_burgers* op, double dt, int32_t n_states, int32_t core,
                        int32_t halo, int32_t refresh, void* stream, lem_plan_t* out) {
  if (!op || !out) return fail(LEM_ERR_INVALID, "NULL argument");
  *out = nullptr;
  if (op->n < 3) return fail(LEM_ERR_INVALID, "n must be >= 3");
  if (!(op->dx > 0) || !std::isfinite(op->dx)) return fail(LEM_ERR_INVALID, "dx must be > 0");
  if (!(op->nu >= 0) || !std::isfinite(op->nu)) return fail(LEM_ERR_INVALID, "nu must be >= 0");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(LEM_ERR_INVALID, "dt must be > 0");
  if (n_states < 1 || refresh < 1) return fail(LEM_ERR_INVALID, "n_states, refresh must be >= 1");
  if (core < 1 || op->n % core != 0 || halo < 0)
    return fail(LEM_ERR_INVALID, "core must divide n and halo be >= 0");
  const bool whole = core == op->n && halo == 0;
  if (!whole && core + 2 * halo >= op->n)
    return fail(LEM_ERR_INVALID, "a box must be smaller than the grid (or core = n, halo = 0)");
  const auto t0 = std::chrono::steady_clock::now();
  auto p = new lem_plan_s();
  auto guard = [&](lem_status s) { if (s != LEM_OK) delete p; return s; };
  lem_options_default(&p->opt);
  p->opt.method = LEM_METHOD_ROSENBROCK;
  p->opt.expm = LEM_EXPM_TAYLOR;  // a refresh of large boxes recurs: GEMM-only pipeline
  p->opt.n_states = n_states;
  p->opt.core = core;
  p->opt.halo = halo;
  p->method = LEM_METHOD_ROSENBROCK;
  p->ns = n_states;
  p->stream = (hipStream_t)stream;
  p->op.ndim = 1;
  p->op.n = op->n;
  p->op.dx = op->dx;
  p->op.dt = dt;
  p->op.nu = op->nu;
  p->N = op->n;
  p->ere_dx = op->dx;
  p->ere_nu = op->nu;
  p->ere_refresh = refresh;
  p->ere_nl = core + 2 * halo;
  p->ere_rows = core;
  const int nb = op->n / core;
  for (int b = 0; b < nb; ++b) p->boxes.push_back({b * core, 0, core, 1, halo});
  hipStream_t st = p->stream;
  const int nl = p->ere_nl, n2 = 2 * nl, U = nb * n_states;
  const size_t mat = (size_t)n2 * n2 * U;
  std::vector<unsigned char> hb(lem::ere_box_size() * nb);
  for (int b = 0; b < nb; ++b) lem::ere_box_fill(hb.data(), b, b * core, halo, core, whole ? 1 : 0);
  lem_status s = dalloc(p, &p->d_status, 1);
  if (s == LEM_OK && hipMemsetAsync(p->d_status, 0, sizeof(int), st) != hipSuccess)
    s = fail(LEM_ERR_HIP, "hipMemsetAsync failed");
  if (s == LEM_OK) s = dalloc(p, &p->d_tmp, (size_t)p->N * p->ns, &p->bytes_work);
  if (s == LEM_OK) {
    unsigned char* d;
    s = dalloc(p, &d, hb.size(), &p->bytes_work);
    p->d_ere_boxes = d;
  }
  if (s == LEM_OK) s = upload(p->d_ere_boxes, hb.data(), hb.size(), st);
  // boxes of up to ere_phi1_max_n() points: phi_1 per (block, member) in one
  // LDS-resident launch; larger ones: the batched Pade pipeline on the
  // augmented matrices [[dt J_M, I], [0, 0]]
  p->ere_small = nl <= lem::ere_phi1_max_n();
  if (p->ere_small && s == LEM_OK)  // member-major phi_1 rows before the transpose
    s = dalloc(p, &p->d_ere_R, (size_t)nb * core * nl * n_states, &p->bytes_work);
  if (!p->ere_small) {
    if (s == LEM_OK) s = dalloc(p, &p->d_ere_A, mat, &p->bytes_work);
    if (s == LEM_OK) s = dalloc(p, &p->d_ere_R, mat, &p->bytes_work);
    for (int q = 0; q < 5 && s == LEM_OK; ++q) {
      double* w;
      s = dalloc(p, &w, mat, &p->bytes_work);
      p->ere_work.push_back(w);
    }
    if (s == LEM_OK) {
      double* w;
      s = dalloc(p, &w, (size_t)U, &p->bytes_work);
      p->ere_work.push_back(w);
    }
  }
  if (s == LEM_OK) s = dalloc(p, &p->d_ere_s, (size_t)U, &p->bytes_work);
  if (s == LEM_OK) s = dalloc(p, &p->d_phi, (size_t)nb * core * nl * n_states, &p->bytes_blocks);
  if (s == LEM_OK) s = dalloc(p, &p->d_f, (size_t)p->N * p->ns, &p->bytes_work);
  if (s == LEM_OK && hipStreamSynchronize(st) != hipSuccess)
    s = fail(LEM_ERR_HIP, "plan synchronization failed");
  if (s != LEM_OK) return guard(s);
  p->plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = p;
  return LEM_OK;
}

lem_status lem_schrodinger_plan(const lem_schrodinger* op, double dt, int32_t n_states,
                                int32_t core, int32_t halo, int32_t autotune, void* stream,
                                lem_plan_t* out) {
  if (!op || !out) return fail(LEM_ERR_INVALID, "NULL argument");
  *out = nullptr;
  if (op->n < 3) return fail(LEM_ERR_INVALID, "n must be >= 3");
  if (!(op->L > 0) || !std::isfinite(op->L)) return fail(LEM_ERR_INVALID, "L must be > 0");
  if (!(op->kappa >= 0) || !std::isfinite(op->kappa))
    return fail(LEM_ERR_INVALID, "kappa must be >= 0");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(LEM_ERR_INVALID, "dt must be > 0");
  if (n_states < 1) return fail(LEM_ERR_INVALID, "n_states must be >= 1");
  if (core < 1 || op->n % core != 0 || halo < 0)
    return fail(LEM_ERR_INVALID, "core must divide n and halo be >= 0");
  const bool whole = core == op->n && halo == 0;
  if (!whole && core + 2 * halo >= op->n)
    return fail(LEM_ERR_INVALID, "a box must be smaller than the grid (or core = n, halo = 0)");
  const int nl = core + 2 * halo, m = 2 * nl, nb = op->n / core;
  if (m > 4096) return fail(LEM_ERR_UNSUPPORTED, "local blocks above 2048 nodes");
  const auto t0 = std::chrono::steady_clock::now();
  auto p = new lem_plan_s();
  auto guard = [&](lem_status s) { if (s != LEM_OK) delete p; return s; };
  lem_options_default(&p->opt);
  p->opt.method = LEM_METHOD_DENSE;
  p->opt.precision = LEM_FP64;
  p->opt.n_states = n_states;
  p->opt.core = 2 * core;
  p->opt.halo = 2 * halo;
  p->method = LEM_METHOD_DENSE;
  p->ns = n_states;
  p->stream = (hipStream_t)stream;
  // the real form lives on a doubled 1D grid: node j holds entries 2j, 2j + 1
  p->op.ndim = 1;
  p->op.n = 2 * op->n;
  p->op.dx = op->L / op->n;
  p->op.dt = dt;
  p->N = 2 * op->n;
  for (int b = 0; b < nb; ++b) p->boxes.push_back({2 * b * core, 0, 2 * core, 1, 2 * halo});
  p->U = nb;
  p->rows = 2 * core;
  p->cols = m;
  p->rows_p = (p->rows + 63) / 64 * 64;
  p->cols_p = (m + 31) / 32 * 32;
  hipStream_t st = p->stream;
  lem_status s = dalloc(p, &p->d_status, 1);
  if (s == LEM_OK && hipMemsetAsync(p->d_status, 0, sizeof(int), st) != hipSuccess)
    s = fail(LEM_ERR_HIP, "hipMemsetAsync failed");
  if (s == LEM_OK) s = dalloc(p, &p->d_tmp, (size_t)p->N * p->ns, &p->bytes_work);
  if (s != LEM_OK) return guard(s);
  // local matrices of every region (the potential makes each one distinct)
  const size_t mat = (size_t)m * m * nb;
  double *A = nullptr, *Vb = nullptr;
  unsigned char* dboxes = nullptr;
  std::vector<unsigned char> hb(lem::sch_box_size() * nb);
  for (int b = 0; b < nb; ++b) lem::sch_box_fill(hb.data(), b, b * core, halo, whole ? 1 : 0);
  s = dalloc(p, &A, mat);
  if (s == LEM_OK) s = dalloc(p, &Vb, mat);
  if (s == LEM_OK) s = dalloc(p, &dboxes, hb.size());
  if (s == LEM_OK) s = upload(dboxes, hb.data(), hb.size(), st);
  if (s == LEM_OK && lem::sch_assemble(dboxes, nb, nl, op->n, op->L, op->kappa, dt, A, st) != hipSuccess)
    s = fail(LEM_ERR_HIP, "Schroedinger assembly failed");
  if (s == LEM_OK) s = dense_expm(p, A, Vb, m, nb, st, &p->squarings);
  const size_t es = (size_t)p->rows_p * p->cols_p;
  if (s == LEM_OK) s = dalloc(p, &p->d_e64, es * nb, &p->bytes_blocks);
  if (s == LEM_OK) s = dalloc(p, &p->d_e32, es * nb, &p->bytes_blocks);
  if (s == LEM_OK) {
    unsigned short* e16;
    s = dalloc(p, &e16, es * 3 * nb, &p->bytes_blocks);
    p->d_e16 = e16;
  }
  if (s == LEM_OK) s = dalloc(p, &p->d_core, (size_t)p->rows * m * nb, &p->bytes_blocks);
  for (int u = 0; u < nb && s == LEM_OK; ++u)
    if (lem::dense_pack(Vb + (size_t)u * m * m, m, m, 2 * halo, 2 * core, 1, 1, p->rows, p->rows_p,
                        p->cols_p, p->d_e64 + u * es, p->d_e32 + u * es,
                        (unsigned short*)p->d_e16 + u * es * 3, p->d_core + (size_t)u * p->rows * m,
                        st) != hipSuccess)
      s = fail(LEM_ERR_HIP, "block packing failed");
  if (s == LEM_OK && hipStreamSynchronize(st) != hipSuccess)
    s = fail(LEM_ERR_HIP, "plan synchronization failed");
  for (void* q : {(void*)A, (void*)Vb, (void*)dboxes})
    if (q) dfree(p, q);
  if (s != LEM_OK) return guard(s);
  std::vector<unsigned char> db(lem::dense_block_size() * nb);
  for (int i = 0; i < nb; ++i)
    lem::dense_block_fill(db.data(), i, 2 * i * core, 0, 2 * core, 1, 2 * halo, m, 1, i);
  {
    unsigned char* d;
    s = dalloc(p, &d, db.size(), &p->bytes_work);
    p->d_db = d;
  }
  if (s == LEM_OK) s = upload(p->d_db, db.data(), db.size(), st);
  p->tile = 0;
  p->opt.autotune = autotune ? 1 : 0;
  if (s == LEM_OK) s = choose_tile(p, st);
  if (s == LEM_OK && hipStreamSynchronize(st) != hipSuccess)
    s = fail(LEM_ERR_HIP, "plan synchronization failed");
  if (s != LEM_OK) return guard(s);
  p->plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = p;
  return LEM_OK;
}

}  // extern "C"
