// Stored local exponentials (sections 3 and 4): the batched Pade / Taylor
// scaling and squaring on the device, dense blocks per distinct local
// operator (forcing terms, variable coefficients), the Kronecker-factored
// form for 2D constant coefficients, and the apply's launch-shape autotuner.
#include "host_internal.h"

namespace lemh {

constexpr double kB[14] = {64764752532480000.0, 32382376266240000.0, 7771770303897600.0,
                           1187353796428800.0,  129060195264000.0,   10559470521600.0,
                           670442572800.0,      33522128640.0,       1323241920.0,
                           40840800.0,          960960.0,            16380.0,
                           182.0,               1.0};


// ---------------------------------------------------------------- dense ----
// exp of the U assembled nl x nl matrices in A (overwritten) into R, by
// Pade [13/13] with scaling and squaring in float64 (Higham 2005): the powers,
// both polynomials and the squarings on FP64 MFMA, Q R = P by pivoted LU.
lem_status dense_expm_pade(lem_plan_s* p, double* A, double* R, int nl, int U, hipStream_t st,
                           int* smax, const std::vector<double*>* work, int* work_s) {
  const size_t mat = (size_t)nl * nl * U;
  double *A2, *A4, *A6, *T, *Ub, *d_norm;
  int* d_s;
  if (work) {  // caller-owned work space (kept between calls)
    A2 = (*work)[0]; A4 = (*work)[1]; A6 = (*work)[2]; T = (*work)[3]; Ub = (*work)[4];
    d_norm = (*work)[5];
    d_s = work_s;
  } else {
    LEM_TRY(dalloc(p, &A2, mat));
    LEM_TRY(dalloc(p, &A4, mat));
    LEM_TRY(dalloc(p, &A6, mat));
    LEM_TRY(dalloc(p, &T, mat));
    LEM_TRY(dalloc(p, &Ub, mat));
    LEM_TRY(dalloc(p, &d_norm, U));
    LEM_TRY(dalloc(p, &d_s, U));
  }
  LEM_HIP(lem::dense_norm1(A, nl, U, d_norm, st));
  std::vector<double> nrm(U);
  LEM_HIP(hipMemcpyAsync(nrm.data(), d_norm, U * 8, hipMemcpyDeviceToHost, st));
  LEM_HIP(hipStreamSynchronize(st));
  std::vector<int> s(U);
  for (int u = 0; u < U; ++u) {
    if (!std::isfinite(nrm[u])) return fail(LEM_ERR_INVALID, "non-finite local operator");
    s[u] = nrm[u] > lem::kTheta13 ? std::min(60, (int)std::ceil(std::log2(nrm[u] / lem::kTheta13))) : 0;
    *smax = std::max(*smax, s[u]);
  }
  LEM_TRY(upload(d_s, s.data(), U * sizeof(int), st));
  LEM_HIP(lem::dense_scale_pow2(A, nl, U, d_s, st));
  LEM_HIP(lem::dense_gemm(A, A, A2, nl, U, st));
  LEM_HIP(lem::dense_gemm(A2, A2, A4, nl, U, st));
  LEM_HIP(lem::dense_gemm(A4, A2, A6, nl, U, st));
  // U = A (A6 (b13 A6 + b11 A4 + b9 A2) + b7 A6 + b5 A4 + b3 A2 + b1 I)
  LEM_HIP(lem::dense_lincomb(A6, kB[13], A4, kB[11], A2, kB[9], nullptr, 0, 0, T, nl, U, st));
  LEM_HIP(lem::dense_gemm(A6, T, Ub, nl, U, st));
  LEM_HIP(lem::dense_lincomb(Ub, 1.0, A6, kB[7], A4, kB[5], A2, kB[3], kB[1], Ub, nl, U, st));
  LEM_HIP(lem::dense_gemm(A, Ub, T, nl, U, st));  // T = U
  // V = A6 (b12 A6 + b10 A4 + b8 A2) + b6 A6 + b4 A4 + b2 A2 + b0 I
  LEM_HIP(lem::dense_lincomb(A6, kB[12], A4, kB[10], A2, kB[8], nullptr, 0, 0, Ub, nl, U, st));
  LEM_HIP(lem::dense_gemm(A6, Ub, R, nl, U, st));
  LEM_HIP(lem::dense_lincomb(R, 1.0, A6, kB[6], A4, kB[4], A2, kB[2], kB[0], R, nl, U, st));
  LEM_HIP(lem::dense_pade_pq(R, T, (int64_t)mat, st));  // R = P, T = Q
  LEM_HIP(lem::dense_solve(T, R, nl, U, st));           // R = Q^-1 P
  for (int u = 0; u < U; ++u) {
    double* src = R + (size_t)u * nl * nl;
    double* dst = A2 + (size_t)u * nl * nl;
    for (int q = 0; q < s[u]; ++q) {
      LEM_HIP(lem::dense_gemm(src, src, dst, nl, 1, st));
      std::swap(src, dst);
    }
    if (src != R + (size_t)u * nl * nl)
      LEM_HIP(hipMemcpyAsync(R + (size_t)u * nl * nl, src, (size_t)nl * nl * 8,
                             hipMemcpyDeviceToDevice, st));
  }
  LEM_HIP(hipStreamSynchronize(st));
  if (!work)
    for (void* q : {(void*)A2, (void*)A4, (void*)A6, (void*)T, (void*)Ub, (void*)d_norm, (void*)d_s})
      dfree(p, q);
  return LEM_OK;
}

// exp of the U assembled nl x nl matrices in A (overwritten) into R by
// scaling and squaring with a Taylor polynomial: with X = A / 2^s scaled to
// ||X||_1 <= 1, T_18(X) = sum_{k<=18} X^k / k! (truncation below 1/19! ~ 9e-18
// relative) evaluated Paterson-Stockmeyer style as a polynomial in X^4 whose
// coefficients are c_{4j} I + c_{4j+1} X + c_{4j+2} X^2 + c_{4j+3} X^3 (seven
// products), then s squarings.  Every product is a batched FP64 MFMA GEMM:
// no factorization, so no latency-bound pivoting on the device.
lem_status dense_expm_taylor(lem_plan_s* p, double* A, double* R, int nl, int U, hipStream_t st,
                             int* smax, const std::vector<double*>* work, int* work_s) {
  const size_t mat = (size_t)nl * nl * U;
  double *A2, *A3, *A4, *T, *d_norm;
  int* d_s;
  std::vector<double*> own;
  if (work) {  // caller-owned work space (kept between calls)
    A2 = (*work)[0]; A4 = (*work)[1]; A3 = (*work)[2]; T = (*work)[3];
    d_norm = (*work)[5];
    d_s = work_s;
  } else {
    LEM_TRY(dalloc(p, &A2, mat));
    LEM_TRY(dalloc(p, &A3, mat));
    LEM_TRY(dalloc(p, &A4, mat));
    LEM_TRY(dalloc(p, &T, mat));
    LEM_TRY(dalloc(p, &d_norm, U));
    LEM_TRY(dalloc(p, &d_s, U));
  }
  LEM_HIP(lem::dense_norm1(A, nl, U, d_norm, st));
  std::vector<double> nrm(U);
  LEM_HIP(hipMemcpyAsync(nrm.data(), d_norm, U * 8, hipMemcpyDeviceToHost, st));
  LEM_HIP(hipStreamSynchronize(st));
  std::vector<int> s(U);
  // one scaling for the whole batch (the largest one needed), so that every
  // squaring is a single batched GEMM
  int sb = 0;
  for (int u = 0; u < U; ++u) {
    if (!std::isfinite(nrm[u])) return fail(LEM_ERR_INVALID, "non-finite local operator");
    sb = std::max(sb, nrm[u] > 1.0 ? std::min(60, (int)std::ceil(std::log2(nrm[u]))) : 0);
  }
  for (int u = 0; u < U; ++u) s[u] = sb;
  *smax = std::max(*smax, sb);
  double c[20];  // c[k] = 1 / k!
  c[0] = 1.0;
  for (int k = 1; k < 20; ++k) c[k] = c[k - 1] / k;
  LEM_TRY(upload(d_s, s.data(), U * sizeof(int), st));
  LEM_HIP(lem::dense_scale_pow2(A, nl, U, d_s, st));
  LEM_HIP(lem::dense_gemm(A, A, A2, nl, U, st));
  LEM_HIP(lem::dense_gemm(A2, A, A3, nl, U, st));
  LEM_HIP(lem::dense_gemm(A2, A2, A4, nl, U, st));
  // R = c16 I + c17 X + c18 X^2, then R <- R X^4 + c_{4j} I + ... + c_{4j+3} X^3
  LEM_HIP(lem::dense_lincomb(A, c[17], A2, c[18], nullptr, 0, nullptr, 0, c[16], R, nl, U, st));
  for (int j = 3; j >= 0; --j) {
    LEM_HIP(lem::dense_gemm(R, A4, T, nl, U, st));
    LEM_HIP(lem::dense_lincomb(T, 1.0, A, c[4 * j + 1], A2, c[4 * j + 2], A3, c[4 * j + 3],
                               c[4 * j], R, nl, U, st));
  }
  double* src = R;
  double* dst = A2;
  for (int q = 0; q < sb; ++q) {
    LEM_HIP(lem::dense_gemm(src, src, dst, nl, U, st));
    std::swap(src, dst);
  }
  if (src != R) LEM_HIP(hipMemcpyAsync(R, src, mat * 8, hipMemcpyDeviceToDevice, st));
  LEM_HIP(hipStreamSynchronize(st));
  if (!work)
    for (void* q : {(void*)A2, (void*)A3, (void*)A4, (void*)T, (void*)d_norm, (void*)d_s})
      dfree(p, q);
  return LEM_OK;
}

// exp of the U assembled nl x nl matrices in A (overwritten) into R, by the
// algorithm the plan asks for (Pade [13/13] by default).
lem_status dense_expm(lem_plan_s* p, double* A, double* R, int nl, int U, hipStream_t st,
                      int* smax, const std::vector<double*>* work, int* work_s) {
  return p->opt.expm == LEM_EXPM_TAYLOR ? dense_expm_taylor(p, A, R, nl, U, st, smax, work, work_s)
                                        : dense_expm_pade(p, A, R, nl, U, st, smax, work, work_s);
}

// The forcing term of a dense-method step, phi_1(dt A_M)(dt g_M) on every core,
// into p->d_bias: phi_1(dt A_M) is the top-right block of the exponential of
// [[dt A_M, I], [0, 0]]; its core rows are applied to dt g by the apply kernel.
lem_status dense_forcing_term(lem_plan_s* p, const void* d_ops, const double* host_g,
                              hipStream_t st) {
  const Op& op = p->op;
  const Box& b0 = p->boxes[0];
  const int Lx = b0.cx + 2 * b0.h, Ly = op.ndim == 2 ? b0.cy + 2 * b0.h : 1;
  const int nl = Lx * Ly, n2 = 2 * nl;
  double *Aa, *Ra, *Phi;
  LEM_TRY(dalloc(p, &Aa, (size_t)n2 * n2));
  LEM_TRY(dalloc(p, &Ra, (size_t)n2 * n2));
  LEM_HIP(lem::dense_assemble_aug(d_ops, Aa, nl, 1, st));
  int sq = 0;
  LEM_TRY(dense_expm(p, Aa, Ra, n2, 1, st, &sq));
  dfree(p, Aa);
  LEM_TRY(dalloc(p, &Phi, (size_t)nl * nl));
  LEM_HIP(hipMemcpy2DAsync(Phi, (size_t)nl * 8, Ra + nl, (size_t)n2 * 8, (size_t)nl * 8, nl,
                           hipMemcpyDeviceToDevice, st));
  dfree(p, Ra);
  const size_t es = (size_t)p->rows_p * p->cols_p;
  double *e64, *core, *dtg;
  float* e32;
  unsigned short* e16;
  LEM_TRY(dalloc(p, &e64, es));
  LEM_TRY(dalloc(p, &e32, es));
  LEM_TRY(dalloc(p, &e16, es * 3));
  LEM_TRY(dalloc(p, &core, (size_t)p->rows * nl));
  LEM_HIP(lem::dense_pack(Phi, nl, Lx, b0.h, b0.cx, op.ndim == 2 ? b0.cy : 1, op.ndim, p->rows,
                          p->rows_p, p->cols_p, e64, e32, e16, core, st));
  const size_t tot = (size_t)p->N * p->ns;
  std::vector<double> hg(tot);
  for (size_t e = 0; e < tot; ++e) hg[e] = op.dt * host_g[e];
  LEM_TRY(dalloc(p, &dtg, tot));
  LEM_TRY(upload(dtg, hg.data(), tot * 8, st));
  LEM_TRY(dalloc(p, &p->d_bias, tot, &p->bytes_work));
  LEM_HIP(lem::dense_apply(LEM_FP64, 0, p->d_db, e64, (int64_t)es, core, dtg, p->d_bias, op.n,
                           op.ndim, p->ns, p->rows, p->rows_p, p->cols, p->cols_p,
                           (int)p->boxes.size(), nullptr, nullptr, st));
  LEM_HIP(hipStreamSynchronize(st));
  for (void* q : {(void*)Phi, (void*)e64, (void*)e32, (void*)e16, (void*)core, (void*)dtg})
    dfree(p, q);
  return LEM_OK;
}

// Variable coefficients: every region has its own local operator, so every
// region gets its own stored block (the HBM holds them all: 3.8 GB for 1024
// blocks of 256 x 1792 in FP64).  All boxes take the largest buffer width of
// the partition (one block shape).  The blocks are assembled from the face
// arrays and exponentiated in chunks that bound the Pade work space.
lem_status plan_dense_variable(lem_plan_s* p, hipStream_t st) {
  const Op& op = p->op;
  int h = 0;
  for (const Box& b : p->boxes) h = std::max(h, b.h);
  for (Box& b : p->boxes) b.h = h;
  const Box& b0 = p->boxes[0];
  const int Lx = b0.cx + 2 * h, Ly = op.ndim == 2 ? b0.cy + 2 * h : 1;
  const int nl = Lx * Ly, nb = (int)p->boxes.size();
  p->U = nb;
  p->rows = b0.cx * (op.ndim == 2 ? b0.cy : 1);
  p->cols = nl;
  p->rows_p = (p->rows + 63) / 64 * 64;
  p->cols_p = (nl + 31) / 32 * 32;
  LEM_TRY(upload_coef(p, st));
  const size_t es = (size_t)p->rows_p * p->cols_p;
  LEM_TRY(dalloc(p, &p->d_e64, es * nb, &p->bytes_blocks));
  if (p->opt.precision == LEM_FP32) LEM_TRY(dalloc(p, &p->d_e32, es * nb, &p->bytes_blocks));
  if (p->ns % 64) LEM_TRY(dalloc(p, &p->d_core, (size_t)p->rows * nl * nb, &p->bytes_blocks));
  // chunk of blocks per Pade batch: seven nl x nl matrices each, within ~24 GB
  const size_t per = (size_t)nl * nl * 8;
  const int chunk = (int)std::max<size_t>(1, std::min<size_t>(nb, (size_t)(24ull << 30) / (7 * per)));
  double *A = nullptr, *Vb = nullptr;
  std::vector<double*> work;
  int* work_s = nullptr;
  unsigned char* dvb = nullptr;
  auto cleanup = [&]() {
    for (void* q : {(void*)A, (void*)Vb, (void*)work_s, (void*)dvb})
      if (q) dfree(p, q);
    for (double* w : work) dfree(p, w);
  };
  lem_status s = dalloc(p, &A, (size_t)chunk * nl * nl);
  if (s == LEM_OK) s = dalloc(p, &Vb, (size_t)chunk * nl * nl);
  for (int q = 0; q < 5 && s == LEM_OK; ++q) {
    double* w;
    s = dalloc(p, &w, (size_t)chunk * nl * nl);
    if (s == LEM_OK) work.push_back(w);
  }
  if (s == LEM_OK) {
    double* w;
    s = dalloc(p, &w, (size_t)chunk);
    if (s == LEM_OK) work.push_back(w);
  }
  if (s == LEM_OK) s = dalloc(p, &work_s, (size_t)chunk);
  if (s == LEM_OK) s = dalloc(p, &dvb, lem::dense_varbox_size() * nb);
  std::vector<unsigned char> hvb(lem::dense_varbox_size() * nb);
  for (int i = 0; i < nb; ++i) {
    const Box& b = p->boxes[i];
    lem::dense_varbox_fill(hvb.data(), i, b.ox, b.oy, h, Lx, Ly);
  }
  if (s == LEM_OK) s = upload(dvb, hvb.data(), hvb.size(), st);
  const size_t N = (size_t)op.N();
  for (int u0 = 0; u0 < nb && s == LEM_OK; u0 += chunk) {
    const int cnt = std::min(chunk, nb - u0);
    if (lem::dense_assemble_var(p->d_coef, p->d_coef + N, op.varvel ? p->d_coef + 2 * N : nullptr,
                                op.varvel ? p->d_coef + 3 * N : nullptr, op.chx, op.chy, op.n,
                                op.ndim, dvb + lem::dense_varbox_size() * u0, cnt, nl, A,
                                st) != hipSuccess) {
      s = fail(LEM_ERR_HIP, "variable assembly failed");
      break;
    }
    s = dense_expm(p, A, Vb, nl, cnt, st, &p->squarings, &work, work_s);
    for (int u = u0; u < u0 + cnt && s == LEM_OK; ++u)
      if (lem::dense_pack(Vb + (size_t)(u - u0) * nl * nl, nl, Lx, h, b0.cx,
                          op.ndim == 2 ? b0.cy : 1, op.ndim, p->rows, p->rows_p, p->cols_p,
                          p->d_e64 + u * es, p->d_e32 ? p->d_e32 + u * es : nullptr, nullptr,
                          p->d_core ? p->d_core + (size_t)u * p->rows * nl : nullptr,
                          st) != hipSuccess)
        s = fail(LEM_ERR_HIP, "block packing failed");
  }
  if (s == LEM_OK && hipStreamSynchronize(st) != hipSuccess)
    s = fail(LEM_ERR_HIP, "plan synchronization failed");
  cleanup();
  if (s != LEM_OK) return s;
  std::vector<unsigned char> db(lem::dense_block_size() * nb);
  for (int i = 0; i < nb; ++i) {
    const Box& b = p->boxes[i];
    lem::dense_block_fill(db.data(), i, b.ox, b.oy, b.cx, op.ndim == 2 ? b.cy : 1, h, Lx, Ly, i);
  }
  {
    unsigned char* d;
    LEM_TRY(dalloc(p, &d, db.size(), &p->bytes_work));
    p->d_db = d;
  }
  LEM_TRY(upload(p->d_db, db.data(), db.size(), st));
  p->tile = p->opt.precision == LEM_FP32 ? 2 : 0;
  return LEM_OK;
}

lem_status plan_dense(lem_plan_s* p, hipStream_t st, const double* host_g) {
  const Op& op = p->op;
  if (op.variable) return plan_dense_variable(p, st);
  if (p->opt.core <= 0) return fail(LEM_ERR_INVALID, "the dense method needs a uniform core");
  if (p->opt.precision >= LEM_BF16X2 && p->ns % 64)
    return fail(LEM_ERR_UNSUPPORTED, "bf16 split application needs n_states % 64 == 0");
  const Box& b0 = p->boxes[0];
  const int Lx = b0.cx + 2 * b0.h, Ly = op.ndim == 2 ? b0.cy + 2 * b0.h : 1;
  const int nl = Lx * Ly;
  // every box of a uniform partition of a constant operator has the same
  // local operator: one stored block, shared by all
  p->U = 1;
  const int U = 1;
  p->rows = b0.cx * (op.ndim == 2 ? b0.cy : 1);
  p->cols = nl;
  p->rows_p = (p->rows + 63) / 64 * 64;
  p->cols_p = (nl + 31) / 32 * 32;
  const size_t mat = (size_t)nl * nl * U;
  double *A, *Vb;
  void* d_ops;
  LEM_TRY(dalloc(p, &A, mat));
  LEM_TRY(dalloc(p, &Vb, mat));
  {
    unsigned char* dp;
    LEM_TRY(dalloc(p, &dp, lem::dense_op_size() * U));
    d_ops = dp;
  }
  std::vector<unsigned char> hops(lem::dense_op_size() * U);
  lem::dense_op_fill(hops.data(), 0, op.w[0], op.w[1], op.w[2], op.w[3], op.w[4], Lx, Ly);
  LEM_TRY(upload(d_ops, hops.data(), hops.size(), st));
  LEM_HIP(lem::dense_assemble(d_ops, A, nl, U, st));
  LEM_TRY(dense_expm(p, A, Vb, nl, U, st, &p->squarings));
  const size_t es = (size_t)p->rows_p * p->cols_p;
  LEM_TRY(dalloc(p, &p->d_e64, es * U, &p->bytes_blocks));
  LEM_TRY(dalloc(p, &p->d_e32, es * U, &p->bytes_blocks));
  {
    unsigned short* e16;
    LEM_TRY(dalloc(p, &e16, es * 3 * U, &p->bytes_blocks));
    p->d_e16 = e16;
  }
  LEM_TRY(dalloc(p, &p->d_core, (size_t)p->rows * nl * U, &p->bytes_blocks));
  for (int u = 0; u < U; ++u)
    LEM_HIP(lem::dense_pack(Vb + (size_t)u * nl * nl, nl, Lx, b0.h, b0.cx, op.ndim == 2 ? b0.cy : 1,
                            op.ndim, p->rows, p->rows_p, p->cols_p, p->d_e64 + u * es,
                            p->d_e32 + u * es, (unsigned short*)p->d_e16 + u * es * 3,
                            p->d_core + (size_t)u * p->rows * nl, st));
  LEM_HIP(hipStreamSynchronize(st));
  for (void* q : {(void*)A, (void*)Vb}) dfree(p, q);
  // (d_ops is kept until the forcing term is built)
  // block table
  const int nb = (int)p->boxes.size();
  std::vector<unsigned char> db(lem::dense_block_size() * nb);
  for (int i = 0; i < nb; ++i) {
    const Box& b = p->boxes[i];
    lem::dense_block_fill(db.data(), i, b.ox, b.oy, b.cx, op.ndim == 2 ? b.cy : 1, b.h,
                          b.cx + 2 * b.h, op.ndim == 2 ? b.cy + 2 * b.h : 1, 0);
  }
  {
    unsigned char* d;
    LEM_TRY(dalloc(p, &d, db.size(), &p->bytes_work));
    p->d_db = d;
  }
  LEM_TRY(upload(p->d_db, db.data(), db.size(), st));
  if (p->forced) LEM_TRY(dense_forcing_term(p, d_ops, host_g, st));
  dfree(p, d_ops);
  // default tile shape of the apply kernel (the autotuner may replace it)
  p->tile = p->opt.precision == LEM_FP32 ? 2 : p->opt.precision == LEM_FP64 ? 0 : (p->rows_p >= 256 ? 1 : 0);
  if (p->opt.precision >= LEM_BF16X2) {  // pieces of the state, split once per step
    const int np = p->opt.precision == LEM_BF16X3 ? 4 : 2;  // pieces per entry (3 padded to 4)
    unsigned short* xp;
    LEM_TRY(dalloc(p, &xp, (size_t)np * p->N * p->ns, &p->bytes_work));
    p->d_xp = xp;
  }
  return LEM_OK;
}

const void* dense_operand(const lem_plan_s* p) {
  switch (p->opt.precision) {
    case LEM_FP64: return p->d_e64;
    case LEM_FP32: return p->d_e32;
    default: return p->d_e16;
  }
}

// ------------------------------------------------------------ Kronecker ----
// The 2D constant-coefficient box matrix is the Kronecker sum of the 1D
// tridiagonal matrices of dt*A along x (west, centre, east weights) and y
// (south, centre, north), each with the couplings leaving the box dropped;
// their exponentials are computed once (opt.expm) and their core rows kept.
lem_status plan_kron(lem_plan_s* p, hipStream_t st) {
  const Op& op = p->op;
  if (op.ndim != 2 || op.variable || p->forced || p->opt.precision != LEM_FP64)
    return fail(LEM_ERR_UNSUPPORTED, "the Kronecker-factored method takes a 2D constant-coefficient "
                                     "operator, FP64 and no forcing");
  const Box& b0 = p->boxes[0];
  const int c = b0.cx, h = b0.h, L = c + 2 * h;
  if (L > lem::kron_max_side() || c > lem::kron_max_core())
    return fail(LEM_ERR_UNSUPPORTED, "Kronecker-factored boxes are at most " +
                                         std::to_string(lem::kron_max_side()) +
                                         " points per side, cores at most " +
                                         std::to_string(lem::kron_max_core()));
  const double mux = op.nu * op.dt / (op.dx * op.dx), muy = op.nu * op.dt / (op.dy * op.dy);
  std::vector<double> hA((size_t)2 * L * L, 0.0);
  double* Ax = hA.data();
  double* Ay = hA.data() + (size_t)L * L;
  for (int i = 0; i < L; ++i) {
    Ax[(size_t)i * L + i] = -(mux + mux);
    Ay[(size_t)i * L + i] = -(muy + muy);
    if (i > 0) {
      Ax[(size_t)i * L + i - 1] = op.w[1];
      Ay[(size_t)i * L + i - 1] = op.w[3];
    }
    if (i + 1 < L) {
      Ax[(size_t)i * L + i + 1] = op.w[2];
      Ay[(size_t)i * L + i + 1] = op.w[4];
    }
  }
  double *A, *R;
  LEM_TRY(dalloc(p, &A, hA.size()));
  LEM_TRY(dalloc(p, &R, hA.size()));
  LEM_TRY(upload(A, hA.data(), hA.size() * 8, st));
  LEM_TRY(dense_expm(p, A, R, L, 2, st, &p->squarings));
  LEM_TRY(dalloc(p, &p->d_ex, (size_t)2 * c * L, &p->bytes_blocks));
  LEM_HIP(hipMemcpyAsync(p->d_ex, R + (size_t)h * L, (size_t)c * L * 8, hipMemcpyDeviceToDevice, st));
  LEM_HIP(hipMemcpyAsync(p->d_ex + (size_t)c * L, R + (size_t)L * L + (size_t)h * L,
                         (size_t)c * L * 8, hipMemcpyDeviceToDevice, st));
  std::vector<lem::KronBlock> kb;
  for (const Box& b : p->boxes) {
    lem::KronBlock k{};
    k.ox = b.ox; k.oy = b.oy; k.c = c; k.h = h; k.L = L; k.n = op.n; k.ns = p->ns;
    k.ex = p->d_ex;
    k.ey = p->d_ex + (size_t)c * L;
    kb.push_back(k);
  }
  LEM_TRY(dalloc(p, &p->d_kron, kb.size(), &p->bytes_work));
  LEM_TRY(upload(p->d_kron, kb.data(), kb.size() * sizeof(lem::KronBlock), st));
  LEM_HIP(hipStreamSynchronize(st));
  dfree(p, A);
  dfree(p, R);
  p->U = 1;
  p->kron_L = L;
  return LEM_OK;
}

// Launch shape of the dense apply: the caller's (opt.tile >= 0, checked
// against the block), else the fastest one timed at plan time (autotune),
// else the plan's default.
lem_status choose_tile(lem_plan_s* p, hipStream_t st);

// Times the dense apply at every launch shape on a scratch state; keeps the fastest.
lem_status autotune_dense(lem_plan_s* p, hipStream_t st) {
  const int64_t tot = p->N * p->ns;
  double *a, *b;
  LEM_TRY(dalloc(p, &a, (size_t)tot));
  LEM_TRY(dalloc(p, &b, (size_t)tot));
  LEM_HIP(lem::launch_probe_fill(a, tot, 99u, st));
  hipEvent_t e0, e1;
  LEM_HIP(hipEventCreate(&e0));
  LEM_HIP(hipEventCreate(&e1));
  float best = INFINITY;
  int besttile = p->tile;
  const int ntile = p->opt.precision <= LEM_FP32 ? lem::kApplyConfigs : lem::kApplyBf16Configs;
  for (int tile = 0; tile < ntile; ++tile) {
    if (!lem::dense_apply_supported(p->opt.precision, tile, p->ns, p->rows_p, p->cols_p, p->N))
      continue;
    p->tile = tile;
    if (run_one(p, a, b, st) != LEM_OK) continue;
    LEM_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < 5; ++r) LEM_TRY(run_one(p, a, b, st));
    LEM_HIP(hipEventRecord(e1, st));
    LEM_HIP(hipEventSynchronize(e1));
    float ms = 0;
    LEM_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (ms < best) { best = ms; besttile = tile; }
  }
  p->tile = besttile;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  dfree(p, a);
  dfree(p, b);
  // the timing runs wrote the plan's status word: start clean
  LEM_HIP(hipMemsetAsync(p->d_status, 0, sizeof(int), st));
  return LEM_OK;
}

lem_status choose_tile(lem_plan_s* p, hipStream_t st) {
  if (p->opt.tile >= 0) {
    if (!lem::dense_apply_supported(p->opt.precision, p->opt.tile, p->ns, p->rows_p, p->cols_p,
                                    p->N))
      return fail(LEM_ERR_UNSUPPORTED, "apply tile shape " + std::to_string(p->opt.tile) +
                                           " does not fit this block and precision");
    p->tile = p->opt.tile;
    return LEM_OK;
  }
  if (p->opt.autotune && p->ns % 64 == 0) return autotune_dense(p, st);
  return LEM_OK;
}


}  // namespace lemh
