// Host-side entry points of the LEM kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "lem_device.hpp"

namespace lem {

// ---- Krylov calibration (krylov_calib.hip)
hipError_t launch_krylov_estimates(const double* calib, const int* mcal, const int64_t* coff,
                                   const int* jlist, int nj, int n_sub_cand, double* est,
                                   int n_blocks, int j_max, hipStream_t st);
hipError_t launch_probe_fill(double* x, int64_t n, uint64_t seed, hipStream_t st);

// ---- Krylov LEM step (krylov_lem.hip)
size_t krylov_lds_bytes(int nt, int m, int nloc, bool vlds, int aug);
// extra LDS of the wide streamed shapes for the staged diffusion coefficients
size_t krylov_stage_bytes(int nt, bool vlds, bool varcoef, bool varvel, int ndim, int lx,
                          int ly);
int krylov_lds_max_m();
void krylov_lds_config(int ndim, int nloc, int* nt, int* pmax);
hipError_t launch_krylov_lds(const KBlock* blocks, int n_blocks, int ns, int nt, int pmax,
                             bool vlds, size_t lds, const double* x_in, double* x_out,
                             const double* coef, double* vwork, double* diag, int* status,
                             double* calib, int mode, bool aug, hipStream_t st);

// ---- Krylov LEM step for large boxes / dimensions (krylov_big.hip): basis
// streamed through device memory, boxes of up to krylov_big_max_n() points
// (basis row, with the augmented coordinate), m <= krylov_big_max_m()
int krylov_big_max_m();
int krylov_big_max_n();
size_t krylov_big_lds_bytes(int nt, int pmax, int m);
// Fills the precomputed stencil weights of the blocks that carry them.
hipError_t launch_krylov_weights(const KBlock* blocks, int n_blocks, int nt, int pmax,
                                 const double* coef, hipStream_t st);
// doubles of padding after each block's basis slices (lanes past the box read
// past a row's end)
int64_t krylov_big_pad(int nt, int pmax);
void krylov_big_config(int nloc, int* nt, int* pmax);
hipError_t launch_krylov_big(const KBlock* blocks, int n_blocks, int ns, int nt, int pmax,
                             size_t lds, const double* x_in, double* x_out, const double* coef,
                             double* vwork, double* diag, int* status, double* calib, int mode,
                             bool aug, hipStream_t st);

// ---- Kronecker-factored local exponentials (kron.hip): one launch over
// blocks x member groups, box sides up to kron_max_side(), cores up to
// kron_max_core(); every block's c, L and ns bounded by max_c, max_L, max_ns
int kron_max_side();
int kron_max_core();
hipError_t launch_kron(const KronBlock* blocks, int n_blocks, int max_ns, int max_L, int max_c,
                       const double* x_in, double* x_out, int* status, hipStream_t st);

// ---- dense local exponentials (dense.hip)
size_t dense_op_size();
void dense_op_fill(void* dst, int i, double w0, double wW, double wE, double wS, double wN,
                   int Lx, int Ly);
hipError_t dense_assemble(const void* ops, double* A, int nl, int nu, hipStream_t st);
// variable coefficients: dt*A_M of count boxes from the face arrays
size_t dense_varbox_size();
void dense_varbox_fill(void* dst, int i, int ox, int oy, int h, int Lx, int Ly);
hipError_t dense_assemble_var(const double* mux, const double* muy, const double* ax,
                              const double* ay, double chx, double chy, int n, int ndim,
                              const void* boxes, int count, int nl, double* A, hipStream_t st);
hipError_t dense_assemble_aug(const void* ops, double* A, int nl, int nu, hipStream_t st);
hipError_t dense_norm1(const double* A, int nl, int nu, double* norms, hipStream_t st);
hipError_t dense_scale_pow2(double* A, int nl, int nu, const int* s, hipStream_t st);
hipError_t dense_gemm(const double* A, const double* B, double* C, int nl, int nu,
                      hipStream_t st);
hipError_t dense_lincomb(const double* X0, double c0, const double* X1, double c1,
                         const double* X2, double c2, const double* X3, double c3, double d,
                         double* out, int nl, int nu, hipStream_t st);
hipError_t dense_pade_pq(double* V, double* U, int64_t total, hipStream_t st);
hipError_t dense_solve(double* Q, double* P, int nl, int nu, hipStream_t st);
hipError_t dense_pack(const double* R, int nl, int Lx, int h, int cx, int cy, int ndim,
                      int rows, int rows_p, int cols_p, double* e64, float* e32, void* e16,
                      double* core_out, hipStream_t st);
size_t dense_block_size();
void dense_block_fill(void* dst, int i, int ox, int oy, int cx, int cy, int h, int Lx, int Ly,
                      int unique);
// Tile shapes of the FP64/FP32 apply (the autotuner times each at plan time);
// the split-bf16 apply has five: 32 or 64 rows per wave, four or eight waves
// per workgroup, 64 states per workgroup (ids 0-3) or 128 (id 4).
constexpr int kApplyConfigs = 8;
constexpr int kApplyBf16Configs = 5;
// Whether tile shape cfg of the apply serves this precision and padded block
// (cfg is ignored for ensembles that are not a multiple of 64).
bool dense_apply_supported(int precision, int cfg, int ns, int rows_p, int cols_p,
                           int64_t n_points);
// Split-bf16 precisions: xpieces (optional) holds the input state already
// split into bf16 pieces (dense_split_pieces, n_points x ns entries per piece).
// status: non-finite outputs latch kStatusNonFinite there (may be null).
hipError_t dense_apply(int precision, int cfg, const void* blocks, const void* E,
                       int64_t e_stride, const double* core, const double* x_in, double* x_out,
                       int n, int ndim, int ns, int rows, int rows_p, int cols, int cols_p,
                       int n_blocks, const double* bias, int* status, hipStream_t st,
                       const void* xpieces = nullptr, int64_t n_points = 0);
// Small 1D problems with one stored block (cores of `rows` points tiling the
// grid, boxes of cols = rows + 2h): every step of a lem_step call in one
// launch.  dense_resident_members returns the members per workgroup (0: the
// problem does not fit: rows outside [4, 128], cols > 128, or two states
// over LDS).
int dense_resident_members(int n, int ns, int rows, int cols, int nb);
hipError_t dense_resident_steps(const double* core, const double* bias, const double* x_in,
                                double* x_out, int* status, int n, int ns, int rows, int cols,
                                int nb, int h, int n_steps, hipStream_t st);
hipError_t dense_split_pieces(const double* x, int64_t total, int np, void* pieces,
                              hipStream_t st);

// ---- Schroedinger with a harmonic potential, real form (schrodinger.hip)
size_t sch_box_size();
void sch_box_fill(void* dst, int i, int ox, int h, int whole);
hipError_t sch_assemble(const void* boxes, int nb, int nl, int n, double L, double kappa,
                        double dt, double* A, hipStream_t st);

// ---- exponential Rosenbrock-Euler LEM for Burgers (rosenbrock.hip)
size_t ere_box_size();
void ere_box_fill(void* dst, int i, int ox, int h, int cx, int whole);
hipError_t ere_assemble(const double* x, const void* boxes, int nb, int ns, int nl, int n,
                        double dt, double dx, double nu, double* A, hipStream_t st);
hipError_t ere_extract(const double* R, const void* boxes, int nb, int ns, int nl, int rows,
                       double* Phi, hipStream_t st);
int ere_phi1_max_n();
// phi_1 core rows of every (block, member) for boxes of <= ere_phi1_max_n()
// points; P (nb * ns * rows * nl doubles) is work space, Phi the step layout.
hipError_t ere_phi1(const double* x, const void* boxes, int nb, int ns, int nl, int rows, int n,
                    double dt, double dx, double nu, double* P, double* Phi, int* sq_out,
                    int* status, hipStream_t st);
hipError_t ere_step(const double* x, double* f, const double* Phi, const void* boxes, int nb,
                    int ns, int nl, int rows, int n, double dt, double dx, double nu, double* y,
                    hipStream_t st);

// ---- global Krylov (global_krylov.hip)
struct GlobalWork {
  int64_t N;
  int ns, n, ndim, m, nsub;
  double w[5];
  double chx, chy, sub_scale;
  const double* mux;
  const double* muy;
  const double* ax;   // face velocity coefficients (conservative advection), or null
  const double* ay;
  double *V, *W, *Wt, *part, *h1, *h2, *hn, *H, *f, *beta, *inv, *est, *estsum;
  double tol;
  int* status;
  // forced steps (force != null): dt_sub scale of the forcing, and the
  // augmented input/output states ((N + 1) x ns each)
  const double* force;
  double gscale;
  double *xa, *ya;
};
int global_grid(int64_t total, int ns);
size_t global_part_doubles(int G, int ns);
hipError_t global_step(const GlobalWork& w, const double* x, double* y, hipStream_t st);
hipError_t global_arnoldi(const GlobalWork& w, const double* x, double* calib, hipStream_t st);

}  // namespace lem
