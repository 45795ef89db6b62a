// Internal declarations shared by the host sources of the LEM library: the
// semi-discrete operator, the partition with decay-bound buffers, the plan
// object and the planning / stepping routines of every method.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <limits>
#include <map>
#include <string>
#include <tuple>
#include <utility>
#include <vector>

#include "arena.h"
#include "lem.h"
#include "lem_internal.h"
#include "lem_launch.h"

namespace lemh {

// Records msg as the thread's last error (lem_last_error) and returns s.
lem_status fail(lem_status s, const std::string& msg);
const char* g_err_text();

#define LEM_HIP(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return ::lemh::fail(LEM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define LEM_TRY(expr)                \
  do {                               \
    lem_status s_ = (expr);          \
    if (s_ != LEM_OK) return s_;     \
  } while (0)

// dt*A of the periodic advection-diffusion operator, centered differences.
struct Op {
  int ndim = 1, n = 0;
  double dx = 0, dy = 0, dt = 0, vel[2] = {0, 0}, nu = 0;
  bool variable = false;
  bool varvel = false;             // face velocities (conservative advection)
  double w[5] = {0, 0, 0, 0, 0};  // w0, wW, wE, wS, wN (constant case)
  double chx = 0, chy = 0;        // dt*C/2 per axis
  std::vector<double> mux, muy;   // face mu's (variable case), dt-scaled
  std::vector<double> ax, ay;     // face dt*a/(2 dx), dt*a/(2 dy) (varvel)
  int64_t N() const { return ndim == 1 ? (int64_t)n : (int64_t)n * n; }
};

lem_status build_op(const lem_operator* o, double dt, Op* op);
// Weights w0, wW, wE, wS, wN of the row of global point (i, j).
void point_weights(const Op& op, int i, int j, double* w);

struct BlockCoef { double aW, aE, aS, aN, w0; };
double eps_bound(const BlockCoef& c, int h, int ndim, double G, bool cut_y = true);
double growth_factor(const Op& op);

struct Box { int ox, oy, cx, cy, h; };

// Buffer widths per axis: none along an axis the core spans whole (column-
// wise decompositions, and the D = 1 box), which keeps the periodic coupling
// along that axis inside the box.
inline int box_hx(const Box& b, int n) { return b.cx == n ? 0 : b.h; }
inline int box_hy(const Box& b, int n, int ndim) { return ndim == 2 ? (b.cy == n ? 0 : b.h) : 0; }
inline int box_lx(const Box& b, int n) { return b.cx + 2 * box_hx(b, n); }
inline int box_ly(const Box& b, int n, int ndim) { return ndim == 2 ? b.cy + 2 * box_hy(b, n, ndim) : 1; }

BlockCoef block_coef(const Op& op, const Box& b, int h);
double block_rho(const Op& op, const Box& b);
int halo_from_bound(const Op& op, Box b, double tol, int h_min, int h_max, double G,
                    bool* clamped);

}  // namespace lemh

// ================================================================= plan ====
struct lem_plan_s {
  lemh::Op op;
  lem_options opt{};
  int method = 0, ns = 1;
  bool global_box = false;  // global method run as one periodic Krylov box
  int64_t N = 0;
  std::vector<lemh::Box> boxes;
  int n_clamped = 0;
  bool dry = false;
  // Krylov
  std::vector<int> m, nsub;
  struct Bucket { int variant, nt, pmax; bool vlds; size_t lds; int first, count; double cost; };
  std::vector<Bucket> buckets;
  // the step launches the costliest bucket on the caller's stream and the
  // others on side streams forked from it and joined back (the launches then
  // share the CUs that one bucket alone leaves idle)
  std::vector<hipStream_t> side;
  std::vector<hipEvent_t> ev_join;
  hipEvent_t ev_fork = nullptr;
  lem::KBlock* d_kb = nullptr;
  double* d_coef = nullptr;
  double* d_vwork = nullptr;
  double* d_wts = nullptr;     // precomputed stencil weights of large Krylov boxes
  double* d_diag = nullptr;
  // dense
  int U = 0, rows = 0, rows_p = 0, cols = 0, cols_p = 0, tile = 0, squarings = 0;
  void* d_db = nullptr;
  double* d_e64 = nullptr;
  float* d_e32 = nullptr;
  void* d_e16 = nullptr;
  void* d_xp = nullptr;  // split-bf16: the input state in bf16 pieces, once per step
  double* d_core = nullptr;
  // forcing (du/dt = A u + g, g constant in time): device copy of g and, for
  // the dense method, the per-step term phi_1(dt A_M)(dt g_M) assembled over
  // the cores
  bool forced = false;
  double* d_force = nullptr;
  double* d_bias = nullptr;
  // exponential Rosenbrock-Euler (Burgers): Jacobian refresh every ere_refresh
  // steps; phi_1 core rows per (block, member); augmented matrices and the
  // Pade work space kept between refreshes
  double ere_dx = 0, ere_nu = 0;
  int ere_refresh = 1, ere_nl = 0, ere_rows = 0;
  bool ere_small = false;  // phi_1 by the one-workgroup LDS kernel (no Pade work space)
  int64_t ere_count = 0;
  void* d_ere_boxes = nullptr;
  double *d_ere_A = nullptr, *d_ere_R = nullptr, *d_phi = nullptr, *d_f = nullptr;
  std::vector<double*> ere_work;  // A2, A4, A6, T, Ub, norms; plus the squaring counts
  int* d_ere_s = nullptr;
  // Kronecker-factored dense method: per-block descriptors and the core rows
  // of the two 1D local exponentials (x then y, core x box side each)
  lem::KronBlock* d_kron = nullptr;
  double* d_ex = nullptr;
  int kron_L = 0;
  // small 1D dense plans: all steps of a lem_step call in one launch
  bool resident = false;
  // global
  lem::GlobalWork gw{};
  // shared
  int* d_status = nullptr;
  double* d_tmp = nullptr;
  std::vector<void*> allocs;
  lem::Arena* arena = nullptr;  // allocate from a serving pool instead of hipMalloc
  std::vector<lem::KBlock> kb_host;  // step descriptors (Krylov), bucket order
  int64_t bytes_blocks = 0, bytes_work = 0;
  hipStream_t stream = nullptr;
  std::map<std::pair<const void*, void*>, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
  double plan_ms = 0;

  ~lem_plan_s() {
    for (auto& g : graphs) {
      hipGraphExecDestroy(g.second.second);
      hipGraphDestroy(g.second.first);
    }
    for (hipStream_t s : side) {  // the last step's side launches read plan memory
      hipStreamSynchronize(s);
      hipStreamDestroy(s);
    }
    for (hipEvent_t e : ev_join) hipEventDestroy(e);
    if (ev_fork) hipEventDestroy(ev_fork);
    for (void* q : allocs) {
      if (arena) arena->release(q);
      else hipFree(q);
    }
  }
};


namespace lemh {

// ---- device memory of a plan (hipMalloc, or the plan's arena)
template <typename T>
lem_status dalloc(lem_plan_s* p, T** out, size_t count, int64_t* account = nullptr) {
  *out = nullptr;
  if (count == 0) count = 1;
  void* ptr = nullptr;
  if (p->arena) {
    ptr = p->arena->alloc(count * sizeof(T));
    if (!ptr)
      return fail(LEM_ERR_BUDGET, "memory budget exhausted (" + std::to_string(count * sizeof(T)) +
                                      " bytes requested)");
  } else {
    hipError_t e = hipMalloc(&ptr, count * sizeof(T));
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(LEM_ERR_NOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
    }
  }
  p->allocs.push_back(ptr);
  if (account) *account += (int64_t)(count * sizeof(T));
  *out = (T*)ptr;
  return LEM_OK;
}
void dfree(lem_plan_s* p, void* ptr);
lem_status upload(void* dst, const void* src, size_t bytes, hipStream_t st);

// ---- partition (host_krylov.cpp)
lem_status make_partition(lem_plan_s* p);

// ---- Krylov local actions (host_krylov.cpp)
// Launch shape of one block: the Krylov kernel with its basis in LDS when the
// whole basis fits there, else with the basis streamed through device memory
// (variants 1, and 2 with the augmented coordinate); boxes above 4096 points
// or dimensions above 30 take the large-box kernel (variants 3 and 4).
struct LaunchKey {
  int variant, nt, pmax;
  bool vlds;
  bool operator<(const LaunchKey& o) const {
    return std::tie(variant, nt, pmax, vlds) < std::tie(o.variant, o.nt, o.pmax, o.vlds);
  }
};
LaunchKey launch_key(int ndim, int nloc, int m, size_t* lds, int aug = 0);
// Relative cost of one block step (dimension m, nsub sub-steps).
double block_cost(int ndim, int nloc, int m, int nsub);
lem_status upload_coef(lem_plan_s* p, hipStream_t st);
hipError_t launch_bucket(int variant, const lem::KBlock* blocks, int count, int ns, int nt,
                         int pmax, bool vlds, size_t lds, const double* src, double* dst,
                         const double* coef, double* vwork, double* diag, int* status,
                         double* calib, int mode, hipStream_t s);
lem_status launch_buckets(const lem_plan_s* p, const lem::KBlock* d_kb,
                          const std::vector<lem_plan_s::Bucket>& bks, int ns, const double* src,
                          double* dst, double* vwork, double* diag, double* calib, int mode,
                          hipStream_t st);
bool choose_m(const double* est, const std::vector<int>& jl, int nsc, double tol, int mfix,
              int mcal, int ndim, int nloc, int* m, int* nsub);
lem_status plan_krylov(lem_plan_s* p, hipStream_t st);

// ---- stored local exponentials (host_dense.cpp)
lem_status dense_expm(lem_plan_s* p, double* A, double* R, int nl, int U, hipStream_t st,
                      int* smax, const std::vector<double*>* work = nullptr,
                      int* work_s = nullptr);
lem_status plan_dense(lem_plan_s* p, hipStream_t st, const double* host_g);
const void* dense_operand(const lem_plan_s* p);
lem_status plan_kron(lem_plan_s* p, hipStream_t st);
lem_status choose_tile(lem_plan_s* p, hipStream_t st);

// ---- exponential Rosenbrock-Euler (host_problems.cpp)
lem_status ere_run_one(lem_plan_s* p, const double* src, double* dst, hipStream_t st);

// ---- global method (host_plan.cpp)
lem_status alloc_global(lem_plan_s* p, int m, int ns, int nsub, lem::GlobalWork* w,
                        bool forced = false);
void free_global(lem_plan_s* p, lem::GlobalWork* w);
lem_status plan_global(lem_plan_s* p, hipStream_t st);

// ---- steps and plan life cycle (host_plan.cpp)
lem_status run_one(lem_plan_s* p, const double* src, double* dst, hipStream_t st);
lem_status run_step(lem_plan_s* p, const double* src, double* dst, hipStream_t st);
lem_status check_options(const lem_options* o);
void fill_info(const lem_plan_s* p, lem_plan_info* in);
bool overlap(const void* a, const void* b, size_t bytes);
// lem_status of latched device status bits (non-finite values first).
int device_status_of(int bits);
lem_status create_plan(const lem_operator* op, double dt, const lem_options* opt, void* stream,
                       lem::Arena* arena, lem_plan_t* out);

}  // namespace lemh
