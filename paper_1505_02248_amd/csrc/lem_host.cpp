// Host side of the LEM library: operator weights, the overlapping partition
// with decay-bound buffer widths, Krylov calibration, the one-off Pade
// computation of stored local exponentials, the step loop and the C ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <deque>
#include <map>
#include <tuple>
#include <string>
#include <utility>
#include <vector>

#include "arena.h"
#include "lem.h"
#include "lem_internal.h"
#include "lem_launch.h"

namespace {

thread_local std::string g_err;

lem_status fail(lem_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define LEM_HIP(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(LEM_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));      \
  } while (0)

#define LEM_TRY(expr)                \
  do {                               \
    lem_status s_ = (expr);          \
    if (s_ != LEM_OK) return s_;     \
  } while (0)

// Pade [13/13] numerator coefficients (Higham 2005, scaled b_13 = 1).
constexpr double kB[14] = {64764752532480000.0, 32382376266240000.0, 7771770303897600.0,
                           1187353796428800.0,  129060195264000.0,   10559470521600.0,
                           670442572800.0,      33522128640.0,       1323241920.0,
                           40840800.0,          960960.0,            16380.0,
                           182.0,               1.0};

// ----------------------------------------------------------- operator ------
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

lem_status build_op(const lem_operator* o, double dt, Op* op) {
  if (!o) return fail(LEM_ERR_INVALID, "operator is NULL");
  if (o->ndim != 1 && o->ndim != 2) return fail(LEM_ERR_INVALID, "ndim must be 1 or 2");
  if (o->n < 3) return fail(LEM_ERR_INVALID, "n must be >= 3");
  if (!(o->dx > 0) || !std::isfinite(o->dx)) return fail(LEM_ERR_INVALID, "dx must be > 0");
  if (!(dt > 0) || !std::isfinite(dt)) return fail(LEM_ERR_INVALID, "dt must be > 0");
  if (!(o->nu >= 0) && !o->nu_field) return fail(LEM_ERR_INVALID, "nu must be >= 0");
  if (!(o->dy >= 0) || !std::isfinite(o->dy)) return fail(LEM_ERR_INVALID, "dy must be >= 0");
  op->ndim = o->ndim;
  op->n = o->n;
  op->dx = o->dx;
  op->dy = (o->ndim == 2 && o->dy > 0) ? o->dy : o->dx;
  op->dt = dt;
  op->vel[0] = o->vel[0];
  op->vel[1] = o->ndim == 2 ? o->vel[1] : 0.0;
  op->nu = o->nu;
  if (o->vel_faces && (op->vel[0] != 0.0 || op->vel[1] != 0.0))
    return fail(LEM_ERR_INVALID, "vel must be zero when vel_faces is given");
  const double cx = op->vel[0] * dt / o->dx;
  const double cy = op->vel[1] * dt / op->dy;
  op->chx = cx / 2.0;
  op->chy = cy / 2.0;
  if (!o->nu_field && !o->vel_faces) {
    const double mu = o->nu * dt / (o->dx * o->dx);
    const double muy = o->nu * dt / (op->dy * op->dy);
    op->variable = false;
    if (o->ndim == 1) {
      op->w[0] = -(mu + mu);
      op->w[1] = mu + cx / 2.0;
      op->w[2] = mu - cx / 2.0;
      op->w[3] = 0.0;
      op->w[4] = 0.0;
    } else {
      op->w[0] = -(((mu + mu) + muy) + muy);
      op->w[1] = mu + cx / 2.0;
      op->w[2] = mu - cx / 2.0;
      op->w[3] = muy + cy / 2.0;
      op->w[4] = muy - cy / 2.0;
    }
    return LEM_OK;
  }
  op->variable = true;
  const int64_t N = op->N();
  const int n = op->n;
  const double s = dt / (2.0 * o->dx * o->dx);
  const double sy = dt / (2.0 * op->dy * op->dy);
  op->mux.assign(N, 0.0);
  op->muy.assign(N, 0.0);
  if (o->nu_field) {
    for (int64_t g = 0; g < N; ++g) {
      const double v = o->nu_field[g];
      if (!(v >= 0) || !std::isfinite(v)) return fail(LEM_ERR_INVALID, "nu_field must be >= 0");
    }
  } else if (!(o->nu >= 0) || !std::isfinite(o->nu)) {
    return fail(LEM_ERR_INVALID, "nu must be >= 0");
  }
  auto nu_at = [&](int64_t g) { return o->nu_field ? o->nu_field[g] : o->nu; };
  const int ny = op->ndim == 1 ? 1 : n;
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < n; ++i) {
      const int64_t g = (int64_t)j * n + i;
      const int64_t e = (int64_t)j * n + (i + 1) % n;
      op->mux[g] = (nu_at(g) + nu_at(e)) * s;
      if (op->ndim == 2) {
        const int64_t t = (int64_t)((j + 1) % n) * n + i;
        op->muy[g] = (nu_at(g) + nu_at(t)) * sy;
      }
    }
  if (o->vel_faces) {
    op->varvel = true;
    op->chx = op->chy = 0.0;
    op->ax.assign(N, 0.0);
    op->ay.assign(N, 0.0);
    for (int64_t g = 0; g < N; ++g) {
      const double a = o->vel_faces[g];
      const double b = op->ndim == 2 ? o->vel_faces[N + g] : 0.0;
      if (!std::isfinite(a) || !std::isfinite(b)) return fail(LEM_ERR_INVALID, "vel_faces must be finite");
      op->ax[g] = a * (dt / (2.0 * o->dx));
      op->ay[g] = b * (dt / (2.0 * op->dy));
    }
  }
  return LEM_OK;
}

// Weights of the row of global point (i, j).
void point_weights(const Op& op, int i, int j, double* w) {
  if (!op.variable) {
    for (int q = 0; q < 5; ++q) w[q] = op.w[q];
    return;
  }
  const int n = op.n;
  const int64_t g = (int64_t)j * n + i;
  const double me = op.mux[g], mw = op.mux[(int64_t)j * n + (i + n - 1) % n];
  double mn = 0, ms = 0;
  if (op.ndim == 2) {
    mn = op.muy[g];
    ms = op.muy[(int64_t)((j + n - 1) % n) * n + i];
  }
  w[0] = -(((me + mw) + mn) + ms);
  w[1] = mw + op.chx;
  w[2] = me - op.chx;
  w[3] = op.ndim == 2 ? ms + op.chy : 0.0;
  w[4] = op.ndim == 2 ? mn - op.chy : 0.0;
  if (op.varvel) {  // conservative centered advection by face velocities
    const double ae = op.ax[g], aw = op.ax[(int64_t)j * n + (i + n - 1) % n];
    double an = 0, as = 0;
    if (op.ndim == 2) {
      an = op.ay[g];
      as = op.ay[(int64_t)((j + n - 1) % n) * n + i];
    }
    w[0] -= (ae - aw) + (an - as);
    w[1] = mw + aw;
    w[2] = me - ae;
    w[3] = op.ndim == 2 ? ms + as : 0.0;
    w[4] = op.ndim == 2 ? mn - an : 0.0;
  }
}

// ------------------------------------------------------------ halo bound --
// eps(h) = G * sum_sides |w_s| min_r [(e^phi - 1)/phi] r^-h,
// phi = w0 + P_s + |w_s| r + |w_sbar| / r   (a Cauchy-estimate bound of the
// per-step LEM error at the core, Duhamel's formula with the outside values
// as a source on the box edge; see the library documentation).
double log_expm1_over(double phi) {
  if (std::fabs(phi) < 1e-8) return phi / 2.0;
  if (phi > 0) return phi + std::log1p(-std::exp(-phi)) - std::log(phi);
  return std::log(-std::expm1(phi)) - std::log(-phi);
}

double side_log_bound(double ws, double wsb, double w0, double P, int h) {
  const double b = std::fabs(ws), c = std::fabs(wsb);
  if (b == 0.0) return -std::numeric_limits<double>::infinity();
  const double a = w0 + P;
  auto f = [&](double t) { return log_expm1_over(a + b * std::exp(t) + c * std::exp(-t)) - h * t; };
  // golden-section search of the convex objective on log r in [-40, 40]
  const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
  double lo = -40.0, hi = 40.0;
  double x1 = hi - gr * (hi - lo), x2 = lo + gr * (hi - lo);
  double f1 = f(x1), f2 = f(x2);
  for (int it = 0; it < 200 && hi - lo > 1e-12; ++it) {
    if (f1 < f2) {
      hi = x2; x2 = x1; f2 = f1; x1 = hi - gr * (hi - lo); f1 = f(x1);
    } else {
      lo = x1; x1 = x2; f1 = f2; x2 = lo + gr * (hi - lo); f2 = f(x2);
    }
  }
  return std::log(b) + std::min(f1, f2);
}

struct BlockCoef { double aW, aE, aS, aN, w0; };

double eps_bound(const BlockCoef& c, int h, int ndim, double G, bool cut_y = true) {
  double t[4] = {side_log_bound(c.aW, c.aE, c.w0, c.aS + c.aN, h),
                 side_log_bound(c.aE, c.aW, c.w0, c.aS + c.aN, h), -INFINITY, -INFINITY};
  if (ndim == 2 && cut_y) {
    t[2] = side_log_bound(c.aS, c.aN, c.w0, c.aW + c.aE, h);
    t[3] = side_log_bound(c.aN, c.aS, c.w0, c.aW + c.aE, h);
  }
  double s = 0.0;
  for (double v : t)
    if (v > -INFINITY) s += std::exp(v);
  return G * s;
}

double growth_factor(const Op& op) {
  double mx = -INFINITY;
  const int ny = op.ndim == 1 ? 1 : op.n;
  double w[5];
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < op.n; ++i) {
      point_weights(op, i, j, w);
      mx = std::max(mx, w[0] + std::fabs(w[1]) + std::fabs(w[2]) + std::fabs(w[3]) + std::fabs(w[4]));
      if (!op.variable) return std::exp(std::max(0.0, mx));
    }
  return std::exp(std::max(0.0, mx));
}

struct Box { int ox, oy, cx, cy, h; };

// Buffer widths per axis: none along an axis the core spans whole (column-
// wise decompositions, and the D = 1 box), which keeps the periodic coupling
// along that axis inside the box.
inline int box_hx(const Box& b, int n) { return b.cx == n ? 0 : b.h; }
inline int box_hy(const Box& b, int n, int ndim) { return ndim == 2 ? (b.cy == n ? 0 : b.h) : 0; }
inline int box_lx(const Box& b, int n) { return b.cx + 2 * box_hx(b, n); }
inline int box_ly(const Box& b, int n, int ndim) { return ndim == 2 ? b.cy + 2 * box_hy(b, n, ndim) : 1; }

BlockCoef block_coef(const Op& op, const Box& b, int h) {
  BlockCoef c{0, 0, 0, 0, -INFINITY};
  double w[5];
  if (!op.variable) {
    c = {std::fabs(op.w[1]), std::fabs(op.w[2]), std::fabs(op.w[3]), std::fabs(op.w[4]), op.w[0]};
    return c;
  }
  const int n = op.n;
  Box bh = b;
  bh.h = h;
  const int hx = box_hx(bh, n), hy = box_hy(bh, n, op.ndim);
  const int Lx = box_lx(bh, n), Ly = box_ly(bh, n, op.ndim);
  for (int ly = 0; ly < Ly; ++ly)
    for (int lx = 0; lx < Lx; ++lx) {
      const int gx = ((b.ox - hx + lx) % n + n) % n;
      const int gy = op.ndim == 2 ? ((b.oy - hy + ly) % n + n) % n : 0;
      point_weights(op, gx, gy, w);
      c.aW = std::max(c.aW, std::fabs(w[1]));
      c.aE = std::max(c.aE, std::fabs(w[2]));
      c.aS = std::max(c.aS, std::fabs(w[3]));
      c.aN = std::max(c.aN, std::fabs(w[4]));
      c.w0 = std::max(c.w0, w[0]);
    }
  return c;
}

// Largest row sum of |dt*A| over the box of b (with its own halo).
double block_rho(const Op& op, const Box& b) {
  double w[5], mx = 0.0;
  const int n = op.n;
  const int hx = box_hx(b, n), hy = box_hy(b, n, op.ndim);
  const int Lx = box_lx(b, n), Ly = box_ly(b, n, op.ndim);
  for (int ly = 0; ly < Ly; ++ly)
    for (int lx = 0; lx < Lx; ++lx) {
      const int gx = ((b.ox - hx + lx) % n + n) % n;
      const int gy = op.ndim == 2 ? ((b.oy - hy + ly) % n + n) % n : 0;
      point_weights(op, gx, gy, w);
      mx = std::max(mx, std::fabs(w[0]) + std::fabs(w[1]) + std::fabs(w[2]) + std::fabs(w[3]) +
                            std::fabs(w[4]));
    }
  return mx;
}

// Smallest h in [h_min, h_max] with eps(h) <= tol (coefficients taken over the
// box of width h itself); h_max and clamped = true when none qualifies.
int halo_from_bound(const Op& op, Box b, double tol, int h_min, int h_max, double G,
                    bool* clamped) {
  for (int h = h_min; h <= h_max; ++h) {
    const BlockCoef c = block_coef(op, b, op.variable ? h : 0);
    if (eps_bound(c, h, op.ndim, G, !(op.ndim == 2 && b.cy == op.n)) <= tol) {
      *clamped = false;
      return h;
    }
  }
  *clamped = true;
  return h_max;
}

}  // namespace

// ================================================================= plan ====
struct lem_plan_s {
  Op op;
  lem_options opt{};
  int method = 0, ns = 1;
  bool global_box = false;  // global method run as one periodic Krylov box
  int64_t N = 0;
  std::vector<Box> boxes;
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

namespace {

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
      hipGetLastError();
      return fail(LEM_ERR_NOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
    }
  }
  p->allocs.push_back(ptr);
  if (account) *account += (int64_t)(count * sizeof(T));
  *out = (T*)ptr;
  return LEM_OK;
}

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

// ------------------------------------------------------------- partition --
double block_cost(int ndim, int nloc, int m, int nsub);

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

// nloc counts the basis row (box points plus the augmented coordinate of a
// forced step, aug = 1).
LaunchKey launch_key(int ndim, int nloc, int m, size_t* lds, int aug = 0) {
  int nt, pm;
  lem::krylov_lds_config(ndim, nloc, &nt, &pm);
  if (nt == 0 || m > lem::krylov_lds_max_m()) {
    lem::krylov_big_config(nloc, &nt, &pm);
    if (nt == 0 || m > lem::krylov_big_max_m()) return {-1, 0, 0, false};
    *lds = lem::krylov_big_lds_bytes(nt, m);
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
  p->kb_host = kb;
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
  LEM_TRY(dalloc(p, &p->d_kb, kb.size(), &p->bytes_work));
  LEM_TRY(upload(p->d_kb, kb.data(), kb.size() * sizeof(lem::KBlock), st));
  LEM_TRY(dalloc(p, &p->d_vwork, (size_t)std::max<int64_t>(vw, 1), &p->bytes_work));
  LEM_TRY(dalloc(p, &p->d_diag, (size_t)nb * p->ns, &p->bytes_work));
  LEM_HIP(hipMemsetAsync(p->d_diag, 0, (size_t)nb * p->ns * 8, st));
  return LEM_OK;
}

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
                      int* smax, const std::vector<double*>* work = nullptr, int* work_s = nullptr) {
  return p->opt.expm == LEM_EXPM_TAYLOR ? dense_expm_taylor(p, A, R, nl, U, st, smax, work, work_s)
                                        : dense_expm_pade(p, A, R, nl, U, st, smax, work, work_s);
}

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

// --------------------------------------------------------------- global ----
lem_status alloc_global(lem_plan_s* p, int m, int ns, int nsub, lem::GlobalWork* w,
                        bool forced = false) {
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
    default:
      LEM_HIP(lem::global_step(p->gw, src, dst, st));
      return LEM_OK;
  }
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
  const int ntile = p->opt.precision <= LEM_FP32 ? lem::kApplyConfigs : 2;
  for (int tile = 0; tile < ntile; ++tile) {
    if (!lem::dense_apply_supported(p->opt.precision, tile, p->ns, p->rows_p, p->cols_p)) continue;
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
    if (!lem::dense_apply_supported(p->opt.precision, p->opt.tile, p->ns, p->rows_p, p->cols_p))
      return fail(LEM_ERR_UNSUPPORTED, "apply tile shape " + std::to_string(p->opt.tile) +
                                           " does not fit this block and precision");
    p->tile = p->opt.tile;
    return LEM_OK;
  }
  if (p->opt.autotune && p->ns % 64 == 0) return autotune_dense(p, st);
  return LEM_OK;
}

lem_status check_options(const lem_options* o) {
  if (!o) return fail(LEM_ERR_INVALID, "options are NULL");
  if (o->method < 0 || o->method > 2) return fail(LEM_ERR_INVALID, "unknown method");
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
// 32 and 64 points are planned and timed on a probe state; the faster is kept.
// (Boxes of 64^2 cores cut the buffer overhead, but each is one workgroup with
// a long Arnoldi chain: whether they pay depends on the grid and the CUs.)
lem_status create_plan(const lem_operator* op, double dt, const lem_options* opt, void* stream,
                       lem::Arena* arena, lem_plan_t* out) {
  if (!opt || !out || opt->method != LEM_METHOD_KRYLOV || opt->core != 0 || !opt->autotune ||
      opt->dry_run || arena || opt->core_max == 16)
    return create_plan_one(op, dt, opt, stream, arena, out);
  const auto t0 = std::chrono::steady_clock::now();
  lem_plan_t best = nullptr;
  double best_ms = INFINITY;
  for (int cm : {32, 64}) {
    if (opt->core_max && cm > opt->core_max) continue;
    lem_options o = *opt;
    o.core_max = cm;
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
  if (p->method == LEM_METHOD_KRYLOV || p->method == LEM_METHOD_DENSE) {
    if (p->opt.core == 0 && p->method == LEM_METHOD_KRYLOV && p->op.ndim == 1)
      p->opt.core = std::min(64, p->op.n);
    if (p->opt.core == p->op.n)
      return guard(fail(LEM_ERR_INVALID, "a single core covering the grid is the global method"));
    s = make_partition(p);
    if (s != LEM_OK) return guard(s);
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
    else s = plan_global(p, st);
    if (s != LEM_OK) return guard(s);
    if (p->method == LEM_METHOD_DENSE) {
      s = choose_tile(p, st);
      if (s != LEM_OK) return guard(s);
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

}  // namespace

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
  // last step writes x_out; earlier steps alternate x_out / tmp backwards
  const double* src = x_in;
  for (int k = 0; k < n_steps; ++k) {
    double* dst = ((n_steps - 1 - k) % 2 == 0) ? x_out : p->d_tmp;
    LEM_TRY(run_step(p, src, dst, st));
    src = dst;
  }
  return LEM_OK;
}

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

const char* lem_last_error(void) { return g_err.c_str(); }

}  // extern "C"

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
      hipHostFree(h_table);
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
  o->halo_max = 32;
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
      if (!r.plan->kb_host.empty()) continue;
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
