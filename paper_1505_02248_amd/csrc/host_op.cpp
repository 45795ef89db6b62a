// The semi-discrete operator (eq. (2), centered differences; conservative
// flux form with face values for variable coefficients, section 4.3) and the
// buffer widths from the off-diagonal decay bound of the local exponential.
#include "host_internal.h"

namespace lemh {

namespace {
thread_local std::string g_err;
}  // namespace

lem_status fail(lem_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

const char* g_err_text() { return g_err.c_str(); }


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


double eps_bound(const BlockCoef& c, int h, int ndim, double G, bool cut_y) {
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


}  // namespace lemh

extern "C" const char* lem_last_error(void) { return lemh::g_err_text(); }
