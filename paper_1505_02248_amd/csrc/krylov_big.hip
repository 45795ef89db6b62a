// Krylov local action for large boxes and large Krylov dimensions (gfx950).
//
// The same step as krylov_lds_kernel -- one workgroup advances one region
// M_i (one ensemble member) by nsub sub-steps of v <- beta V_m exp(H_m) e_1
// (the Krylov action of section 4.3 on the local problem (4)), then writes
// its core rows (step 3) -- for boxes of up to 9216 points and Krylov
// dimensions up to 40, where keeping every working vector of every point in
// registers (the other kernel's design) would spill.
//
// The basis lives in a per-(block, member) slice of device memory and each
// Arnoldi column uses delayed re-orthogonalization (DCGS2, Swirydowicz et al.
// 2021): row j of V holds u_j, the new direction projected once; one sweep
// over the rows i < j computes s = V^T u_j and z = V^T w for w = A u_j, a
// second sweep forms v_j = (u_j - V s)/nu and u_{j+1} = (w - V z - (v_j^T w)
// v_j)/nu and stores both.  Registers hold only w across the two sweeps,
// and nu comes from Pythagoras, nu^2 = |u_j|^2 - |s|^2 (V has orthonormal
// columns), with an extra sweep that measures |u_j - V s| when that
// difference cancels badly (near an invariant subspace).  The current
// direction u_j also sits in LDS (written with its row), so the stencil
// product reads its neighbours there instead of making a round trip to the
// memory system per point.  exp(H_m) is Pade [13/13] scaling and squaring in
// LDS, in the space the direction occupies during the Arnoldi loop.
#include "lem_device.hpp"
#include "lem_launch.h"

namespace lem {

constexpr int kBigMaxM = 40;     // Krylov dimension limit of this kernel
constexpr int kBigMaxN = 9216;   // box points (plus the augmented coordinate)
constexpr int kBigSlots = 128;   // reduction slots per wave: s at 0.., z at 64..

// LDS layout in doubles: Hessenberg, reduction slots, workgroup totals, then
// one region holding the direction u_j (NT * P points) during the Arnoldi
// loop and the exponential's work space after it.
__host__ __device__ inline int64_t big_lds_layout(int NT, int P, int m, int64_t* off_red,
                                                  int64_t* off_tot, int64_t* off_e) {
  int64_t d = (int64_t)(m + 1) * m;  // Hessenberg
  *off_red = d;
  d += (int64_t)(NT / 64) * kBigSlots;
  *off_tot = d;
  d += kBigSlots;
  *off_e = d;
  const int64_t e = 7 * (int64_t)m * m + 2 * (NT / 64) + 4;  // expm_small: A, W (5), R, piv
  d += e > (int64_t)NT * P ? e : (int64_t)NT * P;
  return d;
}

// The five weights (centre, W, E, S, N) of dt_sub A_M at box point (lx, ly)
// of a block with face diffusion coefficients (and face velocities): the
// centered stencil of section 4, couplings leaving the box dropped (weights
// zero on the box edges the core does not span whole).
__device__ __forceinline__ void box_weights(const KBlock& b, const double* coef, int lx, int ly,
                                            double (&w)[5]) {
  w[0] = b.w0; w[1] = b.wW; w[2] = b.wE; w[3] = b.wS; w[4] = b.wN;
  if (b.mu_off >= 0) {
    const double* mux = coef + b.mu_off;
    const int64_t Ng = (b.ndim == 1) ? b.n : (int64_t)b.n * b.n;
    const double* muy = mux + Ng;
    const int gx = wrap(b.ox - b.h + lx, b.n);
    const int gy = (b.ndim == 1) ? 0 : wrap(b.oy - b.hy + ly, b.n);
    const int64_t g = (int64_t)gy * b.n + gx;
    const int64_t gw = (int64_t)gy * b.n + wrap(gx - 1, b.n);
    const int64_t gs = (int64_t)wrap(gy - 1, b.n) * b.n + gx;
    const double me = mux[g], mw = mux[gw];
    const double mn = b.ndim == 2 ? muy[g] : 0.0, ms = b.ndim == 2 ? muy[gs] : 0.0;
    const double sc = b.sub_scale;
    w[0] = -(me + mw + mn + ms) * sc;
    if (b.varvel) {  // conservative centered advection by face velocities
      const double* axf = mux + 2 * Ng;
      const double ae = axf[g] * sc, aw = axf[gw] * sc;
      const double an = b.ndim == 2 ? axf[Ng + g] * sc : 0.0;
      const double as = b.ndim == 2 ? axf[Ng + gs] * sc : 0.0;
      w[0] -= (ae - aw) + (an - as);
      w[1] = fma(mw, sc, aw);
      w[2] = fma(me, sc, -ae);
      w[3] = fma(ms, sc, as);
      w[4] = fma(mn, sc, -an);
    } else {
      w[1] = fma(mw, sc, b.chx);
      w[2] = fma(me, sc, -b.chx);
      w[3] = fma(ms, sc, b.chy);
      w[4] = fma(mn, sc, -b.chy);
    }
  }
  if (!(b.periodic & 1)) {
    if (lx == 0) w[1] = 0.0;
    if (lx == b.Lx - 1) w[2] = 0.0;
  }
  if (b.ndim == 1) {
    w[3] = w[4] = 0.0;
  } else if (!(b.periodic & 2)) {
    if (ly == 0) w[3] = 0.0;
    if (ly == b.Ly - 1) w[4] = 0.0;
  }
}

// The basis slice is addressed through a buffer resource: the slice base in
// scalar registers, the row and point-group offsets as one scalar, and a lane
// offset (tid * 8) shared by every row and point (64-bit per-lane addresses
// for every point would exhaust the register file).  Point p of a lane is
// local index tid + p * NT; lanes past the box read past the row end, which
// stays inside the slice and its padding (the planner pads every block's
// slices by NT * P doubles) and is discarded by the callers.
//
// Rows are the same for every lane, but the compiler may hold a row index in
// a vector register (the Arnoldi loop's exit depends on values it cannot
// prove uniform), and a buffer access with a vector-held scalar offset
// becomes a loop over the distinct values.  The offset therefore goes
// through readfirstlane: one instruction, exact because it is uniform.
template <int NT>
struct BasisRows {
  __amdgpu_buffer_rsrc_t r;
  int row_bytes;
  uint32_t lane_off;
  typedef decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)) raw_t;
  __device__ __forceinline__ int soff(int row, int p) const {
    return __builtin_amdgcn_readfirstlane(row * row_bytes + p * (NT * 8));
  }
  // this lane's point p of row `row`
  __device__ __forceinline__ double ldp(int row, int p) const {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, lane_off, soff(row, p), 0));
  }
  __device__ __forceinline__ void stp(int row, int p, double v) const {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(raw_t, v), r, lane_off, soff(row, p), 0);
  }
};

template <int NT, int P, bool AUG>
__global__ __launch_bounds__(NT) void krylov_big_kernel(KrylovArgs a) {
  constexpr int GR = 4;                  // basis rows per group of the dot sweep
  constexpr int CB = P >= 12 ? 1 : 2;    // rows per load batch of the update sweep
  extern __shared__ double smem[];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int s = blockIdx.y;
  const KBlock b = a.blocks[blockIdx.x];
  const int m = b.m;
  const int nloc = b.Lx * b.Ly;
  const int nlv = nloc + (AUG ? 1 : 0);
  int64_t ored, otot, oe;
  big_lds_layout(NT, P, m, &ored, &otot, &oe);
  double* H = smem;
  double* red = smem + ored;  // [NT/64][kBigSlots]
  double* tot = smem + otot;  // workgroup totals of the slots
  double* U = smem + oe;      // u_j during the Arnoldi loop (aliases the expm work)
  double* EA = smem + oe;
  double* EW = EA + m * m;
  double* ER = EW + 5 * m * m;
  double* piv = ER + m * m;
  double* vslice = (b.vwork ? b.vwork : a.vwork + b.v_off) + (int64_t)s * (m + 1 + (AUG ? 1 : 0)) * nlv;
  // word 3: 32-bit data format, raw (untyped) access
  const BasisRows<NT> V{__builtin_amdgcn_make_buffer_rsrc(vslice, 0, 0x7ffffff0, 0x00020000),
                        nlv * 8, (uint32_t)tid * 8u};
  const double* x_in = b.xin ? b.xin : a.x_in;
  double* x_out = b.xout ? b.xout : a.x_out;
  // variable coefficients: the block's precomputed weights (rows of NT * P
  // points; the planner attaches them to every such block); constant ones:
  // the block's scalar weights
  const bool varcoef = b.mu_off >= 0;
  if (varcoef && b.wts == nullptr) {  // a table built without them: refuse loudly
    if (tid == 0) atomicOr(b.status ? b.status : a.status, kStatusNonFinite);
    return;
  }
  const BasisRows<NT> Wt{__builtin_amdgcn_make_buffer_rsrc((void*)b.wts, 0, 0x7ffffff0, 0x00020000),
                         NT * P * 8, (uint32_t)tid * 8u};

  // point p of this thread is local index tid + p * NT; its box coordinates
  // are recomputed where needed (the stencil, the gather and the core write)
  auto coords = [&](int l, int& lx, int& ly) __attribute__((always_inline)) {
    ly = l / b.Lx;
    lx = l - ly * b.Lx;
  };
  // unsigned 32-bit offsets from a row base held in scalar registers
  auto lidx = [&](int p) __attribute__((always_inline)) { return (uint32_t)(tid + p * NT); };
  auto live = [&](int p) __attribute__((always_inline)) { return tid + p * NT < nlv; };
  auto li = [&](int p) __attribute__((always_inline)) {
    return (uint32_t)min(tid + p * NT, nlv - 1);
  };

  // (dt_sub A_M u_j)_l at point p, u_j from LDS, with the weights w0..wN of
  // the point; couplings leaving the box are dropped (zero weights on the
  // edges the core does not span whole, already zero in a precomputed
  // table), the periodic wrap kept along an axis the box spans whole; the
  // augmented row (forced steps) is zero
  auto stencil = [&](int p, double w0, double wW, double wE, double wS, double wN)
      __attribute__((always_inline)) {
    int l = (int)li(p);
    asm volatile("" : "+v"(l));  // neighbour offsets per use: no hoisting
    int lx, ly;
    coords(l, lx, ly);
    int lW = l - 1, lE = l + 1, lS = l - b.Lx, lN = l + b.Lx;
    if (b.periodic & 1) {
      if (lx == 0) lW += b.Lx;
      if (lx == b.Lx - 1) lE -= b.Lx;
    } else {
      if (lx == 0) { wW = 0.0; lW = l; }
      if (lx == b.Lx - 1) { wE = 0.0; lE = l; }
    }
    if (b.ndim == 1) {
      wS = wN = 0.0; lS = lN = l;
    } else if (b.periodic & 2) {
      if (ly == 0) lS += nloc;
      if (ly == b.Ly - 1) lN -= nloc;
    } else {
      if (ly == 0) { wS = 0.0; lS = l; }
      if (ly == b.Ly - 1) { wN = 0.0; lN = l; }
    }
    if (!live(p) || (AUG && l == nloc)) return 0.0;
    double r = w0 * U[l];
    r = fma(wW, U[lW], r);
    r = fma(wE, U[lE], r);
    r = fma(wS, U[lS], r);
    r = fma(wN, U[lN], r);
    return r;
  };
  // forced steps: the augmented column dt_sub g_M, kept as row m+1 of the
  // basis storage (its entry on the augmented row is zero)
  const int frow = m + 1;
  if constexpr (AUG) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      if (!live(p)) continue;
      asm volatile("" ::: "memory");
      const int l = lidx(p);
      int lx, ly;
      coords(l, lx, ly);
      V.stp(frow, p, l == nloc ? 0.0 : b.gscale * b.force[b.x_off + gather_index(b, lx, ly) * b.ns + s]);
    }
  }
  // workgroup totals of the per-wave slots [0, cnt) and [64, 64 + cnt) into tot
  auto totals = [&]() __attribute__((always_inline)) {
    __syncthreads();
    for (int q = tid; q < kBigSlots; q += NT) {
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) t += red[w * kBigSlots + q];
      tot[q] = t;
    }
    __syncthreads();
  };
  auto wg_total = [&](double v, int slot) __attribute__((always_inline)) {
    v = wave_sum(v);
    if (lane == 0) red[wv * kBigSlots + slot] = v;
    totals();
    return tot[slot];
  };

  double cur[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    asm volatile("" ::: "memory");  // one gather in flight at a time (bounded registers)
    int lx, ly;
    coords(li(p), lx, ly);
    cur[p] = !live(p) ? 0.0
             : (AUG && lidx(p) == nloc) ? 1.0
                                          : x_in[b.x_off + gather_index(b, lx, ly) * b.ns + s];
  }
  auto sq = [&](const double (&x)[P]) __attribute__((always_inline)) {
    double t = 0.0;
#pragma unroll
    for (int p = 0; p < P; ++p) t = fma(x[p], x[p], t);
    return t;
  };
  const double beta0 = sqrt(wg_total(sq(cur), 0));
  double worst = 0.0;
  bool bad = !isfinite(beta0);
  const int nsub = (a.mode == 1) ? 1 : b.nsub;

  for (int sub = 0; sub < nsub; ++sub) {
    const double beta = (sub == 0) ? beta0 : sqrt(wg_total(sq(cur), 0));
    if (!(beta > 0.0) || !isfinite(beta)) {
      if (!isfinite(beta)) bad = true;
      break;
    }
    {
      const double ib = 1.0 / beta;
#pragma unroll
      for (int p = 0; p < P; ++p)
        if (live(p)) {  // u_0 = v_0
          V.stp(0, p, cur[p] * ib);
          U[lidx(p)] = cur[p] * ib;
        }
    }
    for (int idx = tid; idx < (m + 1) * m; idx += NT) H[idx] = 0.0;
    __syncthreads();

    int k = m;
    for (int j = 0; j <= m; ++j) {
      const bool last = j == m;
      // sweep A: w = A u_j; s_i = <v_i, u_j> (slot i), z_i = <v_i, w> (slot
      // 64 + i) for i < j, |u_j|^2 (slot 62), u_j^T w (slot 63)
      double w[P];
      {
        double u[P];
        if (varcoef && !last) {
          // the weight loads of G points in flight together
          constexpr int G = P >= 12 ? 6 : 4;
#pragma unroll
          for (int p0 = 0; p0 < P; p0 += G) {
            asm volatile("" ::: "memory");  // one group's loads at a time (bounded registers)
            double wt[G][5];
#pragma unroll
            for (int q = 0; q < G; ++q)
#pragma unroll
              for (int k = 0; k < 5; ++k) wt[q][k] = p0 + q < P ? Wt.ldp(k, p0 + q) : 0.0;
#pragma unroll
            for (int q = 0; q < G; ++q) {
              const int p = p0 + q;
              if (p < P) {
                u[p] = live(p) ? U[li(p)] : 0.0;
                w[p] = stencil(p, wt[q][0], wt[q][1], wt[q][2], wt[q][3], wt[q][4]);
              }
            }
          }
        } else {
#pragma unroll
          for (int p = 0; p < P; ++p) {
            u[p] = live(p) ? U[li(p)] : 0.0;
            w[p] = last ? 0.0 : stencil(p, b.w0, b.wW, b.wE, b.wS, b.wN);
          }
        }
        if constexpr (AUG) {
          if (!last) {
            const double ve = U[nloc];
#pragma unroll
            for (int p = 0; p < P; ++p)
              if (live(p)) w[p] = fma(V.ldp(frow, p), ve, w[p]);
          }
        }
#pragma unroll 1
        for (int i0 = 0; i0 < j; i0 += GR) {
          double t[2 * GR];
#pragma unroll
          for (int q = 0; q < GR; ++q) {
            asm volatile("" ::: "memory");  // one row's loads in flight at a time
            const int i = min(i0 + q, j - 1);
            double vals[P];
#pragma unroll
            for (int p = 0; p < P; ++p) vals[p] = V.ldp(i, p);
            double ts = 0.0, tz = 0.0;
#pragma unroll
            for (int p = 0; p < P; ++p) {
              const double v = live(p) ? vals[p] : 0.0;
              ts = fma(v, u[p], ts);
              tz = fma(v, w[p], tz);
            }
            const bool ok = i0 + q < j;
            t[q] = ok ? ts : 0.0;
            t[GR + q] = ok ? tz : 0.0;
          }
          const double r = wave_reduce_scatter<2 * GR>(t);
          constexpr int LPV = 64 / (2 * GR);  // lanes per value
          const int v = lane / LPV, row = i0 + (v % GR);
          if (lane % LPV == 0 && row < j) red[wv * kBigSlots + (v < GR ? row : 64 + row)] = r;
        }
        double tu = 0.0, tw = 0.0;
#pragma unroll
        for (int p = 0; p < P; ++p) {
          tu = fma(u[p], u[p], tu);
          tw = fma(u[p], w[p], tw);
        }
        tu = wave_sum(tu);
        tw = wave_sum(tw);
        if (lane == 0) {
          red[wv * kBigSlots + 62] = tu;
          red[wv * kBigSlots + 63] = tw;
        }
      }
      totals();
      // nu = |u_j - V s| by Pythagoras unless it cancels
      const double uu = tot[62];
      // |s|^2 and s^T z, lane i holding row i (every wave sums them itself)
      const double si = lane < j ? tot[lane] : 0.0, zi = lane < j ? tot[64 + lane] : 0.0;
      const double ss = wave_sum(si * si), sz = wave_sum(si * zi);
      double nu2 = uu - ss;
      if (!(nu2 > 1e-4 * uu)) {
        // measured: |u_j - V s|^2 (slot 61)
        double vt[P];
#pragma unroll
        for (int p = 0; p < P; ++p) vt[p] = live(p) ? V.ldp(j, p) : 0.0;
#pragma unroll 1
        for (int i = 0; i < j; ++i) {
          const double si = tot[i];
#pragma unroll
          for (int p = 0; p < P; ++p) vt[p] = fma(-si, live(p) ? V.ldp(i, p) : 0.0, vt[p]);
        }
        double tn = wave_sum(sq(vt));
        __syncthreads();  // everyone has read tot before it is rewritten
        if (lane == 0) red[wv * kBigSlots + 61] = tn;
        totals();
        nu2 = tot[61];
        // tot[0..j) and tot[64..) were summed again from the same slots
      }
      const double nu = sqrt(fmax(nu2, 0.0));
      const double bw = tot[63];
      bool brk;
      if (j > 0) {
        // |corrected column j-1|^2, lane i holding row i (every wave sums it)
        const double hij = lane < j ? H[lane * m + j - 1] + tot[lane] : 0.0;
        const double hs = wave_sum(hij * hij);
        brk = !(nu > 1e-14 * sqrt(hs + nu * nu));  // invariant subspace reached
      } else {
        brk = !(nu > 0.0);
      }
      __syncthreads();  // every thread has read column j-1 before it is rewritten
      const double cj = (bw - sz) / nu;  // v_j^T w
      if (tid <= j) {
        const int i = tid;
        double hcorr = 0.0;
        if (j > 0) hcorr = (i < j) ? H[i * m + j - 1] + tot[i] : nu;
        if (!last && !brk) {
          // four partial sums: the loads of four terms in flight together
          auto hl = [&](int l) __attribute__((always_inline)) {
            return (l == j - 1) ? hcorr : H[i * m + l];
          };
          double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
          int l = i > 0 ? i - 1 : 0;
          for (; l + 3 < j; l += 4) {
            t0 = fma(hl(l), tot[l], t0);
            t1 = fma(hl(l + 1), tot[l + 1], t1);
            t2 = fma(hl(l + 2), tot[l + 2], t2);
            t3 = fma(hl(l + 3), tot[l + 3], t3);
          }
          for (; l < j; ++l) t0 = fma(hl(l), tot[l], t0);
          const double t = (t0 + t1) + (t2 + t3);
          const double num = (i < j) ? tot[64 + i] : cj;
          H[i * m + j] = (num - t) / nu;
        }
        if (j > 0) H[i * m + j - 1] = hcorr;
      }
      if (brk || last) {
        k = j > 0 ? j : 0;
        __syncthreads();
        break;
      }
      // sweep B: vt = u_j - V s, y = w - V z; v_j = vt / nu and
      // u_{j+1} = (y - cj vt / nu) / nu overwrite rows j and j+1, and u_{j+1}
      // replaces u_j in LDS (every stencil read of u_j preceded the
      // reductions' barriers; a thread rewrites only its own points)
      {
        double vt[P];
#pragma unroll
        for (int p = 0; p < P; ++p) vt[p] = live(p) ? U[li(p)] : 0.0;
#pragma unroll 1
        for (int i0 = 0; i0 < j; i0 += CB) {
          double vals[CB][P], sc[CB], zc[CB];
#pragma unroll
          for (int q = 0; q < CB; ++q) {
            const int i = min(i0 + q, j - 1);
            const bool ok = i0 + q < j;
            sc[q] = ok ? tot[i] : 0.0;
            zc[q] = ok ? tot[64 + i] : 0.0;
#pragma unroll
            for (int p = 0; p < P; ++p) vals[q][p] = V.ldp(i, p);
          }
#pragma unroll
          for (int q = 0; q < CB; ++q)
#pragma unroll
            for (int p = 0; p < P; ++p) {
              const double v = live(p) ? vals[q][p] : 0.0;
              vt[p] = fma(-sc[q], v, vt[p]);
              w[p] = fma(-zc[q], v, w[p]);
            }
        }
        const double inv = 1.0 / nu, cc = cj * inv;
#pragma unroll
        for (int p = 0; p < P; ++p) {
          if (!live(p)) continue;
          const double un = (w[p] - cc * vt[p]) * inv;
          V.stp(j, p, vt[p] * inv);
          V.stp(j + 1, p, un);
          U[lidx(p)] = un;
        }
      }
      __syncthreads();
    }

    if (a.mode == 1) {
      double* out = a.calib + ((int64_t)b.diag * b.ns + s) * (2 + (m + 1) * m);
      for (int idx = tid; idx < (m + 1) * m; idx += NT) out[2 + idx] = H[idx];
      if (tid == 0) { out[0] = beta; out[1] = (double)k; }
      return;
    }

    // exp(H_k) e_1
    for (int idx = tid; idx < k * k; idx += NT) {
      const int i = idx / k, jj = idx - i * k;
      EA[idx] = H[i * m + jj];
    }
    __syncthreads();
    if (k > 0) expm_small<NT>(EA, k, EW, ER, piv);
    const double hk = k > 0 ? H[k * m + (k - 1)] : 0.0;
    if (k > 0) worst += beta * hk * fabs(ER[(k - 1) * k]) / beta0;
    {
      double acc[P];
#pragma unroll
      for (int p = 0; p < P; ++p) acc[p] = 0.0;
#pragma unroll 1
      for (int i = 0; i < k; ++i) {
        const double f = ER[i * k];
#pragma unroll
        for (int p = 0; p < P; ++p) acc[p] = fma(f, live(p) ? V.ldp(i, p) : 0.0, acc[p]);
      }
#pragma unroll
      for (int p = 0; p < P; ++p) cur[p] = live(p) ? beta * acc[p] : 0.0;
    }
    __syncthreads();
  }

#pragma unroll
  for (int p = 0; p < P; ++p) {
    if (!live(p)) continue;
    asm volatile("" ::: "memory");
    int lx, ly;
    coords(lidx(p), lx, ly);
    const int rx = lx - b.h;
    const int ry = (b.ndim == 1) ? ly : ly - b.hy;
    if (AUG && lidx(p) == nloc) continue;
    if (rx < 0 || rx >= b.cx || ry < 0 || ry >= b.cy) continue;
    const int64_t g = (b.ndim == 1) ? (int64_t)(b.ox + rx)
                                    : (int64_t)(b.oy + ry) * b.n + (b.ox + rx);
    if (!isfinite(cur[p])) bad = true;
    x_out[b.x_off + g * b.ns + s] = cur[p];
  }
  int* status = b.status ? b.status : a.status;
  if (bad) atomicOr(status, kStatusNonFinite);
  if (tid == 0) {
    a.diag[(int64_t)b.diag * b.ns + s] = worst;
    if (!(worst <= b.tol)) atomicOr(status, isfinite(worst) ? kStatusNotConverged : kStatusNonFinite);
  }
}

// Fills the precomputed weights of blocks that carry them: row k of a block
// (stride doubles, the NT * P points of its launch shape) holds weight k of
// every box point; the augmented coordinate and the padding get zeros.
__global__ void krylov_weights_kernel(const KBlock* blocks, int stride, const double* coef) {
  const KBlock b = blocks[blockIdx.x];
  const int l = blockIdx.y * blockDim.x + threadIdx.x;
  if (b.wts == nullptr || l >= stride) return;
  const int nloc = b.Lx * b.Ly;
  double w[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (l < nloc) {
    const int ly = l / b.Lx, lx = l - ly * b.Lx;
    box_weights(b, b.coef ? b.coef : coef, lx, ly, w);
  }
  double* out = const_cast<double*>(b.wts);
#pragma unroll
  for (int k = 0; k < 5; ++k) out[(int64_t)k * stride + l] = w[k];
}

// ------------------------------------------------------------------ launch --

hipError_t launch_krylov_weights(const KBlock* blocks, int n_blocks, int nt, int pmax,
                                 const double* coef, hipStream_t st) {
  if (n_blocks == 0) return hipSuccess;
  const int stride = nt * pmax;
  hipLaunchKernelGGL(krylov_weights_kernel, dim3(n_blocks, (stride + 255) / 256), dim3(256), 0,
                     st, blocks, stride, coef);
  return hipGetLastError();
}

int krylov_big_max_m() { return kBigMaxM; }

int64_t krylov_big_pad(int nt, int pmax) { return (int64_t)nt * pmax; }
int krylov_big_max_n() { return kBigMaxN; }

size_t krylov_big_lds_bytes(int nt, int pmax, int m) {
  int64_t a, b2, c;
  return (size_t)big_lds_layout(nt, pmax, m, &a, &b2, &c) * 8;
}

// 256 threads up to 2048 points, 512 threads (two waves per SIMD, 256 VGPRs)
// with up to 18 points per lane above
void krylov_big_config(int nloc, int* nt, int* pmax) {
  if (nloc <= 1024) { *nt = 256; *pmax = 4; return; }
  if (nloc <= 2048) { *nt = 256; *pmax = 8; return; }
  if (nloc <= 4096) { *nt = 512; *pmax = 8; return; }
  if (nloc <= 6144) { *nt = 512; *pmax = 12; return; }
  if (nloc <= kBigMaxN) { *nt = 512; *pmax = 18; return; }
  *nt = 0; *pmax = 0;
}

template <int NT, int P, bool AUG>
static hipError_t launch_b(const KrylovArgs& a, int ns, size_t lds, hipStream_t st) {
  auto fn = krylov_big_kernel<NT, P, AUG>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)fn,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, dim3(a.n_blocks, ns), dim3(NT), lds, st, a);
  return hipGetLastError();
}

template <bool AUG>
static hipError_t launch_big_shape(const KrylovArgs& a, int ns, int nt, int pmax, size_t lds,
                                   hipStream_t st) {
  if (nt == 256 && pmax == 4) return launch_b<256, 4, AUG>(a, ns, lds, st);
  if (nt == 256 && pmax == 8) return launch_b<256, 8, AUG>(a, ns, lds, st);
  if (nt == 512 && pmax == 8) return launch_b<512, 8, AUG>(a, ns, lds, st);
  if (nt == 512 && pmax == 12) return launch_b<512, 12, AUG>(a, ns, lds, st);
  if (nt == 512 && pmax == 18) return launch_b<512, 18, AUG>(a, ns, lds, st);
  return hipErrorInvalidValue;
}

hipError_t launch_krylov_big(const KBlock* blocks, int n_blocks, int ns, int nt, int pmax,
                             size_t lds, const double* x_in, double* x_out, const double* coef,
                             double* vwork, double* diag, int* status, double* calib, int mode,
                             bool aug, hipStream_t st) {
  KrylovArgs a{blocks, x_in, x_out, coef, vwork, diag, status, calib, mode, n_blocks};
  if (n_blocks == 0) return hipSuccess;
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  return aug ? launch_big_shape<true>(a, ns, nt, pmax, lds, st)
             : launch_big_shape<false>(a, ns, nt, pmax, lds, st);
}

}  // namespace lem
