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
// v_j)/nu and stores both.  Registers hold only w across the two sweeps: u_j
// is read again from its row, and nu comes from Pythagoras,
// nu^2 = |u_j|^2 - |s|^2 (V has orthonormal columns), with an extra sweep
// that measures |u_j - V s| when that difference cancels badly (near an
// invariant subspace).  exp(H_m) is Pade [13/13] scaling and squaring in LDS.
#include "lem_device.hpp"
#include "lem_launch.h"

namespace lem {

constexpr int kBigMaxM = 40;     // Krylov dimension limit of this kernel
constexpr int kBigMaxN = 9216;   // box points (plus the augmented coordinate)
constexpr int kBigSlots = 128;   // reduction slots per wave: s at 0.., z at 64..

__host__ __device__ inline int64_t big_lds_layout(int NT, int m, int64_t* off_red,
                                                  int64_t* off_tot, int64_t* off_e) {
  int64_t d = (int64_t)(m + 1) * m;  // Hessenberg
  *off_red = d;
  d += (int64_t)(NT / 64) * kBigSlots;
  *off_tot = d;
  d += kBigSlots;
  *off_e = d;
  d += 7 * (int64_t)m * m + 2 * (NT / 64) + 4;  // expm_small: A, W (5), R, piv
  return d;
}

// The basis slice is addressed through a buffer resource: the slice base in
// scalar registers, the row and point-group offsets as one scalar, and a lane
// offset (tid * 8) shared by every row and point (64-bit per-lane addresses
// for every point would exhaust the register file).  Point p of a lane is
// local index tid + p * NT; lanes past the box read past the row end, which
// stays inside the slice and its padding (the planner pads every block's
// slices by NT * P doubles) and is discarded by the callers.
template <int NT>
struct BasisRows {
  __amdgpu_buffer_rsrc_t r;
  int row_bytes;
  uint32_t lane_off;
  typedef decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0)) raw_t;
  // this lane's point p of row `row`
  __device__ __forceinline__ double ldp(int row, int p) const {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                          r, lane_off, row * row_bytes + p * (NT * 8), 0));
  }
  __device__ __forceinline__ void stp(int row, int p, double v) const {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(raw_t, v), r, lane_off,
                                          row * row_bytes + p * (NT * 8), 0);
  }
  // any point l of row `row`
  __device__ __forceinline__ double ld(int row, uint32_t l) const {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, l * 8u, row * row_bytes, 0));
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
  big_lds_layout(NT, m, &ored, &otot, &oe);
  double* H = smem;
  double* red = smem + ored;  // [NT/64][kBigSlots]
  double* tot = smem + otot;  // workgroup totals of the slots
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
  const bool varcoef = b.mu_off >= 0;
  const double* mux = (b.coef ? b.coef : a.coef) + (varcoef ? b.mu_off : 0);
  const int64_t Ng = (b.ndim == 1) ? b.n : (int64_t)b.n * b.n;
  const double* muy = mux + Ng;

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

  // (dt_sub A_M v)_l at point p for the basis row starting at vj; couplings
  // leaving the box are dropped, the periodic wrap kept along an axis the box
  // spans whole; the augmented row (forced steps) is zero
  auto stencil = [&](int j, int p) __attribute__((always_inline)) {
    int l = (int)li(p);
    // recomputed per use: weights and neighbour offsets of every point would
    // otherwise be hoisted out of the Arnoldi loop (about 15 registers each)
    asm volatile("" : "+v"(l));
    int lx, ly;
    coords(l, lx, ly);
    double w0 = b.w0, wW = b.wW, wE = b.wE, wS = b.wS, wN = b.wN;
    if (varcoef) {
      const int gx = wrap(b.ox - b.h + lx, b.n);
      const int gy = (b.ndim == 1) ? 0 : wrap(b.oy - b.hy + ly, b.n);
      const int64_t g = (int64_t)gy * b.n + gx;
      const int64_t gw = (int64_t)gy * b.n + wrap(gx - 1, b.n);
      const int64_t gs = (int64_t)wrap(gy - 1, b.n) * b.n + gx;
      const double me = mux[g], mw = mux[gw];
      const double mn = b.ndim == 2 ? muy[g] : 0.0, ms = b.ndim == 2 ? muy[gs] : 0.0;
      const double sc = b.sub_scale;
      w0 = -(me + mw + mn + ms) * sc;
      if (b.varvel) {  // conservative centered advection by face velocities
        const double* axf = mux + 2 * Ng;
        const double ae = axf[g] * sc, aw = axf[gw] * sc;
        const double an = b.ndim == 2 ? axf[Ng + g] * sc : 0.0;
        const double as = b.ndim == 2 ? axf[Ng + gs] * sc : 0.0;
        w0 -= (ae - aw) + (an - as);
        wW = fma(mw, sc, aw);
        wE = fma(me, sc, -ae);
        wS = fma(ms, sc, as);
        wN = fma(mn, sc, -an);
      } else {
        wW = fma(mw, sc, b.chx);
        wE = fma(me, sc, -b.chx);
        wS = fma(ms, sc, b.chy);
        wN = fma(mn, sc, -b.chy);
      }
    }
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
    double r = w0 * V.ld(j, l);
    r = fma(wW, V.ld(j, lW), r);
    r = fma(wE, V.ld(j, lE), r);
    r = fma(wS, V.ld(j, lS), r);
    r = fma(wN, V.ld(j, lN), r);
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
        if (live(p)) V.stp(0, p, cur[p] * ib);  // u_0 = v_0
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
#pragma unroll
        for (int p = 0; p < P; ++p) {
          // one point's stencil loads in flight at a time (bounded registers)
          asm volatile("" ::: "memory");
          u[p] = live(p) ? V.ldp(j, p) : 0.0;
          w[p] = last ? 0.0 : stencil(j, p);
        }
        if constexpr (AUG) {
          if (!last) {
            const double ve = V.ld(j, nloc);
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
      double ss = 0.0, sz = 0.0;
      for (int i = 0; i < j; ++i) {
        ss = fma(tot[i], tot[i], ss);
        sz = fma(tot[i], tot[64 + i], sz);
      }
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
        double hs = 0.0;
        for (int i = 0; i < j; ++i) {
          const double hij = H[i * m + j - 1] + tot[i];
          hs = fma(hij, hij, hs);
        }
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
          double t = 0.0;
          for (int l = (i > 0 ? i - 1 : 0); l < j; ++l) {
            const double hil = (l == j - 1) ? hcorr : H[i * m + l];
            t = fma(hil, tot[l], t);
          }
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
      // u_{j+1} = (y - cj vt / nu) / nu overwrite rows j and j+1
      {
        double vt[P];
#pragma unroll
        for (int p = 0; p < P; ++p) vt[p] = live(p) ? V.ldp(j, p) : 0.0;
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
          V.stp(j, p, vt[p] * inv);
          V.stp(j + 1, p, (w[p] - cc * vt[p]) * inv);
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

// ------------------------------------------------------------------ launch --

int krylov_big_max_m() { return kBigMaxM; }

int64_t krylov_big_pad(int nt, int pmax) { return (int64_t)nt * pmax; }
int krylov_big_max_n() { return kBigMaxN; }

size_t krylov_big_lds_bytes(int nt, int m) {
  int64_t a, b2, c;
  return (size_t)big_lds_layout(nt, m, &a, &b2, &c) * 8;
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
