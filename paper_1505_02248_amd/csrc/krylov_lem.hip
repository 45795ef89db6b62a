// Batched Arnoldi-Krylov LEM step (gfx950).
//
// One workgroup advances one region M_i of the overlapping decomposition of
// section 3 (one ensemble member) by one step: gather the local state, then
// for each of nsub equal sub-steps build the Krylov basis of dt_sub * A_M
// (the local problem (4): the stencil on the box with the couplings to
// outside nodes dropped) by Arnoldi and set v <- beta V_m exp(H_m) e_1 (the
// Krylov action of section 4.3); finally write the core rows into the new
// state (step 3).  Saad's estimate beta h_{m+1,m} |e_m^T exp(H_m) e_1| is
// accumulated over the sub-steps and latched into the status word when above
// tolerance.  The basis stays in LDS whenever it fits (the planner chooses
// the Krylov dimension and sub-step count for that), otherwise it lives in a
// per-block slice of device memory read through the L2 (a buffer resource:
// row offset in a scalar register, point offset per lane), with the current
// direction also kept in LDS for the stencil product, and the columns follow
// the delayed re-orthogonalization described at the streamed branch.  With
// the basis in LDS each Arnoldi column takes three sweeps and two reductions:
//   * sweep 1: stencil product on the LDS-resident v_j fused with the first
//     Gram-Schmidt dots; one reduction;
//   * sweep 2: first update fused with the re-orthogonalization dots and the
//     squared norm of the updated vector; one reduction; the norm of the
//     twice-orthogonalized vector follows from Pythagoras (the second
//     correction is tiny), with an explicit reduction when cancellation is
//     severe (near an invariant subspace);
//   * sweep 3: second update, normalization, store of v_{j+1}.
// A forcing g, constant over the step, enters update (5) of section 3 as
// exp(dt A_M) v + phi_1(dt A_M)(dt g_M): that is the exponential of the
// augmented matrix [[dt A_M, dt g_M], [0, 0]] applied to [v; 1], so a forced
// block carries one extra coordinate (held at 1 by a zero row; its column is
// dt_sub g_M) and everything else is unchanged.
// Reductions of up to 32 values use a wave64 butterfly reduce-scatter
// (about one cross-lane exchange per value instead of six), then one LDS
// exchange between waves.  exp(H_m) is evaluated by scaling and squaring
// with the degree-18 Taylor polynomial (Paterson-Stockmeyer form), every
// matrix product on FP64 MFMA (v_mfma_f64_16x16x4) over 16- or 32-padded
// tiles in LDS.
#include <type_traits>

#include "lem_device.hpp"
#include "lem_launch.h"

namespace lem {

typedef double d4v __attribute__((ext_vector_type(4)));

constexpr int kLdsMaxM = 30;  // Krylov dimension limit of this kernel

// LDS layout in doubles; mirrored by krylov_lds_bytes() on the host.  An
// LDS-resident basis (vlds) comes first, followed by the Hessenberg, the
// reduction exchange and the exponential's work space.  A streamed basis
// leaves one row in LDS, the current direction u_j for the stencil product,
// which the exponential's work space reuses after the Arnoldi loop.
__host__ __device__ inline int64_t lds_layout(int NT, int m, int nloc, bool vlds, int aug,
                                              int64_t* off_h, int64_t* off_red, int64_t* off_e) {
  const int mp = m <= 16 ? 16 : 32;
  // expm work (A, X^2, X^3, X^4, two Horner terms, R) and per-wave norm maxima
  const int64_t e = 7 * (int64_t)mp * mp + (NT / 64 + 4 > 8 ? NT / 64 + 4 : 8);
  int64_t d;
  if (vlds) {
    d = (int64_t)(m + 1 + aug) * nloc;  // basis (+ the forcing column row)
  } else {
    *off_e = 0;
    d = e > nloc ? e : nloc;            // u_j, then the expm work
  }
  *off_h = d;
  d += (int64_t)(m + 1) * m;            // Hessenberg
  *off_red = d;
  d += (int64_t)(NT / 64) * 64 + 64;    // reduction exchange + scalars
  if (vlds) {
    *off_e = d;
    d += e;
  }
  return d;
}

// Workgroup sum of cnt <= 32 values (held per thread in v[0..cnt)); after the
// call every thread can read total(i) = sum_w red[w*32 + i].
template <int NT>
__device__ __forceinline__ void wg_reduce32(double (&v)[32], int cnt, double* red) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (cnt <= 8) {
    double t[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) t[i] = v[i];
    const double r = wave_reduce_scatter<8>(t);
    if ((lane & 7) == 0) red[wv * 32 + (lane >> 3)] = r;
  } else if (cnt <= 16) {
    double t[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) t[i] = v[i];
    const double r = wave_reduce_scatter<16>(t);
    if ((lane & 3) == 0) red[wv * 32 + (lane >> 2)] = r;
  } else {
    const double r = wave_reduce_scatter<32>(v);
    if ((lane & 1) == 0) red[wv * 32 + (lane >> 1)] = r;
  }
  __syncthreads();
}

template <int NT>
__device__ __forceinline__ double red_total(const double* red, int i) {
  double s = red[i];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w) s += red[w * 32 + i];
  return s;
}

// Same with 64 slots per wave (the paired dots of the streamed Arnoldi).
template <int NT>
__device__ __forceinline__ double red_total64(const double* red, int i) {
  double s = red[i];
#pragma unroll
  for (int w = 1; w < NT / 64; ++w) s += red[w * 64 + i];
  return s;
}

// C = A B for mp x mp matrices (mp = 16 or 32) in LDS, row-major, on FP64
// MFMA.  Waves take 16x16 output tiles round-robin.
// (all LDS reads of a tile are issued before its MFMAs: one wait per tile)
template <int NT, int MP>
__device__ __forceinline__ void mfma_matmul_mp(const double* A, const double* B, double* C) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  constexpr int TT = MP / 16, KS = MP / 4;
  for (int t = wv; t < TT * TT; t += NT / 64) {
    const int ti = t / TT, tj = t - ti * TT;
    double a[KS], bb[KS];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      a[k] = A[(ti * 16 + (lane & 15)) * MP + 4 * k + (lane >> 4)];
      bb[k] = B[(4 * k + (lane >> 4)) * MP + tj * 16 + (lane & 15)];
    }
    d4v acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < KS; ++k) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[k], bb[k], acc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      C[(ti * 16 + 4 * r + (lane >> 4)) * MP + tj * 16 + (lane & 15)] = acc[r];
  }
  __syncthreads();
}
template <int NT>
__device__ __forceinline__ void mfma_matmul(const double* A, const double* B, double* C,
                                            int mp) {
  if (mp == 16) mfma_matmul_mp<NT, 16>(A, B, C);
  else mfma_matmul_mp<NT, 32>(A, B, C);
}

// 1/k! for the degree-18 Taylor polynomial of exp
__host__ __device__ constexpr double inv_factorial(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= i;
  return 1.0 / f;
}

// exp(A) for the leading m x m block of the mp x mp matrix A in LDS (padding
// rows/columns zero): scaling so that ||A / 2^s||_1 <= 1, the degree-18 Taylor
// polynomial (truncation below 1/19! ~ 8e-18 relative) in Paterson-Stockmeyer
// form -- X^2, X^3, X^4, then a Horner recursion in X^4 over blocks of four
// terms, seven products in all -- and s squarings, every step an FP64 MFMA
// product or an elementwise update (no pivoted solve: its chain of per-column
// barriers dominated the step's end on small boxes).  Work W = 5 mp^2, result
// R (mp^2); piv >= NT/64 holds the per-wave norm maxima.
template <int NT>
__device__ __forceinline__ void expm_mfma(double* A, int m, int mp, double* W, double* R,
                                          double* piv) {
  const int tid = threadIdx.x;
  const int mm = mp * mp;
  double* X2 = W;
  double* X3 = W + mm;
  double* X4 = W + 2 * mm;
  double* T = W + 3 * mm;
  double* S = W + 4 * mm;
  double cs = 0.0;
  for (int j = tid; j < m; j += NT) {
    double t = 0.0;
    for (int i = 0; i < m; ++i) t += fabs(A[i * mp + j]);
    cs = fmax(cs, t);
  }
  cs = wave_max(cs);
  if (NT > 64) {
    if ((tid & 63) == 0) piv[tid >> 6] = cs;
    __syncthreads();
    cs = 0.0;
    for (int w = 0; w < NT / 64; ++w) cs = fmax(cs, piv[w]);
    __syncthreads();
  }
  int s = 0;  // a non-finite norm leaves s = 0 (the result is then non-finite too)
  if (cs > 1.0 && cs < 1e300) s = min(60, (int)ceil(log2(cs)));
  if (s > 0) {
    for (int idx = tid; idx < mm; idx += NT) A[idx] = ldexp(A[idx], -s);
    __syncthreads();
  }
  mfma_matmul<NT>(A, A, X2, mp);
  mfma_matmul<NT>(X2, A, X3, mp);
  mfma_matmul<NT>(X2, X2, X4, mp);
  // block j of four terms: c_4j I + c_4j+1 X + c_4j+2 X^2 + c_4j+3 X^3 (the
  // identity on the leading block only, so the padding stays zero)
  auto block = [&](int j, int idx) -> double {
    const int i = idx / mp, k = idx - i * mp;
    const double id = (i == k && i < m) ? inv_factorial(4 * j) : 0.0;
    double v = id + inv_factorial(4 * j + 1) * A[idx] + inv_factorial(4 * j + 2) * X2[idx];
    if (4 * j + 3 <= 18) v += inv_factorial(4 * j + 3) * X3[idx];
    return v;
  };
  // T = c16 I + c17 X + c18 X^2, then T = X^4 T + block(j) for j = 3, 2, 1, 0
  for (int idx = tid; idx < mm; idx += NT) T[idx] = block(4, idx);
  __syncthreads();
  for (int j = 3; j >= 0; --j) {
    mfma_matmul<NT>(X4, T, S, mp);
    for (int idx = tid; idx < mm; idx += NT) T[idx] = S[idx] + block(j, idx);
    __syncthreads();
  }
  double* src = T;
  double* dst = X2;
  for (int q = 0; q < s; ++q) {
    mfma_matmul<NT>(src, src, dst, mp);
    double* t = src; src = dst; dst = t;
  }
  for (int idx = tid; idx < mm; idx += NT) R[idx] = src[idx];
  __syncthreads();
}

typedef __attribute__((address_space(1))) double gdouble;

// One workgroup per (region, ensemble member).  VLDS: basis in LDS; else in
// a per-block slice of device memory (read through the L2).  Points per
// thread P; up to 8 points keep their stencil weights in registers.
template <int NT, int P, bool VLDS, bool AUG>
__global__ __launch_bounds__(NT) void krylov_lds_kernel(KrylovArgs a) {
  constexpr int CH = P >= 16 ? 2 : (P >= 8 ? 2 : (P >= 4 ? 4 : 8));  // rows per chunk
  constexpr int CHS = CH;  // rows per load batch of the streamed sweeps
  // stencil weights in registers for up to 8 points (not in the wide
  // streamed shapes, whose register budget is 128 per lane)
  constexpr bool PREW = P <= 8 && NT <= 256;
  typedef typename std::conditional<VLDS, double*, gdouble*>::type VPtr;
  extern __shared__ double smem[];
  const int tid = threadIdx.x;
  const int s = blockIdx.y;
  const KBlock b = a.blocks[blockIdx.x];
  const int m = b.m;
  const int mp = m <= 16 ? 16 : 32;
  const int nloc = b.Lx * b.Ly;   // points of the box
  const int nlv = nloc + (AUG ? 1 : 0);  // basis row length (plus the augmented coordinate)
  int64_t oh, ored, oe;
  const int64_t ostage = lds_layout(NT, m, nlv, VLDS, AUG ? 1 : 0, &oh, &ored, &oe);
  VPtr V;
  if constexpr (VLDS) {
    V = smem;
  } else {
    double* g = (b.vwork ? b.vwork : a.vwork + b.v_off) + (int64_t)s * (m + 1 + (AUG ? 1 : 0)) * nlv;
    V = (VPtr)g;
  }
  // A streamed basis is addressed through a buffer resource: the slice base
  // and the row offset in scalar registers (readfirstlane: the compiler may
  // hold the uniform row index in a vector register), the point offset per
  // lane, so the sweeps hold no 64-bit address per load.
  const __amdgpu_buffer_rsrc_t vrs =
      __builtin_amdgcn_make_buffer_rsrc((void*)V, 0, 0x7ffffff0, 0x00020000);
  double* H = smem + oh;
  double* red = smem + ored;  // [NT/64][32] (streamed: [NT/64][64])
  double* tot = red + (NT / 64) * 64;  // 64 workgroup totals (streamed sweeps)
  double* EA = smem + oe;
  double* U = smem;  // streamed basis: u_j during the Arnoldi loop (aliases EA)
  double* EW = EA + mp * mp;
  double* ER = EW + 5 * mp * mp;
  double* piv = ER + mp * mp;

  const double* x_in = b.xin ? b.xin : a.x_in;
  double* x_out = b.xout ? b.xout : a.x_out;
  const bool varcoef = b.mu_off >= 0;
  const double* mux = (b.coef ? b.coef : a.coef) + (varcoef ? b.mu_off : 0);
  const int64_t Ng = (b.ndim == 1) ? b.n : (int64_t)b.n * b.n;
  const double* muy = mux + Ng;
  // Wide streamed shapes recompute the stencil weights per use; their
  // diffusion coefficients are staged in LDS once (after the work areas):
  // cmx[ly][lx + 1] = mu_x at box point (lx, ly) for lx = -1 .. Lx-1 and
  // cmy[ly + 1][lx] = mu_y for ly = -1 .. Ly-1, wrapped on the periodic grid.
  const bool stage = !VLDS && NT >= 512 && varcoef && !b.varvel && b.stage;
  const int sx = b.Lx + 1;
  double* cmx = smem + ostage;
  double* cmy = cmx + (int64_t)sx * b.Ly;
  if (stage) {
    for (int e = tid; e < sx * b.Ly; e += NT) {
      const int ly = e / sx, lx = e - ly * sx - 1;
      const int gx = wrap(b.ox - b.h + lx, b.n);
      const int gy = (b.ndim == 1) ? 0 : wrap(b.oy - b.hy + ly, b.n);
      cmx[e] = mux[(int64_t)gy * b.n + gx];
    }
    if (b.ndim == 2) {
      for (int e = tid; e < b.Lx * (b.Ly + 1); e += NT) {
        const int ly = e / b.Lx - 1, lx = e - (ly + 1) * b.Lx;
        const int gx = wrap(b.ox - b.h + lx, b.n);
        const int gy = wrap(b.oy - b.hy + ly, b.n);
        cmy[e] = muy[(int64_t)gy * b.n + gx];
      }
    }
    __syncthreads();
  }

  // Point p of this thread is local index tid + p*NT; its box coordinates
  // are recomputed where needed (keeping them would cost 2P registers).
  int li[P];
  bool live[P];
  int xy[P];  // box coordinates, lx | ly << 16 (one division per point, once)
#pragma unroll
  for (int p = 0; p < P; ++p) {
    const int l = tid + p * NT;
    live[p] = l < nlv;
    li[p] = live[p] ? l : 0;  // safe index for lanes past the box
    const int ly = li[p] / b.Lx;
    xy[p] = (li[p] - ly * b.Lx) | (ly << 16);
  }
  // basis row i at this thread's point p (lanes past the box: point 0)
  auto vld = [&](int i, int p) __attribute__((always_inline)) -> double {
    if constexpr (VLDS) {
      return V[(int64_t)i * nlv + li[p]];
    } else {
      return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(
                                            vrs, (uint32_t)li[p] * 8u,
                                            __builtin_amdgcn_readfirstlane(i * nlv * 8), 0));
    }
  };
  auto vst = [&](int i, int p, double v) __attribute__((always_inline)) {
    if constexpr (VLDS) {
      V[(int64_t)i * nlv + li[p]] = v;
    } else {
      typedef decltype(__builtin_amdgcn_raw_buffer_load_b64(vrs, 0, 0, 0)) raw_t;
      __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(raw_t, v), vrs,
                                            (uint32_t)li[p] * 8u,
                                            __builtin_amdgcn_readfirstlane(i * nlv * 8), 0);
    }
  };
  auto coords = [&](int p, int& lx, int& ly) __attribute__((always_inline)) {
    int c = xy[p];
    if constexpr (!PREW) asm volatile("" : "+v"(c));  // recompute per use: no hoisting
    lx = c & 0xffff;
    ly = c >> 16;
  };
  // stencil weights of point p (couplings leaving the box are dropped)
  auto weights = [&](int p, double& w0, double& wW, double& wE, double& wS, double& wN) __attribute__((always_inline)) {
    int lx, ly;
    coords(p, lx, ly);
    w0 = b.w0; wW = b.wW; wE = b.wE; wS = b.wS; wN = b.wN;
    if (varcoef) {
      int opq = 0;
      if constexpr (!PREW) asm volatile("" : "+s"(opq));  // recompute per use: no hoisting
      lx += opq;
      double me, mw, mn = 0.0, ms = 0.0;
      int64_t g = 0, gw = 0, gs = 0;
      if (stage) {
        const int sy = min(ly, b.Ly - 1);  // the augmented row reads a valid entry
        me = cmx[sy * sx + lx + 1];
        mw = cmx[sy * sx + lx];
        if (b.ndim == 2) {
          mn = cmy[(sy + 1) * b.Lx + lx];
          ms = cmy[sy * b.Lx + lx];
        }
      } else {
        const int gx = wrap(b.ox - b.h + lx, b.n);
        const int gy = (b.ndim == 1) ? 0 : wrap(b.oy - b.hy + ly, b.n);
        g = (int64_t)gy * b.n + gx;
        gw = (int64_t)gy * b.n + wrap(gx - 1, b.n);
        gs = (int64_t)wrap(gy - 1, b.n) * b.n + gx;
        me = mux[g];
        mw = mux[gw];
        if (b.ndim == 2) {
          mn = muy[g];
          ms = muy[gs];
        }
      }
      const double sc = b.sub_scale;
      w0 = -(me + mw + mn + ms) * sc;
      if (b.varvel) {  // conservative centered advection by face velocities
        const double* axf = mux + 2 * Ng;
        const double ae = axf[g] * sc, aw = axf[gw] * sc;
        double an = 0.0, as = 0.0;
        if (b.ndim == 2) {
          an = axf[Ng + g] * sc;
          as = axf[Ng + gs] * sc;
        }
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
    if (!live[p] || (AUG && li[p] == nloc)) w0 = wW = wE = wS = wN = 0.0;  // augmented row: zero
    if (!(b.periodic & 1)) {
      if (lx == 0) wW = 0.0;
      if (lx == b.Lx - 1) wE = 0.0;
    }
    if (!(b.periodic & 2)) {
      if (ly == 0) wS = 0.0;
      if (ly == b.Ly - 1) wN = 0.0;
    }
    if (b.ndim == 1) wS = wN = 0.0;
  };
  // Forced steps: the augmented column dt_sub g_M (zero on the augmented
  // row) is kept as row m+1 of the basis storage, written once here.
  if constexpr (AUG) {
#pragma unroll
    for (int p = 0; p < P; ++p) {
      if (!live[p]) continue;
      int lx, ly;
      coords(p, lx, ly);
      vst(m + 1, p, li[p] == nloc ? 0.0
                    : b.gscale * b.force[b.x_off + gather_index(b, lx, ly) * b.ns + s]);
    }
    __syncthreads();
  }
  double pw[PREW ? P : 1][5];
  if constexpr (PREW) {
#pragma unroll
    for (int p = 0; p < P; ++p) weights(p, pw[p][0], pw[p][1], pw[p][2], pw[p][3], pw[p][4]);
  }
  // (dt_sub A_M v)_l at point p, v the basis row starting at vj
  auto stencil = [&](auto vj, int p) __attribute__((always_inline)) {
    double w0, wW, wE, wS, wN;
    if constexpr (PREW) {
      w0 = pw[p][0]; wW = pw[p][1]; wE = pw[p][2]; wS = pw[p][3]; wN = pw[p][4];
    } else {
      weights(p, w0, wW, wE, wS, wN);
    }
    int l = li[p];
    if constexpr (!PREW) asm volatile("" : "+v"(l));  // neighbour offsets per use: no hoisting
    // Neighbours wrap along the axes the box spans whole; on the other edges
    // (zero weight) and for points without couplings (lanes past the box, the
    // augmented coordinate) they fall back to the point itself, so all five
    // reads are valid, finite and issued together (a zero weight adds 0).
    int lx, ly;
    coords(p, lx, ly);
    int lW = l - 1, lE = l + 1, lS = l - b.Lx, lN = l + b.Lx;
    if (lx == 0) lW = (b.periodic & 1) ? lW + b.Lx : l;
    if (lx == b.Lx - 1) lE = (b.periodic & 1) ? lE - b.Lx : l;
    if (b.ndim == 1) {
      lS = lN = l;
    } else {
      if (ly == 0) lS = (b.periodic & 2) ? lS + nloc : l;
      if (ly == b.Ly - 1) lN = (b.periodic & 2) ? lN - nloc : l;
    }
    if (!live[p] || (AUG && l == nloc)) lW = lE = lS = lN = l;
    double r = w0 * vj[l];
    r = fma(wW, vj[lW], r);
    r = fma(wE, vj[lE], r);
    r = fma(wS, vj[lS], r);
    r = fma(wN, vj[lN], r);
    return r;
  };
  // forced steps: w += (augmented column) x (augmented coordinate of row j)
  auto add_forcing = [&](int j, double (&w)[P]) __attribute__((always_inline)) {
    if constexpr (!AUG) return;
    const double ve = V[(int64_t)j * nlv + nloc];
#pragma unroll
    for (int p = 0; p < P; ++p) w[p] = fma(vld(m + 1, p), ve, w[p]);
  };

  double cur[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    int lx, ly;
    coords(p, lx, ly);
    cur[p] = !live[p] ? 0.0
             : (AUG && li[p] == nloc) ? 1.0  // the augmented coordinate starts (and stays) at 1
                             : x_in[b.x_off + gather_index(b, lx, ly) * b.ns + s];
  }

  double vv[32];
  auto norm2 = [&](const double (&x)[P]) __attribute__((always_inline)) {
    double t = 0.0;
#pragma unroll
    for (int p = 0; p < P; ++p) t = fma(x[p], x[p], t);
#pragma unroll
    for (int i = 0; i < 32; ++i) vv[i] = 0.0;
    vv[0] = t;
    wg_reduce32<NT>(vv, 1, red);
    const double r = red_total<NT>(red, 0);
    __syncthreads();
    return r;
  };
  // Sweeps over the basis rows 0..jj in chunks of CH rows: all loads of a
  // chunk are in flight before the first use.  Rows past jj are clamped to jj
  // (valid data) and enter with a zero weight or are discarded; lanes past
  // the box read point 0 and contribute zero.
  auto dots_chunked = [&](int jj, const double (&x)[P], double (&out)[32]) __attribute__((always_inline)) {
#pragma unroll
    for (int c = 0; c < (VLDS ? 32 / CH : 0); ++c) {
      if (c * CH <= jj) {
        // keeps the loads of later chunks from being hoisted above this one
        // (which would multiply the live registers)
        asm volatile("" ::: "memory");
        double vals[CH][P];
#pragma unroll
        for (int q = 0; q < CH; ++q) {
          const int i = min(c * CH + q, jj);
#pragma unroll
          for (int p = 0; p < P; ++p) vals[q][p] = vld(i, p);
        }
#pragma unroll
        for (int q = 0; q < CH; ++q) {
          double t = 0.0;
#pragma unroll
          for (int p = 0; p < P; ++p) t = fma(live[p] ? vals[q][p] : 0.0, x[p], t);
          out[c * CH + q] = (c * CH + q <= jj) ? t : 0.0;
        }
      }
    }
  };
  // x -= sum_{i<=jj} total_i v_i (totals from the reduction exchange); the
  // totals go to column jj of H (assigned, or added when `second`); returns
  // sum total_i^2.
  auto update_chunked = [&](int jj, double (&x)[P], bool second) __attribute__((always_inline)) {
    double ss = 0.0;
    for (int i0 = 0; i0 <= jj; i0 += CH) {
      double vals[CH][P], hc[CH];
#pragma unroll
      for (int q = 0; q < CH; ++q) {
        const int i = min(i0 + q, jj);
        const double t = red_total<NT>(red, i);
        hc[q] = (i0 + q <= jj) ? t : 0.0;
#pragma unroll
        for (int p = 0; p < P; ++p) vals[q][p] = vld(i, p);
      }
#pragma unroll
      for (int q = 0; q < CH; ++q) {
        ss = fma(hc[q], hc[q], ss);
        if (tid == 0 && i0 + q <= jj) {
          if (second) H[(i0 + q) * m + jj] += hc[q];
          else H[(i0 + q) * m + jj] = hc[q];
        }
#pragma unroll
        for (int p = 0; p < P; ++p)
          x[p] = fma(-hc[q], live[p] ? vals[q][p] : 0.0, x[p]);
      }
    }
    return ss;
  };
  // Totals of <v_i, x> for i <= jj (and, with `norm`, of <x, x> in slot
  // jj + 1), readable through red_total afterwards.  LDS-resident bases reduce
  // all values at once with the butterfly; streamed bases (many points per
  // thread) reduce row by row across the wave and store the wave totals at
  // dynamic LDS slots, which keeps no 32-value register array alive.
  auto reduce_dots = [&](int jj, const double (&x)[P], bool norm) __attribute__((always_inline)) {
    if constexpr (VLDS) {
#pragma unroll
      for (int i = 0; i < 32; ++i) vv[i] = 0.0;
      dots_chunked(jj, x, vv);
      int cnt = jj + 1;
      if (norm) {
        double t = 0.0;
#pragma unroll
        for (int p = 0; p < P; ++p) t = fma(x[p], x[p], t);
        // the norm goes to the last slot of the butterfly width (a static
        // index: a store at jj + 1 would be an indexed store into scratch)
        if (jj + 2 <= 8) { vv[7] = t; cnt = 8; }
        else if (jj + 2 <= 16) { vv[15] = t; cnt = 16; }
        else { vv[31] = t; cnt = 32; }
      }
      wg_reduce32<NT>(vv, cnt, red);
      return norm ? cnt - 1 : -1;
    } else {
      const int lane = tid & 63, wv = tid >> 6;
#pragma unroll 1
      for (int i0 = 0; i0 <= jj; i0 += CH) {
        double vals[CH][P];
#pragma unroll
        for (int q = 0; q < CH; ++q) {
          const int i = min(i0 + q, jj);
#pragma unroll
          for (int p = 0; p < P; ++p) vals[q][p] = vld(i, p);
        }
#pragma unroll
        for (int q = 0; q < CH; ++q) {
          double t = 0.0;
#pragma unroll
          for (int p = 0; p < P; ++p) t = fma(live[p] ? vals[q][p] : 0.0, x[p], t);
          t = wave_sum(t);
          if (lane == 0 && i0 + q <= jj) red[wv * 32 + i0 + q] = t;
        }
      }
      if (norm) {
        double t = 0.0;
#pragma unroll
        for (int p = 0; p < P; ++p) t = fma(x[p], x[p], t);
        t = wave_sum(t);
        if (lane == 0) red[wv * 32 + jj + 1] = t;
      }
      __syncthreads();
      return norm ? jj + 1 : -1;
    }
  };
  auto store_row = [&](int i, const double (&x)[P], double scale) __attribute__((always_inline)) {
#pragma unroll
    for (int p = 0; p < P; ++p)
      if (live[p]) vst(i, p, x[p] * scale);
  };

  const double beta0 = sqrt(norm2(cur));
  double worst = 0.0;
  bool bad = !isfinite(beta0);
  const int nsub = (a.mode == 1) ? 1 : b.nsub;

  for (int sub = 0; sub < nsub; ++sub) {
    const double beta = (sub == 0) ? beta0 : sqrt(norm2(cur));
    if (!(beta > 0.0) || !isfinite(beta)) {
      if (!isfinite(beta)) bad = true;
      break;
    }
    store_row(0, cur, 1.0 / beta);
    if constexpr (!VLDS) {
      const double ib = 1.0 / beta;
#pragma unroll
      for (int p = 0; p < P; ++p)
        if (live[p]) U[li[p]] = cur[p] * ib;
    }
    for (int idx = tid; idx < (m + 1) * m; idx += NT) H[idx] = 0.0;
    __syncthreads();

    int k = m;
    if constexpr (VLDS) {
      for (int j = 0; j < m; ++j) {
        double w[P];
        // sweep 1: stencil product, first dots
  #pragma unroll
        for (int p = 0; p < P; ++p) w[p] = stencil(V + (int64_t)j * nlv, p);
        add_forcing(j, w);
        reduce_dots(j, w, false);
        // sweep 2: first update, second dots and the squared norm
        update_chunked(j, w, false);
        __syncthreads();  // everyone has read red before it is reused
        const int nslot = reduce_dots(j, w, true);  // totals 0..j and the squared norm
        // sweep 3: second update, norm, store
        const double e2 = update_chunked(j, w, true);
        const double n1 = red_total<NT>(red, nslot);
        double hn2 = n1 - e2;
        __syncthreads();
        if (!(hn2 > 1e-4 * n1)) hn2 = norm2(w);  // severe cancellation: measure
        const double hn = sqrt(fmax(hn2, 0.0));
        // |column j of H|^2, lane i holding row i (every wave sums it itself)
        const int ln = tid & 63;
        const double hv = ln <= j ? H[ln * m + j] : 0.0;
        const double hs = wave_sum(hv * hv);
        if (tid == 0) H[(j + 1) * m + j] = hn;
        if (!(hn > 1e-14 * sqrt(hs + hn * hn))) {  // invariant subspace reached
          k = j + 1;
          __syncthreads();
          break;
        }
        store_row(j + 1, w, 1.0 / hn);
        __syncthreads();
      }
    } else {
      // Streamed basis: Arnoldi with delayed re-orthogonalization (DCGS2:
      // Swirydowicz et al. 2021; Bielich et al. 2022).  Row j of V holds u_j,
      // the new direction projected once.  Column j fuses, in one sweep over
      // the rows i < j, the re-orthogonalization dots s = V^T u_j with the
      // projection dots z = V^T w of w = A u_j, then one update sweep forms
      //   v_j = (u_j - V s) / nu,   nu = |u_j - V s|  (measured),
      //   u_{j+1} = (w - V z - (v_j^T w) v_j) / nu
      // so every row is read twice per column instead of four times.  The
      // Hessenberg column j-1 is completed with s and nu (u_j = nu v_j + V s),
      // and column j is (V_j^T w - Hbar_{j-1} s) / nu, the projections of
      // A v_j = (w - A V_{j-1} s) / nu.  Column m-1 is completed by a last
      // pass without a new direction.
      const int lane = tid & 63, wv = tid >> 6;
      double u[P];
      const double ib = 1.0 / beta;  // row 0 holds cur * ib (store_row)
#pragma unroll
      for (int p = 0; p < P; ++p) u[p] = live[p] ? cur[p] * ib : 0.0;
      for (int j = 0; j <= m; ++j) {
        const bool last = j == m;
        double w[P];
#pragma unroll
        for (int p = 0; p < P; ++p) w[p] = last ? 0.0 : stencil(U, p);
        if (!last) add_forcing(j, w);
        // sweep A: s_i at slot i, z_i at slot 32 + i, |u|^2 at 31, u^T w at 63.
        // Rows go in groups of GR; the 2*GR partial sums of a group are
        // reduced across the wave at once by the butterfly reduce-scatter
        // (lane l ends with the total of value l / (32 / GR)).
        constexpr int GR = (P >= 16 || NT >= 1024) ? 4 : 8;  // 1024 threads: 128 VGPRs
#pragma unroll 1
        for (int i0 = 0; i0 < j; i0 += GR) {
          double t[2 * GR];
#pragma unroll
          for (int q = 0; q < 2 * GR; ++q) t[q] = 0.0;
#pragma unroll
          for (int q0 = 0; q0 < GR; q0 += CHS) {
            // keeps the loads of later rows from being hoisted above these
            asm volatile("" ::: "memory");
            double vals[CHS][P];
#pragma unroll
            for (int q = 0; q < CHS; ++q) {
              const int i = min(i0 + q0 + q, j - 1);
#pragma unroll
              for (int p = 0; p < P; ++p) vals[q][p] = vld(i, p);
            }
#pragma unroll
            for (int q = 0; q < CHS; ++q) {
              double ts = 0.0, tz = 0.0;
#pragma unroll
              for (int p = 0; p < P; ++p) {
                const double vq = live[p] ? vals[q][p] : 0.0;
                ts = fma(vq, u[p], ts);
                tz = fma(vq, w[p], tz);
              }
              const bool ok = i0 + q0 + q < j;
              t[q0 + q] = ok ? ts : 0.0;
              t[GR + q0 + q] = ok ? tz : 0.0;
            }
          }
          const double r = wave_reduce_scatter<2 * GR>(t);
          constexpr int LPV = 32 / GR;  // lanes per value
          const int v = lane / LPV, row = i0 + (v % GR);
          if (lane % LPV == 0 && row < j) red[wv * 64 + (v < GR ? row : 32 + row)] = r;
        }
        {
          double ta = 0.0, tb = 0.0;
#pragma unroll
          for (int p = 0; p < P; ++p) {
            ta = fma(u[p], u[p], ta);
            tb = fma(u[p], w[p], tb);
          }
          ta = wave_sum(ta);
          tb = wave_sum(tb);
          if (lane == 0) {
            red[wv * 64 + 31] = ta;
            red[wv * 64 + 63] = tb;
          }
        }
        __syncthreads();
        // one thread per slot sums the wave partials, so that the sweeps below
        // read each total once instead of once per wave
        if (tid < 64) tot[tid] = red_total64<NT>(red, tid);
        __syncthreads();
        // sweep B: vt = u - V s, y = w - V z, and |vt|^2 (slot 30)
        double vt[P], y[P];
#pragma unroll
        for (int p = 0; p < P; ++p) { vt[p] = u[p]; y[p] = w[p]; }
        double sz = 0.0;
#pragma unroll 1
        for (int i0 = 0; i0 < j; i0 += CHS) {
          double vals[CHS][P], sc[CHS], zc[CHS];
#pragma unroll
          for (int q = 0; q < CHS; ++q) {
            const int i = min(i0 + q, j - 1);
            const bool ok = i0 + q < j;
            sc[q] = ok ? tot[i] : 0.0;
            zc[q] = ok ? tot[32 + i] : 0.0;
#pragma unroll
            for (int p = 0; p < P; ++p) vals[q][p] = vld(i, p);
          }
#pragma unroll
          for (int q = 0; q < CHS; ++q) {
            sz = fma(sc[q], zc[q], sz);
#pragma unroll
            for (int p = 0; p < P; ++p) {
              const double vq = live[p] ? vals[q][p] : 0.0;
              vt[p] = fma(-sc[q], vq, vt[p]);
              y[p] = fma(-zc[q], vq, y[p]);
            }
          }
        }
        {
          double tn = 0.0;
#pragma unroll
          for (int p = 0; p < P; ++p) tn = fma(vt[p], vt[p], tn);
          tn = wave_sum(tn);
          if (lane == 0) red[wv * 64 + 30] = tn;
        }
        __syncthreads();
        const double nu = sqrt(fmax(red_total64<NT>(red, 30), 0.0));
        const double bw = tot[63];  // u^T w
        // complete column j-1: H[i][j-1] += s_i, H[j][j-1] = nu
        bool brk = false;
        if (j > 0) {
          // |corrected column j-1|^2, lane i holding row i (every wave sums it)
          const double hij = lane < j ? H[lane * m + j - 1] + tot[lane] : 0.0;
          const double hs = wave_sum(hij * hij);
          brk = !(nu > 1e-14 * sqrt(hs + nu * nu));  // invariant subspace reached
        } else {
          brk = !(nu > 0.0);
        }
        __syncthreads();  // every thread has read column j-1 before it is rewritten
        // thread i <= j: corrected H[i][j-1], and (unless stopping) the new
        // column H[i][j] = (z_i - t_i) / nu with t = Hbar_{j-1} s (the
        // corrected Hessenberg of columns < j), H[j][j] = (v_j^T w - t_j) / nu
        const double cj = (bw - sz) / nu;  // v_j^T w
        if (tid <= j) {
          const int i = tid;
          double hcorr = 0.0;
          if (j > 0) {
            hcorr = (i < j) ? H[i * m + j - 1] + tot[i] : nu;
          }
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
            const double num = (i < j) ? tot[32 + i] : cj;
            H[i * m + j] = (num - t) / nu;
          }
          if (j > 0) H[i * m + j - 1] = hcorr;
        }
        if (brk || last) {
          k = j > 0 ? j : 0;
          __syncthreads();
          break;
        }
        // v_j and u_{j+1}
        const double inv = 1.0 / nu, cc = cj * inv;
#pragma unroll
        for (int p = 0; p < P; ++p) {
          const double vj = vt[p] * inv;
          u[p] = (y[p] - cc * vt[p]) * inv;
          if (live[p]) {
            vst(j, p, vj);
            vst(j + 1, p, u[p]);
            U[li[p]] = u[p];  // every stencil read of u_j preceded the barriers above
          } else {
            u[p] = 0.0;
          }
        }
        __syncthreads();
      }
    }

    if (a.mode == 1) {
      double* out = a.calib + ((int64_t)b.diag * b.ns + s) * (2 + (m + 1) * m);
      for (int idx = tid; idx < (m + 1) * m; idx += NT) out[2 + idx] = H[idx];
      if (tid == 0) { out[0] = beta; out[1] = (double)k; }
      return;
    }

    // exp(H_k) e_1 on MFMA
    const int kp = k <= 16 ? 16 : 32;
    for (int idx = tid; idx < kp * kp; idx += NT) {
      const int i = idx / kp, jj = idx - i * kp;
      EA[idx] = (i < k && jj < k) ? H[i * m + jj] : 0.0;
    }
    __syncthreads();
    expm_mfma<NT>(EA, k, kp, EW, ER, piv);
    const double hk = H[k * m + (k - 1)];
    worst += beta * hk * fabs(ER[(k - 1) * kp]) / beta0;
    {
      double acc[P];
#pragma unroll
      for (int p = 0; p < P; ++p) acc[p] = 0.0;
      for (int i0 = 0; i0 < k; i0 += CH) {
        double vals[CH][P], f[CH];
#pragma unroll
        for (int q = 0; q < CH; ++q) {
          const int i = min(i0 + q, k - 1);
          f[q] = (i0 + q < k) ? ER[i * kp] : 0.0;
#pragma unroll
          for (int p = 0; p < P; ++p) vals[q][p] = vld(i, p);
        }
#pragma unroll
        for (int q = 0; q < CH; ++q)
#pragma unroll
          for (int p = 0; p < P; ++p) acc[p] = fma(f[q], live[p] ? vals[q][p] : 0.0, acc[p]);
      }
#pragma unroll
      for (int p = 0; p < P; ++p) cur[p] = live[p] ? beta * acc[p] : 0.0;
    }
    __syncthreads();
  }

#pragma unroll
  for (int p = 0; p < P; ++p) {
    if (!live[p]) continue;
    int lx, ly;
    coords(p, lx, ly);
    const int rx = lx - b.h;
    const int ry = (b.ndim == 1) ? ly : ly - b.hy;
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

size_t krylov_lds_bytes(int nt, int m, int nloc, bool vlds, int aug) {
  int64_t a, b2, c;
  return (size_t)lds_layout(nt, m, nloc, vlds, aug, &a, &b2, &c) * 8;
}

size_t krylov_stage_bytes(int nt, bool vlds, bool varcoef, bool varvel, int ndim, int lx,
                          int ly) {
  if (vlds || nt < 512 || !varcoef || varvel) return 0;
  return ((size_t)(lx + 1) * ly + (ndim == 2 ? (size_t)lx * (ly + 1) : 0)) * 8;
}

int krylov_lds_max_m() { return kLdsMaxM; }

// Launch shape for a box of nloc points: threads and points per thread.
void krylov_lds_config(int ndim, int nloc, int* nt, int* pmax) {
  if (ndim == 1 && nloc <= 128) { *nt = 64; *pmax = 2; return; }
  if (ndim == 1 && nloc <= 512) { *nt = 64; *pmax = 8; return; }
  if (nloc <= 1024) { *nt = 256; *pmax = 4; return; }
  if (nloc <= 2048) { *nt = 256; *pmax = 8; return; }
  if (nloc <= 4096) { *nt = 1024; *pmax = 4; return; }  // streamed basis only
  *nt = 0; *pmax = 0;  // larger boxes would spill registers: not supported
}

template <int NT, int P, bool VLDS, bool AUG>
static hipError_t launch_l(const KrylovArgs& a, int ns, size_t lds, hipStream_t st) {
  auto fn = krylov_lds_kernel<NT, P, VLDS, AUG>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)fn,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(fn, dim3(a.n_blocks, ns), dim3(NT), lds, st, a);
  return hipGetLastError();
}

template <bool AUG>
static hipError_t launch_shape(const KrylovArgs& a, int ns, int nt, int pmax, bool vlds,
                               size_t lds, hipStream_t st) {
  if (vlds) {
    if (nt == 64 && pmax == 2) return launch_l<64, 2, true, AUG>(a, ns, lds, st);
    if (nt == 64 && pmax == 8) return launch_l<64, 8, true, AUG>(a, ns, lds, st);
    if (nt == 256 && pmax == 4) return launch_l<256, 4, true, AUG>(a, ns, lds, st);
    if (nt == 256 && pmax == 8) return launch_l<256, 8, true, AUG>(a, ns, lds, st);
    return hipErrorInvalidValue;
  }
  if (nt == 64 && pmax == 2) return launch_l<64, 2, false, AUG>(a, ns, lds, st);
  if (nt == 64 && pmax == 8) return launch_l<64, 8, false, AUG>(a, ns, lds, st);
  if (nt == 256 && pmax == 4) return launch_l<256, 4, false, AUG>(a, ns, lds, st);
  if (nt == 256 && pmax == 8) return launch_l<256, 8, false, AUG>(a, ns, lds, st);
  if (nt == 1024 && pmax == 4) return launch_l<1024, 4, false, AUG>(a, ns, lds, st);
  return hipErrorInvalidValue;
}

hipError_t launch_krylov_lds(const KBlock* blocks, int n_blocks, int ns, int nt, int pmax,
                             bool vlds, size_t lds, const double* x_in, double* x_out,
                             const double* coef, double* vwork, double* diag, int* status,
                             double* calib, int mode, bool aug, hipStream_t st) {
  KrylovArgs a{blocks, x_in, x_out, coef, vwork, diag, status, calib, mode, n_blocks};
  if (n_blocks == 0) return hipSuccess;
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  return aug ? launch_shape<true>(a, ns, nt, pmax, vlds, lds, st)
             : launch_shape<false>(a, ns, nt, pmax, vlds, lds, st);
}

}  // namespace lem
